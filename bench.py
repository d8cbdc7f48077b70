#!/usr/bin/env python3
"""Benchmark of FSAI-preconditioned CG (M^-1 = G G^T) on one MI355X.

Workload: 3D variable-coefficient Poisson, 7-point stencil on a 128^3 grid
(n = 2,097,152, nnz = 14,581,760), lognormal face coefficients (sigma = 1),
b ~ N(0, 1) (seed 0), G = FSAI on tril(A), solved in FP64 from x0 = 0 to
||b - A x|| <= 1e-8 ||b||. One step = one complete solve with A, G, b resident
in HBM (the preconditioner is built once, outside the timed region, as the
paper's T_construct).

Prints one JSON line: solves/s (value), time to tolerance, HBM GB/s per
iteration, the roofline of the dominant kernel (the A-kernel) from live
HIP-event timing, the measured copy ceiling, and the FP64 CPU oracle timed on
the host cores on a bounded sample of the same solve.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PCG time-to-1e-8 rel. residual; HBM GB/s per iter; batched solves/s + p99 latency"
HBM_PEAK_GBPS = 8000.0
N_SIDE = 128
TOL = 1e-8
MAXIT = 5000
KERNEL_SOURCES = ["paper_2510_27517_amd/csrc/kernels.hip", "paper_2510_27517_amd/csrc/kernels.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_iter_A_poisson3d_128_f64_traffic.md")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic():
    """HBM bytes per A-kernel launch from the committed counter summary, if it
    was taken on the current kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    m_sha = re.search(r"kernel_sources_sha:\s*([0-9a-f]+)", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_b or m_sha.group(1) != kernel_sha():
        return None
    return float(m_b.group(1))


def cpu_baseline(A, b, gpu_iters, budget_s):
    """The FP64 oracle (as it stands) on the host cores: a bounded number of
    iterations of the same solve, scaled to the GPU's iteration count."""
    import oracle

    threads = len(os.sched_getaffinity(0))
    G = oracle.fsai_g(A)
    t0 = time.perf_counter()
    oracle.pcg(A, G, b, tol=TOL, maxit=3, delta_form=1, threads=threads)
    t3 = time.perf_counter() - t0
    per = t3 / 3
    m = int(max(5, min(400, budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    r = oracle.pcg(A, G, b, tol=TOL, maxit=m, delta_form=1, threads=threads)
    el = time.perf_counter() - t0
    per_it = el / max(r.iters, 1)
    t_solve = per_it * gpu_iters
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{r.iters} FP64 oracle PCG iterations of the same 128^3 FSAI solve on {threads} host threads "
                      f"({el:.1f} s, {per_it * 1e3:.1f} ms/iteration), scaled to the GPU's {gpu_iters} iterations",
            "ms_per_iteration": per_it * 1e3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kernel-iters", type=int, default=60)
    ap.add_argument("--cpu-budget-s", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-probe", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build runs single-GPU solves only (independent systems would "
              "shard by request across GPUs, a single system by row slabs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2510_27517_amd import inputs, pcg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    log("generating 128^3 system")
    A = inputs.poisson(3, N_SIDE, 1.0, 0)
    b = inputs.rhs(A.n, 0)
    solver = pcg.Solver(pcg.default_config(device=0))
    solver.set_matrix(A)
    t0 = time.perf_counter()
    solver.build_precond(pcg.G_FSAI)
    t_construct = time.perf_counter() - t0
    b_dev = torch.from_numpy(b).to(dev)
    torch.cuda.synchronize()

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        out = solver.solve(b_dev, tol=TOL, maxit=MAXIT)
    torch.cuda.synchronize()
    log(f"timing {args.steps} solves")
    results = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        results.append(solver.solve(b_dev, tol=TOL, maxit=MAXIT))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    last = results[-1]
    assert all(r.status == pcg.OK for r in results), [r.status for r in results]
    ms_per_step = elapsed * 1e3 / args.steps
    iters = last.iters
    bpi = last.bytes_per_iter
    gbps_iter = bpi / (ms_per_step * 1e-3 / iters) / 1e9

    log("kernel timing")
    kt = solver.time_kernels(args.kernel_iters)
    ms_a, bytes_a = kt["ms"][0], kt["bytes"][0]
    achieved = bytes_a / (ms_a * 1e-3) / 1e9
    traffic = stored_traffic()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": "k_iter_A (q = A d fused with the d and x updates and d^T q)",
                "bytes_per_launch": bytes_a, "avg_launch_ms": ms_a}
    kernels = {name: {"avg_ms": kt["ms"][k], "alg_bytes": kt["bytes"][k],
                      "gbps": kt["bytes"][k] / (kt["ms"][k] * 1e-3) / 1e9}
               for k, name in enumerate(["k_iter_A", "k_iter_GT", "k_iter_G"])}
    copy = None
    if not args.no_copy_probe:
        log("copy probe")
        gb, ms = pcg.copy_bandwidth(4 << 30, reps=10)
        copy = {"gbps": round(gb, 1), "bytes": 4 << 30, "ms_per_copy": ms}

    relres = last.relres_true  # ||b - A x|| / ||b|| from the library's FP64 residual kernel
    solver.close()
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(A, b, iters, args.cpu_budget_s)

    line = {
        "metric": METRIC, "value": round(1e3 / ms_per_step, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "poisson3d_7pt_128^3_lognormal_sigma1_fsai_f64_tol1e-8", "n": A.n, "nnz_a": A.nnz,
                   "nnz_g": (A.nnz + A.n) // 2, "tol": TOL, "x0": "zeros", "rr_period": 50},
        "time_to_tol_ms": round(ms_per_step, 3), "iters": iters, "ms_per_iter": round(ms_per_step / iters, 5),
        "hbm_gbps_per_iter": round(gbps_iter, 1), "alg_bytes_per_iter": bpi,
        "relres_true_fp64": relres, "t_construct_s": round(t_construct, 3),
        "roofline": roofline, "kernels": kernels, "copy_probe": copy, "cpu_baseline": cpu,
        "kernel_sources_sha": kernel_sha(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
