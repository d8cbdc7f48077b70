#!/usr/bin/env python3
"""Benchmark of FSAI-preconditioned CG (M^-1 = G G^T) on one MI355X.

Headline workload (the JSON line's `value`): 3D variable-coefficient Poisson,
7-point stencil on a 128^3 grid (n = 2,097,152, nnz = 14,581,760), lognormal
face coefficients (sigma = 1), b ~ N(0, 1) (seed 0), G = FSAI on tril(A),
solved in FP64 from x0 = 0 to ||b - A x|| <= 1e-8 ||b||. One step = one
complete solve with A, G, b resident in HBM (the preconditioner is built
once, outside the timed region, as the paper's T_construct; reported for the
host builder and for the device builder).

Further sections, each under its own key of the same JSON line:
  mixed      the same system in FP32 (A, vectors) with BF16 G and FP64
             iterative refinement to 1e-8, against the FP64 time to tolerance;
  batched    512 2D/3D lognormal Poisson systems of uneven size solved as one
             batch (FP32, FP64 refinement, tol 1e-6): solves/s, latency;
  serving    random-geometric-graph Laplacian requests arriving as a Poisson
             stream at 0.5, 0.8 and 0.95 of the measured closed-loop rate:
             p50/p99 latency, queue depth and admitted bytes;
  sai_loss   the SAI/L2/cosine preconditioner losses (Sec. 3.3) over 32
             Gaussian probes on the 128^3 system;
  synthetic  the paper's synthetic P P^T + 1e-4 I systems (n 18000 and 72000,
             and a batch of 64 with n in [12000, 24000]);
  elasticity Q1 elasticity, 64^3 free nodes x 3 dof (n = 786,432, 61.7M
             nonzeros): BF16/FP16 G with FP64 refinement to 1e-10 against the
             plain FP64 solve.
The oracle leg (cpu_baseline) times the FP64 CPU oracle on the host cores on
the headline solve, checks the GPU solve against it at full size (the oracle's
FSAI G handed to the library: both trajectories bit for bit), and states every
result's error against an oracle solution converged to 1e-12: the headline,
the mixed-precision solves, the elasticity solves, and samples of the batched
and served systems.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import threading
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
PROFILES = os.path.join(ROOT, "profiles")
SECTIONS = ["mixed", "sai_loss", "autotune", "small", "batched", "serving", "elasticity", "synthetic"]
# long runs, only when named: the serving workload at its configured length
OPTIONAL_SECTIONS = ["serving_stream"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` on the headline system from the
    committed counter summary, if it was taken on the current kernel sources."""
    path = os.path.join(PROFILES, f"{kernel}_poisson3d_128_f64_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"kernel_sources_sha:\s*([0-9a-f]+)", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_b or m_sha.group(1) != kernel_sha():
        return None
    return float(m_b.group(1))


def algorithmic_bytes(n, a, g, sa, sg, sv, eps=False):
    """Algorithmic bytes per launch of the three iteration kernels over int32
    CSR (4-byte column indices and row pointers): A-kernel a(sa + 4) + 4(n+1)
    + 2 n sv (reads d, writes q); G^T-kernel g(sg + 4) + 4(n+1) + 4 n sv
    (reads r and q, writes r and t); G-kernel g(sg + 4) + 4(n+1) + 5 n sv
    (reads t, d, x, writes d, x; one more with eps). Their sum is one
    iteration with 11 vector streams."""
    rp = 4.0 * (n + 1)
    k = [a * (sa + 4) + rp + 2 * n * sv, g * (sg + 4) + rp + 4 * n * sv, g * (sg + 4) + rp + (6 if eps else 5) * n * sv]
    return k + [sum(k)]


def pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else None


def _err(x, ref):
    return float(np.linalg.norm(np.asarray(x) - ref) / np.linalg.norm(ref))


def oracle_leg(pcg, torch, A, b, gpu, budget_s, extra_refs):
    """The FP64 oracle as it stands, on the host cores:
    - timing (the `cpu_baseline` figures): the headline solve with the oracle's
      own FSAI G, as many iterations as the budget allows (all, normally),
      scaled to the GPU's iteration count;
    - parity at full size: the library solves the same system with the
      oracle's G (its own FSAI agrees with the oracle's to 1e-13 row-normwise
      only); with exact inner products on both sides the trajectories must be
      identical: status, iterations and x bit for bit;
    - accuracy: every result's error against an oracle solution converged to
      1e-12 (the headline and mixed solves, elasticity, and samples of the
      batched and served systems, each against its own reference).
    The oracle's results do not depend on its thread count."""
    import oracle

    threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    G = oracle.fsai_g(A)
    t_fsai = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.pcg(A, G, b, tol=TOL, maxit=3, delta_form=1, threads=threads)
    per = (time.perf_counter() - t0) / 3
    m = int(max(5, min(MAXIT, budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    r = oracle.pcg(A, G, b, tol=TOL, maxit=m, delta_form=1, threads=threads)
    el = time.perf_counter() - t0
    per_it = el / max(r.iters, 1)
    gpu_iters = gpu["iters"]
    out = {"value": 1.0 / (per_it * gpu_iters), "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": f"{r.iters} FP64 oracle PCG iterations of the same 128^3 FSAI solve (oracle FSAI G) on "
                     f"{threads} host threads ({el:.1f} s, {per_it * 1e3:.1f} ms/iteration), scaled to the GPU's "
                     f"{gpu_iters} iterations",
           "ms_per_iteration": per_it * 1e3, "oracle_iters": r.iters, "oracle_status": r.status,
           "oracle_fsai_s": round(t_fsai, 2)}
    # full-size parity: the library on the oracle's G, the launch configuration timed above
    if r.status == oracle.OK:
        with pcg.Solver(pcg.default_config()) as s:
            s.set_matrix(A)
            s.set_precond(rowptr=G.rowptr, col=G.col, val=G.val)
            got = s.solve(torch.from_numpy(b).to("cuda:0"), tol=TOL, maxit=MAXIT)
        xg = got.x.cpu().numpy()
        out["parity_full_size"] = {
            "workload": "the headline system solved by the library with the oracle's FSAI G",
            "gpu_iters": got.iters, "oracle_iters": r.iters, "gpu_status": got.status,
            "x_bitwise_equal": bool(np.array_equal(xg, r.x)), "rel_diff_x": _err(xg, r.x),
            "max_abs_diff_x": float(np.max(np.abs(xg - r.x)))}
    # accuracy against solutions converged to 1e-12
    ref = oracle.pcg(A, G, b, tol=1e-12, maxit=4 * MAXIT, delta_form=1, threads=threads)
    acc = {"reference": f"oracle FSAI PCG to 1e-12 ({ref.iters} iterations, status {ref.status})"}
    for k, x in gpu["solutions"].items():
        acc[k] = _err(x, ref.x)
    for name, items in extra_refs.items():
        got = {}
        for tag, (Ak, bk, xs) in items.items():
            t1 = time.perf_counter()
            Gk = oracle.fsai_g(Ak)
            rk = oracle.pcg(Ak, Gk, bk, tol=1e-12, maxit=50000, delta_form=1, threads=threads)
            e = {"n": Ak.n, "oracle_iters": rk.iters, "oracle_status": rk.status,
                 "oracle_s": round(time.perf_counter() - t1, 1)}
            for sol, xk in xs.items():
                e[sol] = _err(xk, rk.x)
            got[tag] = e
        acc[name] = got
    out["error_vs_oracle_1e-12"] = acc
    return out


# ---------------------------------------------------------------- sections

def _timed_solves(pcg, torch, cfg, A, G, b_dev, steps, tol=TOL):
    with pcg.Solver(cfg) as s:
        s.set_matrix(A)
        s.set_precond(rowptr=G[0], col=G[1], val=G[2])
        s.solve(b_dev, tol=tol, maxit=MAXIT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = s.solve(b_dev, tol=tol, maxit=MAXIT)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps, r


def section_mixed(pcg, torch, A, G, b_dev, steps, t_fp64_ms):
    """128^3 in FP32 (A, vectors) with BF16 G and FP64 refinement to 1e-8; and
    FP64 vectors and A with the BF16 G (FP64 PCG, 16-bit preconditioner)."""
    cfg = pcg.default_config(vec_dtype="f32", a_dtype="f32", g_dtype="bf16", refine=1)
    ms, r = _timed_solves(pcg, torch, cfg, A, G, b_dev, steps)
    ms64, r64 = _timed_solves(pcg, torch, pcg.default_config(g_dtype="bf16"), A, G, b_dev, steps)
    cfg32 = pcg.default_config(vec_dtype="f32", a_dtype="f32", g_dtype="f32")
    ms32, r32 = _timed_solves(pcg, torch, cfg32, A, G, b_dev, steps, tol=1e-6)
    return {"workload": "poisson3d_128^3_sigma1_fsai, A/vectors f32, G bf16, FP64 refinement to 1e-8",
            "time_to_tol_ms": round(ms, 3), "speedup_vs_fp64": round(t_fp64_ms / ms, 3), "status": r.status,
            "inner_iters": r.iters, "outer_iters": r.outer_iters, "relres_true_fp64": r.relres_true,
            "alg_bytes_per_inner_iter": r.bytes_per_iter,
            "fp64_bf16_g": {"workload": "same system, A/vectors f64, G bf16 (no refinement), tol 1e-8",
                            "time_to_tol_ms": round(ms64, 3), "speedup_vs_fp64": round(t_fp64_ms / ms64, 3),
                            "status": r64.status, "iters": r64.iters, "relres_true_fp64": r64.relres_true,
                            "ms_per_iter": round(ms64 / max(r64.iters, 1), 5),
                            "alg_bytes_per_iter": r64.bytes_per_iter},
            "fp32_plain": {"workload": "same system, A/vectors/G f32, no refinement, tol 1e-6 (plain FP32 cannot "
                                       "certify 1e-8)",
                           "time_to_tol_ms": round(ms32, 3), "status": r32.status, "iters": r32.iters,
                           "relres_true_fp32": r32.relres_true, "ms_per_iter": round(ms32 / max(r32.iters, 1), 5),
                           "alg_bytes_per_iter": r32.bytes_per_iter}}, r.x.cpu().numpy()


def section_autotune(pcg, torch, inputs, A, G, b_dev, steps, t_auto_ms):
    """The autotuner on the 128^3 FP64 system: layouts and grid it keeps, the
    time it took, and timed solves with its choice; and the same on a
    launch-bound 2D system of 32761 rows."""
    with pcg.Solver(pcg.default_config()) as s:
        s.set_matrix(A)
        s.set_precond(rowptr=G[0], col=G[1], val=G[2])
        t0 = time.perf_counter()
        t = s.autotune(20)
        t_tune = time.perf_counter() - t0
        s.solve(b_dev, tol=TOL, maxit=MAXIT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = s.solve(b_dev, tol=TOL, maxit=MAXIT)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
    names = {v: k for k, v in pcg.LAYOUTS.items()}
    out = {"workload": "poisson3d_128^3_sigma1_fsai, FP64, tol 1e-8", "tune_s": round(t_tune, 2),
           "candidates": t["candidates"], "layout_a": names.get(t["layout_a"]), "layout_g": names.get(t["layout_g"]),
           "grid_mult": t["grid_mult"], "temporal": t["temporal"], "rows_per_lane_gt": t["rows_per_lane_gt"],
           "loads_in_flight_a": t["loads_in_flight_a"], "ms_per_iter_tuned": round(t["ms_per_iter"], 5),
           "ms_per_iter_auto": round(t["ms_per_iter_auto"], 5), "time_to_tol_ms": round(ms, 3),
           "time_to_tol_ms_auto": round(t_auto_ms, 3), "iters": r.iters, "status": r.status}
    # a launch-bound size, where fewer rows per lane (more busy waves) or
    # fewer loads in flight can pay
    As = inputs.poisson(2, 181, 1.0, 181)
    bs = torch.from_numpy(inputs.rhs(As.n, 181)).to("cuda:0")
    times = {}
    for tag, tune in (("auto", False), ("tuned", True)):
        with pcg.Solver(pcg.default_config(wg_max_n=-1)) as s:
            s.set_matrix(As)
            s.build_precond(pcg.G_FSAI)
            if tune:
                t0 = time.perf_counter()
                ts = s.autotune(20)
                t_tune_s = time.perf_counter() - t0
            s.solve(bs, tol=TOL, maxit=MAXIT)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(10):
                rs = s.solve(bs, tol=TOL, maxit=MAXIT)
            torch.cuda.synchronize()
            times[tag] = (time.perf_counter() - t0) * 1e3 / 10
    out["small"] = {"workload": "poisson2d_181^2_sigma1_fsai (32761 rows), FP64, tol 1e-8", "tune_s": round(t_tune_s, 2),
                    "candidates": ts["candidates"], "layout_a": names.get(ts["layout_a"]),
                    "layout_g": names.get(ts["layout_g"]), "grid_mult": ts["grid_mult"], "temporal": ts["temporal"],
                    "rows_per_lane_gt": ts["rows_per_lane_gt"], "loads_in_flight_a": ts["loads_in_flight_a"],
                    "ms_per_iter_tuned": round(ts["ms_per_iter"], 5), "ms_per_iter_auto": round(ts["ms_per_iter_auto"], 5),
                    "time_to_tol_ms": round(times["tuned"], 3), "time_to_tol_ms_auto": round(times["auto"], 3),
                    "iters": rs.iters, "status": rs.status}
    return out


def section_sai_loss(pcg, inputs, A, G, k, reps=3):
    """The SAI/L2/cosine losses of Sec. 3.3 for k Gaussian probes on the 128^3
    system with its FSAI G (three multi-probe products and the sums)."""
    import torch

    W = torch.from_numpy(inputs.normal(0, inputs.STREAM_PROBE, A.n * k).reshape(A.n, k)).to("cuda:0")
    with pcg.Solver(pcg.default_config()) as s:
        s.set_matrix(A)
        s.set_precond(rowptr=G[0], col=G[1], val=G[2])
        out = s.sai_loss(W)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = s.sai_loss(W)
        ms = (time.perf_counter() - t0) * 1e3 / reps
    # each product streams its matrix once and two n x k probe blocks
    mat = A.nnz * 12 + 2 * int(G[1].shape[0]) * 12 + 3 * 4 * (A.n + 1)
    vec = (2 + 2 + 3 + 2) * A.n * k * 8
    return {"workload": f"SAI, L2 and cosine losses, 128^3 FSAI, {k} N(0,1) probes (FP64)", "probes": k,
            "ms_per_call": round(ms, 3), "probes_per_s": round(k / (ms * 1e-3), 1),
            "alg_gbps": round((mat + vec) / (ms * 1e-3) / 1e9, 1), "sai_mean": float(np.mean(out["sai"])),
            "l2_mean": float(np.mean(out["l2"])), "cs_mean": float(np.mean(out["cs"])),
            "note": "probes resident on the device; scratch kept by the context after the first call"}


def section_synthetic(pcg, inputs, count):
    """The paper's synthetic set (Sec. 4.1, App. C): A = P P^T + 1e-4 I, P of
    density 3e-4, n uniform in [12000, 24000] (and one Synthetic-Large system,
    n = 72000), FSAI, FP64, tol 1e-8: the small, latency-bound regime."""
    out = {"workload": "synthetic P P^T + 1e-4 I (P density 3e-4), FSAI G, FP64, tol 1e-8"}
    for tag, n in (("n18000", 18000), ("large_n72000", 72000)):
        A = inputs.synthetic_ppt(n, 7)
        b = inputs.rhs(A.n, 7)
        with pcg.Solver(pcg.default_config()) as s:
            s.set_matrix(A)
            s.build_precond(pcg.G_FSAI)
            s.solve(b, tol=1e-8, maxit=20000)
            t0 = time.perf_counter()
            r = s.solve(b, tol=1e-8, maxit=20000)
            ms = (time.perf_counter() - t0) * 1e3
        out[tag] = {"n": A.n, "nnz": A.nnz, "time_to_tol_ms": round(ms, 2), "iters": r.iters, "status": r.status,
                    "us_per_iter": round(ms * 1e3 / max(r.iters, 1), 2), "relres_true_fp64": r.relres_true}
        with pcg.Solver(pcg.default_config()) as s:  # the same solve with the autotuner's choice
            s.set_matrix(A)
            s.build_precond(pcg.G_FSAI)
            t = s.autotune(20)
            s.solve(b, tol=1e-8, maxit=20000)
            t0 = time.perf_counter()
            r = s.solve(b, tol=1e-8, maxit=20000)
            ms = (time.perf_counter() - t0) * 1e3
        names = {v: k for k, v in pcg.LAYOUTS.items()}
        out[tag]["autotuned"] = {"time_to_tol_ms": round(ms, 2), "iters": r.iters, "status": r.status,
                                 "layout_a": names.get(t["layout_a"]), "layout_g": names.get(t["layout_g"]),
                                 "grid_mult": t["grid_mult"], "temporal": t["temporal"],
                                 "rows_per_lane_gt": t["rows_per_lane_gt"],
                                 "loads_in_flight_a": t["loads_in_flight_a"],
                                 "ms_per_iter_tuned": round(t["ms_per_iter"], 5),
                                 "ms_per_iter_auto": round(t["ms_per_iter_auto"], 5)}
    log(f"synthetic: batch of {count}")
    u = inputs.u01(11, inputs.STREAM_SIZES, count)
    systems = []
    for i in range(count):
        A = inputs.synthetic_ppt(12000 + min(12000, int(u[i] * 12001)), 100 + i)
        systems.append(dict(A=A, b=inputs.rhs(A.n, 100 + i), tol=1e-8, maxit=20000))
    with pcg.Solver(pcg.default_config()) as s:
        t0 = time.perf_counter()
        res = s.solve_batch(systems, iters_per_step=50)
        wall = time.perf_counter() - t0
    st = [r["status"] for _, r in res]
    out["batch"] = {"systems": count, "solves_per_s": round(count / wall, 2), "wall_s": round(wall, 3),
                    "ok": st.count(pcg.OK), "iters_max": max(r["iters"] for _, r in res),
                    "iters_median": float(np.median([r["iters"] for _, r in res])),
                    "note": "n uniform in [12000, 24000]; wall time includes host FSAI and uploads"}
    return out


def section_small(pcg, inputs):
    """Small systems, where launches and not bytes bound the iteration: 2D
    lognormal (sigma 1) Poisson with FSAI, FP64, tol 1e-8, solved with the
    three-kernel iteration and with the one-workgroup solver (the whole solve
    in one launch), microseconds per iteration; and the three-kernel floor on
    a tiny system (kernels with almost no work)."""
    out = {"workload": "2D lognormal Poisson (sigma 1), FSAI G, FP64, tol 1e-8: three kernels per iteration "
                       "against one persistent workgroup per solve", "sizes": {}}
    for N in (8, 16, 32, 45, 64, 91, 128, 181):
        A = inputs.poisson(2, N, 1.0, N)
        b = inputs.rhs(A.n, N)
        row = {"n": A.n}
        for tag, wg in (("three_kernels", -1), ("one_workgroup", 1 << 30)):
            with pcg.Solver(pcg.default_config(wg_max_n=wg)) as s:
                s.set_matrix(A)
                s.build_precond(pcg.G_FSAI)
                s.solve(b, tol=1e-8, maxit=20000)
                reps = 5
                t0 = time.perf_counter()
                for _ in range(reps):
                    r = s.solve(b, tol=1e-8, maxit=20000)
                ms = (time.perf_counter() - t0) * 1e3 / reps
            row[tag] = {"time_to_tol_ms": round(ms, 3), "iters": r.iters, "status": r.status,
                        "us_per_iter": round(ms * 1e3 / max(r.iters, 1), 2)}
        out["sizes"][f"{N}^2"] = row
    return out


def batch_systems(inputs, count):
    """2D (side U{16..256}) or 3D (side U{8..64}) lognormal (sigma 0.5) Poisson
    with probability 1/2 each, b ~ N(0,1); system i uses seed i."""
    kind = inputs.u01(0, inputs.STREAM_KIND, count)
    size = inputs.u01(0, inputs.STREAM_SIZES, count)
    out = []
    for i in range(count):
        if kind[i] < 0.5:
            N = 16 + min(240, int(size[i] * 241))
            A = inputs.poisson(2, N, 0.5, i)
        else:
            N = 8 + min(56, int(size[i] * 57))
            A = inputs.poisson(3, N, 0.5, i)
        out.append(dict(A=A, b=inputs.rhs(A.n, i), tol=1e-6, maxit=10000))
    return out


def section_batched(pcg, inputs, count):
    log(f"batched: generating {count} systems")
    systems = batch_systems(inputs, count)
    n_tot = sum(s["A"].n for s in systems)
    nnz_tot = sum(s["A"].nnz for s in systems)
    cfg = pcg.default_config(vec_dtype="f32", a_dtype="f32", g_dtype="f32", refine=1)
    log(f"batched: solving {count} systems, {n_tot} rows")
    with pcg.Solver(cfg) as s:
        t0 = time.perf_counter()
        res = s.solve_batch(systems, iters_per_step=10)
        wall = time.perf_counter() - t0
        gs = s.batch_stats()
    # the same batch with every G built beforehand (the host FSAI outside the
    # clock): what remains on the host is layout, staging and scheduling
    log("batched: G built beforehand")
    pre = [dict(sd, G=inputs.CSR(*pcg.build_g_host(pcg.G_FSAI, sd["A"]))) for sd in systems]
    with pcg.Solver(cfg) as s:
        t0 = time.perf_counter()
        rpre = s.solve_batch(pre, iters_per_step=10)
        wall_pre = time.perf_counter() - t0
        gs_pre = s.batch_stats()
    gpu = {"iteration_steps": gs["steps"], "step_device_ms": round(gs["step_ms"], 2),
           "step_bytes": gs["step_bytes"],
           "aggregate_gbps_over_active_set": round(gs["step_bytes"] / (gs["step_ms"] * 1e-3) / 1e9, 1)
           if gs["step_ms"] > 0 else None,
           "one_workgroup_launches": gs["wg_launches"], "one_workgroup_device_ms": round(gs["wg_ms"], 2),
           "one_workgroup_bytes": gs["wg_bytes"],
           "gpu_only_solves_per_s": round(count / ((gs["step_ms"]) * 1e-3), 1) if gs["step_ms"] > 0 else None,
           "host_ms": {k: round(gs["host_" + k + "_ms"], 1) for k in ("prep", "admit", "step", "retire", "progress", "idle")},
           "g_prebuilt": {"wall_s": round(wall_pre, 3), "solves_per_s": round(count / wall_pre, 2),
                          "ok": sum(1 for _, r in rpre if r["status"] == pcg.OK),
                          "step_device_ms": round(gs_pre["step_ms"], 2),
                          "bitwise_equal_to_host_fsai_run": bool(all(np.array_equal(a[0], c[0])
                                                                     for a, c in zip(res, rpre)))},
           "note": "device time of the scheduler's iteration steps (events around each step's launches on the "
                   "library stream; refinement's FP64 steps, uploads and readbacks outside), bytes = per system "
                   "iterations run x bytes_per_iter of its stored layouts; one-workgroup launches of small "
                   "systems run on a second stream beside the steps. gpu_only_solves_per_s = systems / step "
                   "device time"}
    st = [r["status"] for _, r in res]
    lat = [r["t_latency_ms"] for _, r in res]
    solve = [r["t_solve_ms"] for _, r in res]
    # plain FP64 (no refinement): small systems solved whole by one
    # persistent workgroup each, and the same batch without
    plain = {}
    for tag, wgb in (("one_workgroup_small", 0), ("three_kernels_only", -1)):
        cfgp = pcg.default_config(wg_max_n_batch=wgb)
        log(f"batched: plain FP64, {tag}")
        with pcg.Solver(cfgp) as s:
            t0 = time.perf_counter()
            rp = s.solve_batch(systems, iters_per_step=10)
            wp = time.perf_counter() - t0
        plain[tag] = {"solves_per_s": round(count / wp, 2), "wall_s": round(wp, 3),
                      "ok": sum(1 for _, r in rp if r["status"] == pcg.OK),
                      "latency_ms_p50": pct([r["t_latency_ms"] for _, r in rp], 50),
                      "latency_ms_p99": pct([r["t_latency_ms"] for _, r in rp], 99),
                      "max_relres_true_fp64": max(r["relres_true"] for _, r in rp)}
    plain["small_systems"] = int(sum(1 for sd in systems if sd["A"].n <= 16384))
    order = np.argsort([sd["A"].n for sd in systems])
    samples = {f"system{int(i)}": (systems[i]["A"], systems[i]["b"], {"x": res[i][0]})
               for i in order[np.linspace(0, count - 1, min(6, count)).astype(int)]}
    return {"workload": f"{count} systems: 2D side U[16,256] / 3D side U[8,64] lognormal sigma 0.5 Poisson, "
                        "FSAI G built on the host, A/vectors/G f32, FP64 refinement, tol 1e-6",
            "fp64_plain": plain, "gpu": gpu,
            "systems": count, "rows_total": n_tot, "nnz_total": nnz_tot,
            "solves_per_s": round(count / wall, 2), "wall_s": round(wall, 3),
            "ok": st.count(pcg.OK), "statuses": sorted(set(st)),
            "latency_ms_p50": pct(lat, 50), "latency_ms_p99": pct(lat, 99),
            "solve_ms_p50": pct(solve, 50), "solve_ms_p99": pct(solve, 99),
            "max_relres_true_fp64": max(r["relres_true"] for _, r in res),
            "inner_iters_max": max(r["iters"] for _, r in res),
            "note": "wall time from submission to the last completion, including host FSAI construction and "
                    "uploads"}, samples


def serving_requests(inputs, count):
    """RGG Laplacian + 1e-3 I, n log-uniform in [1e3, 1e6]."""
    u = inputs.u01(7, inputs.STREAM_SIZES, count)
    out = []
    for i in range(count):
        n = int(round(10 ** (3 + 3 * u[i])))
        A = inputs.rgg_laplacian(n, 10_000 + i)
        out.append(dict(A=A, b=inputs.rhs(A.n, 10_000 + i), tol=1e-6, maxit=20000))
    return out


def _serve(pcg, cfg, make_req, count, arrive, window, iters_per_step):
    """Serve `count` requests made on demand by make_req(i): submitted by a
    thread of their own at their arrival times (open loop), or, with arrive
    None, whenever fewer than `window` are in flight (closed loop), while
    this thread drives the scheduler and collects finished tickets. Only
    statistics are kept: each solution is dropped when its ticket completes.
    Latency runs from arrival (or, in the closed loop, submission) to
    completion."""
    lat, st, qms, sms, depth, used = [], [], [], [], [], []
    rel = [0.0]
    lock = threading.Lock()
    outstanding = {}  # ticket -> submission lag behind the arrival (ms)
    with pcg.Solver(cfg) as s:
        t0 = time.perf_counter()

        def submitter():
            nxt = 0
            while nxt < count:
                now = time.perf_counter() - t0
                if arrive is None:
                    with lock:
                        room = window - len(outstanding)
                    if room <= 0:
                        time.sleep(0.0005)
                        continue
                    batch = list(range(nxt, min(count, nxt + room)))
                else:
                    if arrive[nxt] > now:
                        time.sleep(min(0.005, arrive[nxt] - now))
                        continue
                    batch = []
                    while nxt + len(batch) < count and arrive[nxt + len(batch)] <= now:
                        batch.append(nxt + len(batch))
                nxt += len(batch)
                tk = s.submit([make_req(i) for i in batch])
                with lock:
                    for i, t in zip(batch, tk):
                        outstanding[t] = 0.0 if arrive is None else (now - arrive[i]) * 1e3

        th = threading.Thread(target=submitter, daemon=True)
        th.start()
        done, last_log = 0, t0
        while done < count:
            with lock:
                waiting = len(outstanding)
            if waiting == 0:
                time.sleep(0.0005)
                continue
            a, q = s.progress(iters_per_step)
            depth.append(a + q)
            used.append(s.pool_info()[1])
            if a + q < waiting:  # some ticket completed and waits to be collected
                with lock:
                    tks = list(outstanding)
                for t in tks:
                    r = s.poll(t)
                    if r is not None:
                        res = r[1]
                        with lock:
                            lag = outstanding.pop(t)
                        lat.append(res["t_latency_ms"] + lag)
                        st.append(res["status"])
                        rel[0] = max(rel[0], res["relres_true"])
                        qms.append(res["t_queue_ms"])
                        sms.append(res["t_solve_ms"])
                        done += 1
            if time.perf_counter() - last_log > 30:
                last_log = time.perf_counter()
                log(f"serving: {done}/{count} done, {waiting} in flight")
        span = time.perf_counter() - t0
        th.join()
        gs = s.batch_stats()
    return dict(lat=lat, st=st, span=span, depth=depth, used=used, rel=rel[0], qms=qms, sms=sms, gs=gs)


def section_serving_stream(pcg, inputs, count, pool, window, iters_per_step, loads, mu_given=0.0):
    """The serving workload at its configured length: `count` requests whose
    matrices come from a pool of `pool` generated RGG Laplacians (sizes
    log-uniform in [1e3, 1e6], the serving recipe), request i taking pool
    matrix i mod pool with a right-hand side of its own, generated at
    submission. A closed loop with `window` requests in flight gives the
    sustainable rate mu (or mu_given, from an earlier run); then Poisson
    arrivals at the given fractions of mu."""
    log(f"serving stream: generating {pool} pool matrices")
    mats = [r["A"] for r in serving_requests(inputs, pool)]

    def make_req(i):
        A = mats[i % pool]
        return dict(A=A, b=inputs.rhs(A.n, 30_000 + i), tol=1e-6, maxit=20000)

    cfg = pcg.default_config(vec_dtype="f32", a_dtype="f32", g_dtype="bf16", refine=1)
    ns = [mats[i % pool].n for i in range(count)]
    out = {"workload": f"{count} RGG Laplacian + 1e-3 I requests from a pool of {pool} matrices (n log-uniform "
                       f"[1e3,1e6], mean over the stream {np.mean(ns):.0f}), right-hand side per request; f32 "
                       "A/vectors, bf16 FSAI G, FP64 refinement, tol 1e-6",
           "requests": count, "pool_matrices": pool, "closed_loop_window": window, "loads": {}}

    def summary(r):
        gs = r["gs"]
        return {"solves_per_s": round(count / r["span"], 2), "span_s": round(r["span"], 1),
                "latency_ms_p50": pct(r["lat"], 50), "latency_ms_p99": pct(r["lat"], 99),
                "latency_ms_p999": pct(r["lat"], 99.9), "ok": r["st"].count(pcg.OK),
                "max_relres_true_fp64": r["rel"], "queue_ms_p50": pct(r["qms"], 50),
                "solve_ms_p50": pct(r["sms"], 50),
                "queue_depth_mean": float(np.mean(r["depth"])) if r["depth"] else 0.0,
                "queue_depth_max": int(max(r["depth"])) if r["depth"] else 0,
                "admitted_mb_max": float(max(r["used"])) / 2**20 if r["used"] else 0.0,
                "gpu_busy_fraction_iteration_steps": round(gs["step_ms"] / (r["span"] * 1e3), 3),
                "host_ms": {k: round(gs["host_" + k + "_ms"], 1) for k in ("prep", "admit", "step", "retire", "progress", "idle")}}

    if mu_given > 0:
        mu = mu_given
        out["closed_loop_solves_per_s"] = mu
        out["closed_loop"] = "rate given (measured in an earlier run of this section)"
    else:
        log(f"serving stream: closed loop, {count} requests, {window} in flight")
        closed = _serve(pcg, cfg, make_req, count, None, window, iters_per_step)
        mu = count / closed["span"]
        out["closed_loop"] = summary(closed)
        out["closed_loop_solves_per_s"] = round(mu, 2)
    gaps01 = -np.log(inputs.u01(7, inputs.STREAM_ARRIVALS, count))
    for f in loads:
        lam = f * mu
        log(f"serving stream: open loop at {lam:.1f} requests/s ({f} mu)")
        r = _serve(pcg, cfg, make_req, count, np.cumsum(gaps01 / lam), window, iters_per_step)
        out["loads"][str(f)] = {"arrival_rate": round(lam, 2), **summary(r)}
    return out


def section_serving(pcg, inputs, count, iters_per_step):
    log(f"serving: generating {count} requests")
    reqs = serving_requests(inputs, count)
    cfg = pcg.default_config(vec_dtype="f32", a_dtype="f32", g_dtype="bf16", refine=1)
    # closed loop: everything at once gives the sustainable rate mu
    with pcg.Solver(cfg) as s:
        t0 = time.perf_counter()
        res = s.solve_batch(reqs, iters_per_step=iters_per_step)
        wall = time.perf_counter() - t0
        gs = s.batch_stats()
    mu = count / wall
    ns = [r["A"].n for r in reqs]
    order = np.argsort(ns)
    samples = {f"request{int(i)}": (reqs[i]["A"], reqs[i]["b"], {"x": res[i][0]})
               for i in order[(np.array([0.1, 0.3, 0.5, 0.7, 0.9]) * (count - 1)).astype(int)]}
    out = {"workload": f"{count} RGG Laplacian + 1e-3 I requests, n log-uniform [1e3,1e6] (mean {np.mean(ns):.0f}), "
                       "mean degree ~8, weights U[0.1,10]; f32 A/vectors, bf16 FSAI G, FP64 refinement, tol 1e-6; "
                       "Poisson arrivals at 0.5/0.8/0.95 of the closed-loop rate",
           "requests": count, "closed_loop_solves_per_s": round(mu, 2),
           "closed_loop_latency_ms_p99": pct([r["t_latency_ms"] for _, r in res], 99),
           "closed_loop_gpu": {"step_device_ms": round(gs["step_ms"], 1), "wall_ms": round(wall * 1e3, 1),
                               "busy_fraction_iteration_steps": round(gs["step_ms"] / (wall * 1e3), 3),
                               "one_workgroup_device_ms": round(gs["wg_ms"], 1),
                               "host_ms": {k: round(gs["host_" + k + "_ms"], 1) for k in ("prep", "admit", "step", "retire", "progress", "idle")},
                               "aggregate_gbps_over_active_set": round(gs["step_bytes"] / (gs["step_ms"] * 1e-3) / 1e9,
                                                                       1) if gs["step_ms"] > 0 else None},
           "loads": {}}
    # open loop: Poisson arrivals (exponential gaps from the arrivals stream)
    gaps01 = -np.log(inputs.u01(7, inputs.STREAM_ARRIVALS, count))
    for f in (0.5, 0.8, 0.95):
        lam = f * mu
        log(f"serving: open loop at {lam:.1f} requests/s ({f} mu)")
        r = _serve(pcg, cfg, lambda i: reqs[i], count, np.cumsum(gaps01 / lam), 0, iters_per_step)
        depth, used = r["depth"], r["used"]
        out["loads"][str(f)] = {
            "arrival_rate": round(lam, 2), "solves_per_s": round(count / r["span"], 2),
            "latency_ms_p50": pct(r["lat"], 50), "latency_ms_p99": pct(r["lat"], 99), "ok": r["st"].count(pcg.OK),
            "max_relres_true_fp64": r["rel"], "queue_depth_mean": float(np.mean(depth)) if depth else 0.0,
            "queue_depth_max": int(max(depth)) if depth else 0,
            "admitted_mb_mean": float(np.mean(used)) / 2**20 if used else 0.0,
            "admitted_mb_max": float(max(used)) / 2**20 if used else 0.0,
            "queue_ms_p50": pct(r["qms"], 50), "solve_ms_p50": pct(r["sms"], 50),
            "note": "queue = submission to admission (host G construction, staging, waiting for memory); "
                    "solve = admission to completion; requests submitted by a thread of their own at their "
                    "arrival times"}
    main = out["loads"]["0.8"]
    out["latency_ms_p50"], out["latency_ms_p99"] = main["latency_ms_p50"], main["latency_ms_p99"]
    # the same requests with each FSAI factored on the device at admission
    # (g_device = 1): closed loop only
    log("serving: closed loop, FSAI on the device at admission")
    cfg_d = pcg.default_config(vec_dtype="f32", a_dtype="f32", g_dtype="bf16", refine=1, g_device=1)
    with pcg.Solver(cfg_d) as s:
        t0 = time.perf_counter()
        res_d = s.solve_batch(reqs, iters_per_step=iters_per_step)
        wall_d = time.perf_counter() - t0
    out["device_fsai_at_admission"] = {
        "closed_loop_solves_per_s": round(count / wall_d, 2),
        "ok": sum(1 for _, r in res_d if r["status"] == pcg.OK),
        "note": "the scheduler thread uploads A in FP64 CSR and factors each G at admission, serially; the "
                "host builder runs on worker threads alongside the GPU"}
    return out, samples


def section_elasticity(pcg, inputs, N):
    log(f"elasticity: generating {N}^3 x 3")
    A = inputs.elasticity(N, 1.0, 0.3, 0)
    b = inputs.rhs(A.n, 0)
    t0 = time.perf_counter()
    G = pcg.build_g_host(pcg.G_FSAI, A)
    t_fsai = time.perf_counter() - t0
    with pcg.Solver(pcg.default_config(g_device=1)) as s:
        s.set_matrix(A)
        t0 = time.perf_counter()
        s.build_precond(pcg.G_FSAI)
        t_dev = time.perf_counter() - t0
    t0 = time.perf_counter()
    GB = pcg.build_g_host(pcg.G_BFSAI, A)
    t_bfsai = time.perf_counter() - t0
    out = {"workload": f"Q1 elasticity {N}^3 free nodes x 3 dof, E lognormal sigma 1, nu 0.3, scalar FSAI G "
                       f"(and block FSAI, 3x3 blocks), tol 1e-10",
           "n": A.n, "nnz": A.nnz, "nnz_g_fsai": int(G[1].shape[0]), "nnz_g_block_fsai": int(GB[1].shape[0]),
           "t_construct_fsai_s": round(t_fsai, 2), "t_construct_fsai_device_s": round(t_dev, 3),
           "t_construct_block_fsai_s": round(t_bfsai, 2)}
    x64 = None
    xs = {}
    mixed = dict(vec_dtype="f32", a_dtype="f32", g_dtype="bf16", refine=1)
    for name, kw, GG in [("fp64", dict(), G), ("f32_bf16_refined", mixed, G),
                         ("f32_f16_refined", dict(vec_dtype="f32", a_dtype="f32", g_dtype="f16", refine=1), G),
                         ("fp64_block_fsai", dict(), GB), ("f32_bf16_refined_block_fsai", mixed, GB)]:
        log(f"elasticity: {name}")
        with pcg.Solver(pcg.default_config(**kw)) as s:
            s.set_matrix(A)
            s.set_precond(rowptr=GG[0], col=GG[1], val=GG[2])
            t0 = time.perf_counter()
            r = s.solve(b, tol=1e-10, maxit=20000)
            ms = (time.perf_counter() - t0) * 1e3
        d = {"time_to_tol_ms": round(ms, 2), "status": r.status, "iters": r.iters, "outer_iters": r.outer_iters,
             "relres_true_fp64": r.relres_true}
        xs[name] = r.x
        if x64 is None:
            x64 = r.x
            out["ms_per_iter_fp64"] = round(ms / max(r.iters, 1), 4)
        else:
            d["error_vs_fp64_gpu"] = float(np.linalg.norm(r.x - x64) / np.linalg.norm(x64))
        out[name] = d
    return out, {f"{N}^3x3": (A, b, xs)}


# ---------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kernel-iters", type=int, default=60)
    ap.add_argument("--cpu-budget-s", type=float, default=25.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--sections", default=",".join(SECTIONS), help="comma list of " + ",".join(SECTIONS) + " or none")
    ap.add_argument("--probes", type=int, default=32)
    ap.add_argument("--batch-systems", type=int, default=512)
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-step", type=int, default=10)
    ap.add_argument("--serve-pool", type=int, default=500, help="pool matrices of the serving_stream section")
    ap.add_argument("--serve-window", type=int, default=200, help="requests in flight in its closed loop")
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95", help="arrival rates of the serving_stream section, "
                    "as fractions of its closed-loop rate")
    ap.add_argument("--serve-mu", type=float, default=0.0, help="closed-loop rate of the serving_stream section "
                    "from an earlier run (0: measure it)")
    ap.add_argument("--elasticity-n", type=int, default=64)
    ap.add_argument("--synthetic-batch", type=int, default=64)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library runs each solve on one GPU (independent systems would "
              "shard by request across GPUs, a single system by row slabs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    sections = [x for x in args.sections.split(",") if x in SECTIONS + OPTIONAL_SECTIONS]

    import torch

    from paper_2510_27517_amd import inputs, pcg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    log("generating 128^3 system")
    A = inputs.poisson(3, N_SIDE, 1.0, 0)
    b = inputs.rhs(A.n, 0)
    t0 = time.perf_counter()
    G = pcg.build_g_host(pcg.G_FSAI, A)
    t_construct = time.perf_counter() - t0
    solver = pcg.Solver(pcg.default_config(device=0))
    solver.set_matrix(A)
    t0 = time.perf_counter()
    solver.set_precond(rowptr=G[0], col=G[1], val=G[2])
    t_place = time.perf_counter() - t0
    b_dev = torch.from_numpy(b).to(dev)
    torch.cuda.synchronize()

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        solver.solve(b_dev, tol=TOL, maxit=MAXIT)
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
    x_fp64 = last.x.cpu().numpy()

    log("kernel timing")
    kt = solver.time_kernels(args.kernel_iters)
    names = ["k_iter_A", "k_iter_GT", "k_iter_G"]
    sv = algorithmic_bytes(A.n, A.nnz, int(G[1].shape[0]), 8, 8, 8)
    kernels = {name: {"avg_ms": kt["ms"][k], "layout_bytes": kt["bytes"][k], "alg_bytes": sv[k],
                      "alg_gbps": sv[k] / (kt["ms"][k] * 1e-3) / 1e9,
                      "layout_gbps": kt["bytes"][k] / (kt["ms"][k] * 1e-3) / 1e9}
               for k, name in enumerate(names)}
    dom = max(range(3), key=lambda k: kt["ms"][k])
    achieved = sv[dom] / (kt["ms"][dom] * 1e-3) / 1e9
    traffic = stored_traffic(names[dom])
    ms_iter = ms_per_step / iters
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": names[dom], "alg_bytes_per_launch": sv[dom], "avg_launch_ms": kt["ms"][dom],
                "bytes_basis": "int32 CSR indices and row pointers, 8-byte values, the vector streams the kernel "
                               "needs; the stored layouts move fewer (kernels[...].layout_bytes: sliced "
                               "diagonals keep one offset per slice entry, sliced ELL 16-bit differences)",
                "per_iteration": {"alg_bytes": sv[3], "ms": round(ms_iter, 5),
                                  "achieved_gbps": round(sv[3] / (ms_iter * 1e-3) / 1e9, 1),
                                  "frac": round(sv[3] / (ms_iter * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                                  "note": "one iteration's algorithmic bytes (11 vector streams) over the timed "
                                          "solve's time per iteration (graph gaps and replacement steps "
                                          "included)"}}
    # the same kernels with every matrix read nontemporally (nothing kept in
    # the memory-side cache): the HBM-only figures
    log("kernel timing, nontemporal loads only")
    with pcg.Solver(pcg.default_config(device=0, cache_mb=-1)) as snt:
        snt.set_matrix(A)
        snt.set_precond(rowptr=G[0], col=G[1], val=G[2])
        snt.solve(b_dev, tol=TOL, maxit=MAXIT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rnt = snt.solve(b_dev, tol=TOL, maxit=MAXIT)
        ms_nt = (time.perf_counter() - t0) * 1e3
        ktn = snt.time_kernels(args.kernel_iters)
    hbm_only = {name: {"avg_ms": ktn["ms"][k], "alg_gbps": sv[k] / (ktn["ms"][k] * 1e-3) / 1e9,
                       "frac": sv[k] / (ktn["ms"][k] * 1e-3) / 1e9 / HBM_PEAK_GBPS}
                for k, name in enumerate(names)}
    hbm_only["solve"] = {"time_to_tol_ms": round(ms_nt, 3), "iters": rnt.iters,
                         "alg_gbps_per_iter": round(sv[3] / (ms_nt / rnt.iters * 1e-3) / 1e9, 1),
                         "frac_per_iter": round(sv[3] / (ms_nt / rnt.iters * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
    copy = None
    if not args.no_copy_probe:
        log("copy and read probes")
        gb, ms = pcg.copy_bandwidth(4 << 30, reps=10)
        gr, msr = pcg.read_bandwidth(4 << 30, reps=10)
        copy = {"copy_gbps": round(gb, 1), "read_gbps": round(gr, 1), "bytes": 4 << 30, "ms_per_copy": ms,
                "ms_per_read": msr}
    relres = last.relres_true  # ||b - A x|| / ||b|| from the library's FP64 residual kernel
    solver.close()
    # the same FSAI factored on the device (pattern work on the host, rows on
    # the GPU, placement into the layouts), A already set
    log("device FSAI construction")
    with pcg.Solver(pcg.default_config(device=0, g_device=1)) as s2:
        s2.set_matrix(A)
        s2.build_precond(pcg.G_FSAI)  # warm-up (first-use costs)
        t0 = time.perf_counter()
        s2.build_precond(pcg.G_FSAI)
        t_construct_dev = time.perf_counter() - t0

    extra, sols, refs = {}, {"fp64": x_fp64}, {}
    if "mixed" in sections:
        log("mixed precision")
        extra["mixed"], sols["mixed_f32_bf16_refined"] = section_mixed(pcg, torch, A, G, b_dev, max(3, args.steps // 2),
                                                                       ms_per_step)
    if "sai_loss" in sections:
        log("sai loss")
        extra["sai_loss"] = section_sai_loss(pcg, inputs, A, G, args.probes)
    if "autotune" in sections:
        log("autotune")
        extra["autotune"] = section_autotune(pcg, torch, inputs, A, G, b_dev, max(3, args.steps // 2), ms_per_step)
    if "small" in sections:
        log("small systems")
        extra["small"] = section_small(pcg, inputs)
    if "batched" in sections and args.batch_systems > 0:
        extra["batched"], refs["batched_sample"] = section_batched(pcg, inputs, args.batch_systems)
    if "serving_stream" in sections and args.serve_requests > 0:
        extra["serving_stream"] = section_serving_stream(
            pcg, inputs, args.serve_requests, args.serve_pool, args.serve_window, args.serve_step,
            [float(f) for f in args.serve_loads.split(",") if f], args.serve_mu)
    if "serving" in sections and args.serve_requests > 0:
        extra["serving"], refs["served_sample"] = section_serving(pcg, inputs, args.serve_requests, args.serve_step)
    if "elasticity" in sections and args.elasticity_n > 0:
        extra["elasticity"], refs["elasticity"] = section_elasticity(pcg, inputs, args.elasticity_n)
    if "synthetic" in sections and args.synthetic_batch > 0:
        extra["synthetic"] = section_synthetic(pcg, inputs, args.synthetic_batch)
    cpu = None
    if not args.no_cpu_baseline:
        log("oracle leg: cpu baseline, full-size parity, errors against converged oracle solutions")
        cpu = oracle_leg(pcg, torch, A, b, {"iters": iters, "solutions": sols}, args.cpu_budget_s, refs)
    del b_dev

    line = {
        "metric": METRIC, "value": round(1e3 / ms_per_step, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "poisson3d_7pt_128^3_lognormal_sigma1_fsai_f64_tol1e-8", "n": A.n, "nnz_a": A.nnz,
                   "nnz_g": int(G[1].shape[0]), "tol": TOL, "x0": "zeros", "rr_period": 50},
        "time_to_tol_ms": round(ms_per_step, 3), "iters": iters, "ms_per_iter": round(ms_per_step / iters, 5),
        "hbm_gbps_per_iter": round(gbps_iter, 1), "alg_bytes_per_iter": bpi,
        "relres_true_fp64": relres, "t_construct_s": round(t_construct, 3),
        "t_construct_host_total_s": round(t_construct + t_place, 4), "t_construct_device_s": round(t_construct_dev, 4),
        "roofline": roofline, "kernels": kernels, "hbm_only": hbm_only, "stream_probes": copy,
        "cpu_baseline": cpu,
        "kernel_sources_sha": kernel_sha(),
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
