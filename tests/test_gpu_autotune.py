"""The autotuner on the GPU: it times the layouts and grids a matrix admits,
keeps the fastest, caches the choice per matrix signature, and the tuned
solve still holds FP64 parity with the oracle."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2510_27517_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def _parity(s, got, A, b, tol):
    """The parity bar for converged solves whose stop test may land one
    iteration apart: the first 10 iterates within 1e-10 of the oracle's, the
    converged iteration count within one of the oracle's, the FP64 residual
    within tol."""
    G = oracle.fsai_g(A)
    ten = s.solve(b, tol=0.0, maxit=10)
    ref10 = oracle.pcg(A, G, b, tol=0.0, maxit=10, delta_form=1)
    err = np.linalg.norm(ten.x - ref10.x) / np.linalg.norm(ref10.x)
    assert err <= 1e-10, err
    ref = oracle.pcg(A, G, b, tol=tol, maxit=5000, delta_form=1)
    assert got.status == ref.status == 0 and abs(got.iters - ref.iters) <= 1, (got.iters, ref.iters)
    assert np.linalg.norm(b - oracle.spmv(A, got.x)) <= tol * np.linalg.norm(b) * (1 + 1e-6)
    return err


def test_autotune_search_cache_and_parity(gpu_lib, tmp_path):
    pcg = gpu_lib
    cache = tmp_path / "tune.txt"
    os.environ["PCG_TUNE_CACHE"] = str(cache)
    A = inputs.poisson(3, 40, 1.0, 11)
    b = inputs.rhs(A.n, 11)
    with pcg.Solver(pcg.default_config()) as s:
        s.set_matrix(A)
        s.build_precond(pcg.G_FSAI)
        pre = s.solve(b, tol=1e-8, maxit=5000)
        t = s.autotune(10)
        say("poisson 40^3 tuned:", t)
        assert t["candidates"] >= 5  # automatic, {CSR, SELL} x {CSR, SELL}, two grids
        assert t["ms_per_iter"] <= t["ms_per_iter_auto"]
        got = s.solve(b, tol=1e-8, maxit=5000)
        err = _parity(s, got, A, b, 1e-8)
    say(f"  untuned {pre.iters}, tuned {got.iters} iterations, 10-iterate error {err:.2e}")
    # layouts give the same products and the inner products are exact, so any
    # choice of layouts, grid and load policy gives the same solve bit for bit
    assert got.iters == pre.iters and np.array_equal(got.x, pre.x)
    with pcg.Solver(pcg.default_config()) as s:
        s.set_matrix(A)
        s.build_precond(pcg.G_FSAI)
        t2 = s.autotune(10)
        assert t2["candidates"] == 0
        for k in ("layout_a", "layout_g", "grid_mult", "fmt_a", "fmt_g", "fmt_gt", "idx16", "temporal",
                  "rows_per_lane_gt", "loads_in_flight_a"):
            assert t2[k] == t[k], k
        got2 = s.solve(b, tol=1e-8, maxit=5000)
    assert np.array_equal(got2.x, got.x)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith(f"n{A.n}_a{A.nnz}_")


def test_autotune_elasticity_considers_blocks(gpu_lib):
    pcg = gpu_lib
    A = inputs.elasticity(6, 1.0, 0.3, 12)
    b = inputs.rhs(A.n, 12)
    with pcg.Solver(pcg.default_config()) as s:
        s.set_matrix(A)
        s.build_precond(pcg.G_FSAI)
        t = s.autotune(10)
        say("elasticity 6^3 tuned:", t)
        assert t["candidates"] >= 8  # automatic, {CSR, SELL, 3x3} x {CSR, SELL}, two grids
        got = s.solve(b, tol=1e-10, maxit=5000)
        _parity(s, got, A, b, 1e-10)


def test_autotune_on_create_with_device_fsai(gpu_lib):
    """autotune = 1: pcg_build_precond tunes at once; G built on the device is
    factored again for each G layout, and the result keeps parity."""
    pcg = gpu_lib
    A = inputs.poisson(3, 28, 0.5, 13)
    b = inputs.rhs(A.n, 13)
    with pcg.Solver(pcg.default_config(autotune=1, g_device=1)) as s:
        s.set_matrix(A)
        s.build_precond(pcg.G_FSAI)
        got = s.solve(b, tol=1e-8, maxit=5000)
        t = s.autotune(10)  # cached by the build's own tuning
        assert t["candidates"] == 0
        _parity(s, got, A, b, 1e-8)


def test_autotune_keeps_forced_layout(gpu_lib):
    pcg = gpu_lib
    A = inputs.poisson(3, 24, 1.0, 14)
    b = inputs.rhs(A.n, 14)
    with pcg.Solver(pcg.default_config(layout="csr")) as s:
        s.set_matrix(A)
        s.build_precond(pcg.G_FSAI)
        t = s.autotune(10)
        assert t["fmt_a"] == 0 and t["fmt_g"] == 0 and t["fmt_gt"] == 0 and t["candidates"] == 13
        got = s.solve(b, tol=1e-8, maxit=5000)
        _parity(s, got, A, b, 1e-8)


def test_autotune_mixed_precision_with_refinement(gpu_lib):
    """FP32 vectors and A, BF16 G, FP64 refinement: the tuner times the FP32
    inner iteration; the refined solve still reaches 1e-10 in FP64 and
    equals the untuned solve bit for bit when the automatic choice wins."""
    pcg = gpu_lib
    A = inputs.poisson(3, 32, 1.0, 15)
    b = inputs.rhs(A.n, 15)
    kw = dict(vec_dtype="f32", a_dtype="f32", g_dtype="bf16", refine=1)
    with pcg.Solver(pcg.default_config(**kw)) as s:
        s.set_matrix(A)
        s.build_precond(pcg.G_FSAI)
        pre = s.solve(b, tol=1e-10, maxit=3000)
        t = s.autotune(10)
        got = s.solve(b, tol=1e-10, maxit=3000)
    say("mixed tuned:", t)
    r64 = np.linalg.norm(b - oracle.spmv(A, got.x)) / np.linalg.norm(b)
    assert got.status == pcg.OK and r64 <= 1.0001e-10 and t["candidates"] >= 5
    assert got.iters == pre.iters and np.array_equal(got.x, pre.x)
