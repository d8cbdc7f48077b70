"""Caller-supplied device memory and stream: a context whose allocations all
go through PyTorch's caching allocator, and one that runs on PyTorch's
stream, give the same results bit for bit as the default context."""
import sys

import numpy as np
import pytest

from paper_2510_27517_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def test_torch_allocator_single_and_batch(gpu_lib):
    import torch

    pcg = gpu_lib
    A = inputs.poisson(3, 30, 1.0, 21)
    b = inputs.rhs(A.n, 21)
    with pcg.Solver(pcg.default_config()) as s:
        s.set_matrix(A)
        s.build_precond(pcg.G_FSAI)
        ref = s.solve(b, tol=1e-8, maxit=3000)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(0)
    alloc = pcg.TorchAllocator(0)
    with pcg.Solver(pcg.default_config(), allocator=alloc) as s:
        s.set_matrix(A)
        s.build_precond(pcg.G_FSAI)
        held = sum(alloc.live.values())
        grown = torch.cuda.memory_allocated(0) - base
        say(f"torch allocator: {len(alloc.live)} blocks, {held} bytes held, torch reports +{grown}")
        assert held >= A.nnz * 10 and grown >= held
        got = s.solve(b, tol=1e-8, maxit=3000)
    assert got.status == ref.status == pcg.OK and got.iters == ref.iters
    assert np.array_equal(got.x, ref.x)
    assert not alloc.live and torch.cuda.memory_allocated(0) == base
    systems = [dict(A=inputs.poisson(2, 20 + 7 * k, 0.5, k), b=inputs.rhs((20 + 7 * k) ** 2, k), tol=1e-8,
                    maxit=3000) for k in range(6)]
    with pcg.Solver(pcg.default_config(mem_budget_mb=16)) as s:
        ref_b = s.solve_batch(systems)
    alloc = pcg.TorchAllocator(0)
    with pcg.Solver(pcg.default_config(mem_budget_mb=16), allocator=alloc) as s:
        got_b = s.solve_batch(systems)
        assert max(alloc.live.values()) >= 16 << 20  # the pool came from torch
    assert not alloc.live
    for (xr, rr), (xg, rg) in zip(ref_b, got_b):
        assert rg["status"] == rr["status"] == pcg.OK and rg["iters"] == rr["iters"]
        assert np.array_equal(xg, xr)


def test_caller_stream(gpu_lib):
    import torch

    pcg = gpu_lib
    A = inputs.poisson(3, 24, 1.0, 22)
    b = torch.from_numpy(inputs.rhs(A.n, 22)).to("cuda:0")
    with pcg.Solver(pcg.default_config()) as s:
        s.set_matrix(A)
        s.build_precond(pcg.G_FSAI)
        ref = s.solve(b, tol=1e-8, maxit=3000)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        with pcg.Solver(pcg.default_config(stream=st.cuda_stream)) as s:
            s.set_matrix(A)
            s.build_precond(pcg.G_FSAI)
            got = s.solve(b, tol=1e-8, maxit=3000)
            got2 = s.solve(b, tol=1e-8, maxit=3000)
    torch.cuda.synchronize()
    assert got.iters == ref.iters and torch.equal(got.x, ref.x) and torch.equal(got2.x, ref.x)
