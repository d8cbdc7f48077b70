"""Caller-supplied device memory and stream: a context whose allocations all
go through PyTorch's caching allocator, and one that runs on PyTorch's
stream, give the same results bit for bit as the default context."""
import sys
import time

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


def test_admission_failure_finishes_tickets(gpu_lib):
    """A device allocation refused during admission (the scratch of the device
    FSAI, by the caller's allocator) starts none of that step's systems: each
    ticket finishes with PCG_ENOMEM, the pool is empty again, and the same
    context then solves the same systems as a fresh one does."""
    pcg = gpu_lib

    class Refusing(pcg.TorchAllocator):
        def __init__(self):
            super().__init__(0)
            self.refuse = False
            inner = self.alloc_fn

            def _alloc(nbytes, user):
                return None if self.refuse else inner(nbytes, user)

            self.alloc_fn = pcg.ALLOC_FN(_alloc)

    systems = [dict(A=inputs.poisson(3, 12 + 2 * k, 1.0, 30 + k), b=inputs.rhs((12 + 2 * k) ** 3, k), tol=1e-8,
                    maxit=3000) for k in range(3)]
    cfg = dict(g_device=1, mem_budget_mb=64)
    with pcg.Solver(pcg.default_config(**cfg)) as s:
        ref = s.solve_batch(systems)
    alloc = Refusing()
    with pcg.Solver(pcg.default_config(**cfg), allocator=alloc) as s:
        first = s.solve_batch(systems)  # pool and scheduler buffers exist from here on
        alloc.refuse = True
        tickets = s.submit(systems)
        done, errors = {}, 0
        for _ in range(5000):
            try:
                s.progress(1)
            except pcg.PCGError:
                errors += 1
            for t in tickets:
                if t not in done:
                    r = s.poll(t)
                    if r is not None:
                        done[t] = r
            if len(done) == len(tickets):
                break
            time.sleep(0.002)
        say(f"refused admission: {errors} failing steps, statuses {[r[1]['status'] for r in done.values()]}")
        assert len(done) == len(tickets) and errors >= 1
        assert all(r[1]["status"] == pcg.ENOMEM for r in done.values())
        assert s.pool_info()[1] == 0
        alloc.refuse = False
        again = s.solve_batch(systems)
    assert not alloc.live
    for (xr, rr), (xf, rf), (xa, ra) in zip(ref, first, again):
        assert rr["status"] == rf["status"] == ra["status"] == pcg.OK
        assert rr["iters"] == rf["iters"] == ra["iters"]
        assert np.array_equal(xf, xr) and np.array_equal(xa, xr)
