"""The allocation-free loss entry point (pcg_sai_loss_noalloc) against the
allocating one (pcg_sai_loss): same kernels and summation order, so the same
losses, on two calls in a row (the second with a smaller input) and from two
contexts sharing the device's static scratch."""
import sys

import numpy as np
import pytest

from paper_2510_27517_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def _probes(torch, n, k, seed):
    return torch.from_numpy(inputs.normal(seed, inputs.STREAM_PROBE, n * k).reshape(n, k)).to("cuda:0")


def _same(a, b):
    assert np.array_equal(a["sai"], b["sai"]) and np.array_equal(a["l2"], b["l2"])
    assert np.allclose(a["cs"], b["cs"], rtol=4e-16, atol=0)


def test_noalloc_loss_equals_allocating_loss(gpu_lib):
    import torch

    pcg = gpu_lib
    A1 = inputs.poisson(3, 24, 1.0, 3)
    A2 = inputs.rgg_laplacian(3000, 4)
    with pcg.Solver(pcg.default_config(eps=0.01)) as s1, pcg.Solver(pcg.default_config()) as s2:
        s1.set_matrix(A1)
        s1.build_precond(pcg.G_FSAI)
        s2.set_matrix(A2)
        s2.build_precond(pcg.G_FSAI)
        for s, A, k, seed in [(s1, A1, 16, 1), (s1, A1, 5, 2), (s2, A2, 3, 3)]:
            say(f"noalloc loss n={A.n} k={k}")
            W = _probes(torch, A.n, k, seed)
            got = s.sai_loss_noalloc(W)
            ref = s.sai_loss(W)
            _same(got, ref)
        # a request beyond the static scratch is refused, nothing computed
        W = _probes(torch, A1.n, 700, 4)
        with pytest.raises(pcg.PCGError) as ei:
            s1.sai_loss_noalloc(W)
        assert ei.value.status == pcg.EINVAL and "static scratch" in str(ei.value)
        # and the scratch still serves the next call
        W = _probes(torch, A1.n, 4, 5)
        _same(s1.sai_loss_noalloc(W), s1.sai_loss(W))
