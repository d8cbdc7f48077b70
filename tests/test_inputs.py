"""Pins for the seeded input generators (no solver arithmetic here)."""
import numpy as np
import pytest

from paper_2510_27517_amd import inputs

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def _mix(z):
    # SplitMix64 output finaliser, from the published definition
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def test_splitmix_reference_vector():
    # first output of SplitMix64 seeded with state 0 is 0xE220A8397B1DCDAF
    assert _mix(GAMMA) == 0xE220A8397B1DCDAF


@pytest.mark.parametrize("seed,stream", [(0, 1), (7, 2), (2**40 + 3, 9)])
def test_counter_generator_matches_definition(seed, stream):
    key = _mix((_mix((seed + GAMMA) & MASK) + (stream + 1) * GAMMA) & MASK)
    for i in [0, 1, 2, 1000, 123456789]:
        assert inputs.bits(seed, stream, i) == _mix((key + (i + 1) * GAMMA) & MASK)
    u = inputs.u01(seed, stream, 4)
    for i in range(4):
        v = _mix((key + (i + 1) * GAMMA) & MASK)
        assert u[i] == ((v >> 11) + 1) * 2.0 ** -53


def test_indexed_draws_match_definition():
    seed, stream = 11, 3
    key = _mix((_mix((seed + GAMMA) & MASK) + (stream + 1) * GAMMA) & MASK)
    idx = np.array([0, 5, 2**33 + 7, 123456789012, 3], np.uint64)
    got = inputs.u01_at(seed, stream, idx)
    for k, i in enumerate(idx.tolist()):
        v = _mix((key + (i + 1) * GAMMA) & MASK)
        assert got[k] == ((v >> 11) + 1) * 2.0 ** -53
    assert np.array_equal(inputs.u01_at(seed, stream, np.arange(50)), inputs.u01(seed, stream, 50))


def test_normal_moments_and_determinism():
    z = inputs.normal(0, inputs.STREAM_B, 200_000)
    assert abs(z.mean()) < 4 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 0.02
    assert np.array_equal(z[:1000], inputs.normal(0, inputs.STREAM_B, 1000))
    assert not np.array_equal(z[:1000], inputs.normal(1, inputs.STREAM_B, 1000))
    u = inputs.u01(3, 4, 100_000)
    assert u.min() > 0 and u.max() <= 1 and abs(u.mean() - 0.5) < 0.01


@pytest.mark.parametrize("dim,N", [(2, 1), (2, 7), (2, 64), (3, 1), (3, 5), (3, 12)])
def test_poisson_nnz_formula_and_symmetry(dim, N):
    A = inputs.poisson(dim, N, sigma=1.0, seed=3)
    expect = 5 * N * N - 4 * N if dim == 2 else 7 * N ** 3 - 6 * N ** 2
    assert A.nnz == expect
    S = A.to_scipy()
    assert abs(S - S.T).max() == 0.0
    for i in range(A.n):
        cols = A.col[A.rowptr[i]:A.rowptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols


@pytest.mark.parametrize("dim,N", [(2, 6), (3, 4)])
def test_poisson_constant_eigenvalues_closed_form(dim, N):
    A = inputs.poisson(dim, N, sigma=0.0).to_dense()
    th = np.arange(1, N + 1) * np.pi / (N + 1)
    one = 2 - 2 * np.cos(th)
    if dim == 2:
        lam = (one[:, None] + one[None, :]).ravel()
    else:
        lam = (one[:, None, None] + one[None, :, None] + one[None, None, :]).ravel()
    assert np.allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(lam), atol=1e-12)


def test_poisson_variable_coefficients_structure():
    N = 5
    A = inputs.poisson(3, N, sigma=1.0, seed=11)
    D = A.to_dense()
    # off-diagonals are negative face coefficients; the diagonal exceeds the
    # off-diagonal row sum by the boundary faces, which are positive
    off = D - np.diag(np.diag(D))
    assert np.all(off <= 0)
    excess = np.diag(D) + off.sum(axis=1)
    interior = [x + N * (y + N * z) for z in range(1, N - 1) for y in range(1, N - 1) for x in range(1, N - 1)]
    assert np.allclose(excess[interior], 0.0, atol=1e-12)
    boundary = sorted(set(range(N ** 3)) - set(interior))
    assert np.all(excess[boundary] > 0)
    assert np.linalg.eigvalsh(D).min() > 0
    # coefficients are lognormal(sigma=1): log of the faces has unit spread
    faces = -off[np.triu_indices(N ** 3, 1)]
    faces = faces[faces > 0]
    assert 0.7 < np.log(faces).std() < 1.3


def test_rgg_laplacian():
    n = 20_000
    A = inputs.rgg_laplacian(n, seed=5)
    S = A.to_scipy()
    assert abs(S - S.T).max() == 0.0
    rows = np.asarray(S.sum(axis=1)).ravel()
    assert np.allclose(rows, 1e-3, atol=1e-9)
    deg = np.diff(A.rowptr) - 1
    assert 7.0 < deg.mean() < 8.05
    off = S.copy()
    off.setdiag(0)
    w = -off.data[off.data != 0]
    assert w.min() >= 0.1 and w.max() <= 10.0
    small = inputs.rgg_laplacian(200, seed=1).to_dense()
    assert np.linalg.eigvalsh(small).min() > 0


def test_elasticity_structure_and_patch_test():
    N = 5
    A = inputs.elasticity(N, sigma=0.0)
    assert A.nnz == 9 * (3 * N - 2) ** 3
    D = A.to_dense()
    assert np.allclose(D, D.T, atol=1e-12 * np.abs(D).max())
    assert np.linalg.eigvalsh(D).min() > 0
    # patch test: a linear displacement field produces no force at nodes whose
    # whole 3x3x3 neighbourhood is free (constant material)
    h = 1.0 / (N + 1)
    rng = np.random.default_rng(0)
    Mg = rng.standard_normal((3, 3))
    c0 = rng.standard_normal(3)
    u = np.zeros(3 * N ** 3)
    for z in range(N):
        for y in range(N):
            for x in range(N):
                p = np.array([(x + 1) * h, (y + 1) * h, (z + 1) * h])
                u[3 * (x + N * (y + N * z)):3 * (x + N * (y + N * z)) + 3] = Mg @ p + c0
    f = D @ u
    for z in range(1, N - 1):
        for y in range(1, N - 1):
            for x in range(1, N - 1):
                i = x + N * (y + N * z)
                assert np.abs(f[3 * i:3 * i + 3]).max() < 1e-10 * np.abs(D).max()


def test_elasticity_lognormal_symmetric():
    A = inputs.elasticity(3, sigma=1.0, seed=2)
    D = A.to_dense()
    assert np.allclose(D, D.T, atol=1e-12 * np.abs(D).max())
    assert np.linalg.eigvalsh(D).min() > 0
