"""Host-side checks of the C ABI library: it loads, exports every declared
symbol, validates CSR input, and its host preconditioner builders agree with
the oracle's independent ones. No GPU calls."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2510_27517_amd import inputs, pcg
from paper_2510_27517_amd.inputs import CSR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(pcg.LIB_PATH):
        from paper_2510_27517_amd import build

        build.build()
    pcg.load()


def _declared():
    text = open(os.path.join(ROOT, "include", "pcg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pcg_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 14
    lib = pcg.load()
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(pcg.EXPORTS) == names


def test_strerror_covers_codes():
    lib = pcg.load()
    for code in (0, 1, 2, -1, -2, -3, -4, -5):
        assert lib.pcg_strerror(code).decode() != "unknown status"


def test_validate_csr():
    A = inputs.poisson(2, 5)
    assert pcg.validate_csr(A.rowptr, A.col) == pcg.OK
    bad = A.col.copy()
    bad[3], bad[4] = bad[4], bad[3]
    assert pcg.validate_csr(A.rowptr, bad) == pcg.EINVAL
    oob = A.col.copy()
    oob[-1] = A.n
    assert pcg.validate_csr(A.rowptr, oob) == pcg.EINVAL
    rp = A.rowptr.copy()
    rp[0] = 1
    assert pcg.validate_csr(rp, A.col) == pcg.EINVAL
    nodiag = CSR(np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.ones(2))
    assert pcg.validate_csr(nodiag.rowptr, nodiag.col, require_diag=True) == pcg.EINVAL
    assert pcg.validate_csr(nodiag.rowptr, nodiag.col, require_diag=False) == pcg.OK
    dup = CSR(np.array([0, 2], np.int32), np.array([0, 0], np.int32), np.ones(2))
    assert pcg.validate_csr(dup.rowptr, dup.col, n=1) == pcg.EINVAL


@pytest.mark.parametrize("case", ["poisson3d", "rgg", "elasticity"])
def test_library_fsai_matches_oracle(case):
    A = {"poisson3d": lambda: inputs.poisson(3, 10, 1.0, 3), "rgg": lambda: inputs.rgg_laplacian(3000, 2),
         "elasticity": lambda: inputs.elasticity(4, 1.0)}[case]()
    grp, gci, gv = pcg.build_g_host(pcg.G_FSAI, A)
    G = oracle.fsai_g(A)
    assert np.array_equal(grp, G.rowptr) and np.array_equal(gci, G.col)
    # row-wise: entries are relative to the row's largest (small entries come
    # from cancellation in the local solves)
    for i in range(A.n):
        sl = slice(G.rowptr[i], G.rowptr[i + 1])
        assert np.max(np.abs(gv[sl] - G.val[sl])) <= 1e-13 * np.max(np.abs(G.val[sl]))


def test_library_fixed_g_matches_oracle_exactly():
    A = inputs.poisson(2, 64)
    grp, gci, gv = pcg.build_g_host(pcg.G_FIXED, A)
    G = oracle.g_cfg1(A)
    assert np.array_equal(grp, G.rowptr) and np.array_equal(gci, G.col) and np.array_equal(gv, G.val)


@pytest.mark.parametrize("case", ["poisson3d", "rgg", "elasticity"])
def test_library_seeded_g_matches_oracle_exactly(case):
    A = {"poisson3d": lambda: inputs.poisson(3, 9, 1.0, 3), "rgg": lambda: inputs.rgg_laplacian(3000, 2),
         "elasticity": lambda: inputs.elasticity(4, 1.0)}[case]()
    for seed in (0, 2**40 + 9):
        grp, gci, gv = pcg.build_g_host(pcg.G_SEEDED, A, seed)
        G = oracle.seeded_g(A, seed)
        assert np.array_equal(grp, G.rowptr) and np.array_equal(gci, G.col) and np.array_equal(gv, G.val)


def test_library_jacobi_identity():
    A = inputs.poisson(3, 4, 1.0, 1)
    grp, gci, gv = pcg.build_g_host(pcg.G_JACOBI, A)
    J = oracle.diag_inv_sqrt(A)
    assert np.array_equal(gci, J.col) and np.allclose(gv, J.val, rtol=1e-15)
    _, _, iv = pcg.build_g_host(pcg.G_IDENTITY, A)
    assert np.all(iv == 1.0)


def test_bytes_per_iter_formula():
    n, a, g = 2_097_152, 14_581_760, 8_339_456
    got = pcg.bytes_per_iter(n, a, g, pcg.F64, pcg.F64, pcg.F64)
    assert got == a * 12 + 2 * g * 12 + 12 * (n + 1) + 11 * n * 8
    got32 = pcg.bytes_per_iter(n, a, g, pcg.F32, pcg.BF16, pcg.F32)
    assert got32 == a * 8 + 2 * g * 6 + 12 * (n + 1) + 11 * n * 4


def test_estimate_bytes_bounds():
    """Host-only admission estimate: at least the stored matrices and vectors,
    growing with the precision, with refinement, and with the sizes."""
    n, a, g = 262_144, 1_810_432, 1_036_288
    e64 = pcg.estimate_bytes(pcg.default_config(), n, a, g)
    assert e64 >= a * 12 + 2 * g * 12 + 8 * n * 8
    assert e64 <= 1.25 * (a * 12 + 2 * g * 12) + 16 * n * 8 + (1 << 20)
    mixed = pcg.default_config(vec_dtype="f32", a_dtype="f32", g_dtype="bf16")
    e32 = pcg.estimate_bytes(mixed, n, a, g)
    assert a * 8 + 2 * g * 6 + 8 * n * 4 <= e32 < e64
    mixed.refine = 1
    assert pcg.estimate_bytes(mixed, n, a, g) >= e32 + a * 8
    assert pcg.estimate_bytes(pcg.default_config(), 2 * n, 2 * a, 2 * g) > e64
    with pytest.raises(pcg.PCGError):
        pcg.estimate_bytes(pcg.default_config(), 0, a, g)


def test_allocator_callbacks_come_in_pairs():
    """alloc without free (or the reverse) is refused before any device work."""
    cfg = pcg.default_config()
    keep = pcg.ALLOC_FN(lambda n, u: None)
    cfg.alloc = pcg.ctypes.cast(keep, pcg.ctypes.c_void_p)
    with pytest.raises(pcg.PCGError) as e:
        pcg.Solver(cfg)
    assert e.value.status == pcg.EINVAL


@pytest.mark.parametrize("kw", [dict(rows_per_lane=3), dict(rows_per_lane=-1), dict(loads_in_flight=6),
                                dict(loads_in_flight=16)])
def test_kernel_knobs_validated(kw):
    """Knob values outside {0, 1, 2} rows per lane and {0, 4, 8} loads in
    flight are refused before any device work."""
    with pytest.raises(pcg.PCGError) as e:
        pcg.Solver(pcg.default_config(**kw))
    assert e.value.status == pcg.EINVAL


def test_create_without_gpu_fails_cleanly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(pcg.PCGError) as e:
        pcg.Solver()
    assert e.value.status == pcg.EDEVICE


@pytest.mark.parametrize("N", [3, 6])
def test_library_block_fsai_matches_oracle(N):
    """The library's block FSAI (last rows of the local L^-1) and the oracle's
    (the Cholesky factor of the local solution's diagonal block) pick
    different bases within each block row, but the same preconditioner:
    same pattern (full 3x3 blocks), M^-1 = G G^T equal to 1e-13, and the
    library's G_L A G_L^T has identity diagonal blocks."""
    A = inputs.elasticity(N, 1.0, 0.3, 2)
    grp, gci, gv = pcg.build_g_host(pcg.G_BFSAI, A)
    G = oracle.fsai_block_g(A)
    assert np.array_equal(grp, G.rowptr) and np.array_equal(gci, G.col)
    Gl, Go = CSR(grp, gci, gv).to_dense(), CSR(G.rowptr, G.col, G.val).to_dense()
    Ml, Mo = Gl @ Gl.T, Go @ Go.T
    assert np.abs(Ml - Mo).max() <= 1e-13 * np.abs(Mo).max()
    P = Gl.T @ A.to_dense() @ Gl
    for I in range(A.n // 3):
        assert np.abs(P[3 * I:3 * I + 3, 3 * I:3 * I + 3] - np.eye(3)).max() <= 1e-13
    assert pcg.load().pcg_g_nnz(pcg.G_BFSAI, A.n, A.rowptr.ctypes.data, A.col.ctypes.data) == G.nnz
    B = inputs.poisson(2, 6)  # n = 36 but not 3x3-blocked
    assert pcg.load().pcg_g_nnz(pcg.G_BFSAI, B.n, B.rowptr.ctypes.data, B.col.ctypes.data) == -1
