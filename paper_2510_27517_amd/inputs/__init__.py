"""Seeded synthetic inputs for the preconditioned-CG path.

Thin ctypes front end over ``gen.c`` (built to ``libpcggen.so`` beside it).
It produces the systems A x = b that the workloads describe and the random
draws they need; it holds none of the solver's arithmetic, so the HIP library
and the FP64 oracle can both take their inputs from it without sharing any
method code.

Workloads (stand-ins for the paper's FEM heat/Poisson, hyperelasticity and
algebraic datasets, Sec. 4.1, which are not available):
  * ``poisson(dim, N, sigma)``: 2D 5-point / 3D 7-point Dirichlet Poisson with
    lognormal face coefficients k = exp(sigma Z).
  * ``rgg_laplacian(n)``: random-geometric-graph Laplacian + 1e-3 I.
  * ``elasticity(N)``: Q1 hexahedral linear-elasticity block system, 3 dof per
    node (the paper's blocked case, b = 3, Sec. 3.1).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcggen.so")

# Stream ids of the counter-based generator (one per kind of draw).
STREAM_B = 1
STREAM_COEF = 2
STREAM_G = 3
STREAM_PTS = 4
STREAM_W = 5
STREAM_SIZES = 6
STREAM_ARRIVALS = 7
STREAM_KIND = 8
STREAM_E = 9
STREAM_REQ = 10
STREAM_PROBE = 11  # probe vectors of the loss estimators
STREAM_SYN_POS = 12  # positions of P's entries (synthetic P P^T systems)
STREAM_SYN_VAL = 13  # values of P's entries

_lib = None


def build(verbose: bool = False) -> str:
    """Compile gen.c into libpcggen.so (plain gcc, no GPU code)."""
    import subprocess

    src = os.path.join(_HERE, "gen.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    global _lib
    _lib = None
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    u64, i64, dbl, i32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    P = ctypes.c_void_p
    lib.gen_bits.restype = u64
    lib.gen_bits.argtypes = [u64, u64, u64]
    lib.gen_u01.restype = dbl
    lib.gen_u01.argtypes = [u64, u64, u64]
    lib.gen_normal.restype = dbl
    lib.gen_normal.argtypes = [u64, u64, u64]
    lib.gen_u01_vec.argtypes = [u64, u64, i64, P]
    lib.gen_u01_at.argtypes = [u64, u64, i64, P, P]
    lib.gen_normal_vec.argtypes = [u64, u64, i64, P]
    lib.gen_poisson_nnz.restype = i64
    lib.gen_poisson_nnz.argtypes = [i32, i64]
    lib.gen_poisson.restype = i64
    lib.gen_poisson.argtypes = [i32, i64, dbl, u64, u64, P, P, P]
    lib.gen_rgg_laplacian.restype = i64
    lib.gen_rgg_laplacian.argtypes = [i64, dbl, u64, u64, u64, P, P, P]
    lib.gen_free.argtypes = [P]
    lib.gen_elasticity_nnz.restype = i64
    lib.gen_elasticity_nnz.argtypes = [i64]
    lib.gen_elasticity.restype = i64
    lib.gen_elasticity.argtypes = [i64, dbl, dbl, u64, u64, P, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass
class CSR:
    """Square CSR matrix: int32 rowptr (n+1), int32 col (nnz), float64 val (nnz)."""

    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        for i in range(self.n):
            for k in range(self.rowptr[i], self.rowptr[i + 1]):
                d[i, self.col[k]] += self.val[k]
        return d

    @staticmethod
    def from_dense(d: np.ndarray, keep_zeros_on_diag: bool = True) -> "CSR":
        n = d.shape[0]
        rp = [0]
        cols, vals = [], []
        for i in range(n):
            for j in range(d.shape[1]):
                if d[i, j] != 0.0 or (keep_zeros_on_diag and i == j):
                    cols.append(j)
                    vals.append(d[i, j])
            rp.append(len(cols))
        return CSR(np.asarray(rp, np.int32), np.asarray(cols, np.int32), np.asarray(vals, np.float64))

    @staticmethod
    def from_scipy(m) -> "CSR":
        m = m.tocsr()
        m.sort_indices()
        return CSR(m.indptr.astype(np.int32), m.indices.astype(np.int32), m.data.astype(np.float64))


def bits(seed: int, stream: int, i: int) -> int:
    return int(_load().gen_bits(seed, stream, i))


def u01(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, np.float64)
    _load().gen_u01_vec(seed, stream, n, _ptr(out))
    return out


def u01_at(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """u01 draws at the given (non-negative) indices of a stream."""
    ix = np.ascontiguousarray(idx, dtype=np.uint64)
    out = np.empty(ix.shape[0], np.float64)
    _load().gen_u01_at(seed, stream, ix.shape[0], _ptr(ix), _ptr(out))
    return out


def normal(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, np.float64)
    _load().gen_normal_vec(seed, stream, n, _ptr(out))
    return out


def rhs(n: int, seed: int = 0) -> np.ndarray:
    """b ~ N(0, 1), entry i drawn at index i of the right-hand-side stream."""
    return normal(seed, STREAM_B, n)


def poisson(dim: int, N: int, sigma: float = 0.0, seed: int = 0) -> CSR:
    lib = _load()
    n = N ** dim
    nnz = int(lib.gen_poisson_nnz(dim, N))
    rp = np.empty(n + 1, np.int32)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    got = lib.gen_poisson(dim, N, float(sigma), seed, STREAM_COEF, _ptr(rp), _ptr(col), _ptr(val))
    if got != nnz:
        raise RuntimeError(f"gen_poisson returned {got}, expected {nnz}")
    return CSR(rp, col, val)


def rgg_laplacian(n: int, seed: int = 0, shift: float = 1e-3) -> CSR:
    lib = _load()
    prp, pcol, pval = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    nnz = lib.gen_rgg_laplacian(n, float(shift), seed, STREAM_PTS, STREAM_W,
                                ctypes.byref(prp), ctypes.byref(pcol), ctypes.byref(pval))
    if nnz < 0:
        raise ValueError("bad RGG arguments")
    try:
        rp = np.ctypeslib.as_array(ctypes.cast(prp, ctypes.POINTER(ctypes.c_int32)), (n + 1,)).copy()
        col = np.ctypeslib.as_array(ctypes.cast(pcol, ctypes.POINTER(ctypes.c_int32)), (nnz,)).copy()
        val = np.ctypeslib.as_array(ctypes.cast(pval, ctypes.POINTER(ctypes.c_double)), (nnz,)).copy()
    finally:
        lib.gen_free(prp)
        lib.gen_free(pcol)
        lib.gen_free(pval)
    return CSR(rp, col, val)


def synthetic_ppt(n: int, seed: int = 0, density: float = 3e-4, shift: float = 1e-4) -> CSR:
    """The paper's synthetic SPD system (Sec. 4.1, App. C): A = P P^T + shift I
    with P an n x n random sparse matrix of the given density. P has
    round(density n^2) entries at uniform positions (row, column from two
    draws of the position stream; coinciding positions add up) with N(0,1)
    values; A's density comes out near 1.2e-3 for n in [12000, 24000]."""
    import scipy.sparse as sp

    m = int(round(density * n * n))
    u = u01(seed, STREAM_SYN_POS, 2 * m)
    rows = np.minimum((u[0::2] * n).astype(np.int64), n - 1)
    cols = np.minimum((u[1::2] * n).astype(np.int64), n - 1)
    vals = normal(seed, STREAM_SYN_VAL, m)
    P = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A = (P @ P.T + shift * sp.identity(n, format="csr")).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return CSR.from_scipy(A)


def elasticity(N: int, sigma: float = 1.0, nu: float = 0.3, seed: int = 0) -> CSR:
    lib = _load()
    n = 3 * N ** 3
    nnz = int(lib.gen_elasticity_nnz(N))
    rp = np.empty(n + 1, np.int32)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    got = lib.gen_elasticity(N, float(sigma), float(nu), seed, STREAM_E, _ptr(rp), _ptr(col), _ptr(val))
    if got != nnz:
        raise RuntimeError(f"gen_elasticity returned {got}, expected {nnz}")
    return CSR(rp, col, val)


def random_spd(n: int, density: float, seed: int) -> CSR:
    """Small random sparse SPD test matrix: symmetric random pattern with
    U(-1,1) off-diagonals and a strictly dominant positive diagonal (plus a
    random positive excess), so it is SPD by Gershgorin."""
    u = u01(seed, STREAM_REQ, 3 * n * n)
    pat = u[: n * n].reshape(n, n) < density
    vals = 2.0 * u[n * n: 2 * n * n].reshape(n, n) - 1.0
    m = np.where(pat, vals, 0.0)
    m = np.triu(m, 1)
    m = m + m.T
    diag = np.abs(m).sum(axis=1) + 0.1 + u[2 * n * n: 2 * n * n + n]
    m[np.arange(n), np.arange(n)] = diag
    return CSR.from_dense(m)
