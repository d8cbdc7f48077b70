"""FP64 CPU oracle for PCG with M^-1 = G G^T + eps I (paper Sec. 3.2.1 and
Appendix A, Algorithm 1).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()``
and by the benchmark's ``cpu_baseline`` leg, never by the library. It wraps
``oracle.c`` (built to ``liboracle.so`` with gcc, contraction off) with numpy
arrays and shares no code with the HIP path.

Every function names the passage it follows; see ``oracle.c`` for the
readings of Algorithm 1 (replacement branch, stopping rule, restart on a
failed true-residual check) and of the inner products (exact sums of
products rounded once, so that no summation order is implied). ``pcg_ir`` emulates the mixed-precision solve
(FP64 iterative refinement around a PCG on rounded operands) in FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK = 0
NOT_CONVERGED = 2
EINVAL = -1
EBREAKDOWN = -4

_lib = None


def build(verbose: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    global _lib
    _lib = None
    return LIB_PATH


class _Opts(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("tol", ctypes.c_double), ("maxit", ctypes.c_int32),
                ("rr_period", ctypes.c_int32), ("delta_form", ctypes.c_int32), ("stop_rule", ctypes.c_int32),
                ("threads", ctypes.c_int32)]


class _Res(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("relres_rec", ctypes.c_double), ("relres_true", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.or_spmv.argtypes = [i32, P, P, P, P, P, ctypes.c_int]
    lib.or_spmv_t.argtypes = [i32, i32, P, P, P, P, P]
    lib.or_transpose.argtypes = [i32, i32, P, P, P, P, P, P]
    lib.or_spmv_f32.argtypes = [i32, P, P, P, P, P]
    lib.or_spmv_t_f32.argtypes = [i32, i32, P, P, P, P, P]
    lib.or_dot.restype = ctypes.c_double
    lib.or_dot.argtypes = [i32, P, P]
    lib.or_dot_threads.restype = ctypes.c_double
    lib.or_dot_threads.argtypes = [i32, P, P, ctypes.c_int]
    lib.or_apply_precond.argtypes = [i32, P, P, P, ctypes.c_double, P, P]
    lib.or_pcg.restype = ctypes.c_int
    lib.or_pcg.argtypes = [i32, P, P, P, P, P, P, P, P, ctypes.POINTER(_Opts), ctypes.POINTER(_Res), P, P]
    lib.or_tril_nnz.restype = ctypes.c_int64
    lib.or_tril_nnz.argtypes = [i32, P, P]
    lib.or_fsai_lower.restype = ctypes.c_int
    lib.or_fsai_lower.argtypes = [i32, P, P, P, P, P, P, ctypes.c_int]
    lib.or_bfsai_pattern.restype = ctypes.c_int64
    lib.or_bfsai_pattern.argtypes = [i32, P, P, ctypes.c_int, P]
    lib.or_fsai_block_lower.restype = ctypes.c_int
    lib.or_fsai_block_lower.argtypes = [i32, P, P, P, ctypes.c_int, P, P, P, ctypes.c_int]
    lib.or_g_cfg1.restype = ctypes.c_int
    lib.or_g_cfg1.argtypes = [i32, P, P, P, P, P, P]
    lib.or_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


@dataclass
class Mat:
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def n(self):
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self):
        return int(self.col.shape[0])


def _mat(m) -> Mat:
    return Mat(_c(m.rowptr, np.int32), _c(m.col, np.int32), _c(m.val, np.float64))


def spmv(A, x, threads: int = 1) -> np.ndarray:
    """y = A x, rows summed left to right (plain CSR definition)."""
    A = _mat(A)
    x = _c(x, np.float64)
    y = np.empty(A.n, np.float64)
    _load().or_spmv(A.n, _p(A.rowptr), _p(A.col), _p(A.val), _p(x), _p(y), threads)
    return y


def spmv_t(G, x, ncols: int | None = None) -> np.ndarray:
    """y = G^T x by scattering rows of G (definition of the transpose product)."""
    G = _mat(G)
    ncols = G.n if ncols is None else ncols
    x = _c(x, np.float64)
    y = np.empty(ncols, np.float64)
    _load().or_spmv_t(G.n, ncols, _p(G.rowptr), _p(G.col), _p(G.val), _p(x), _p(y))
    return y


def spmv_f32(rowptr, col, val32, x32) -> np.ndarray:
    """y = A x with FP32 values, vector and sums (FP32 storage path)."""
    rp, ci = _c(rowptr, np.int32), _c(col, np.int32)
    v, x = _c(val32, np.float32), _c(x32, np.float32)
    y = np.empty(rp.shape[0] - 1, np.float32)
    _load().or_spmv_f32(rp.shape[0] - 1, _p(rp), _p(ci), _p(v), _p(x), _p(y))
    return y


def spmv_t_f32(rowptr, col, val32, x32) -> np.ndarray:
    """y = G^T x with FP32 values, vector and sums, rows of G scattered in order."""
    rp, ci = _c(rowptr, np.int32), _c(col, np.int32)
    v, x = _c(val32, np.float32), _c(x32, np.float32)
    n = rp.shape[0] - 1
    y = np.empty(n, np.float32)
    _load().or_spmv_t_f32(n, n, _p(rp), _p(ci), _p(v), _p(x), _p(y))
    return y


def transpose(G, ncols: int | None = None) -> Mat:
    G = _mat(G)
    ncols = G.n if ncols is None else ncols
    trp = np.empty(ncols + 1, np.int32)
    tci = np.empty(G.nnz, np.int32)
    tv = np.empty(G.nnz, np.float64)
    _load().or_transpose(G.n, ncols, _p(G.rowptr), _p(G.col), _p(G.val), _p(trp), _p(tci), _p(tv))
    return Mat(trp, tci, tv)


def dot(a, b, threads: int = 1) -> float:
    """sum_i a_i b_i computed exactly and rounded once to the nearest double
    (ties to even), the same for every thread count."""
    a = _c(a, np.float64)
    b = _c(b, np.float64)
    return float(_load().or_dot_threads(a.shape[0], _p(a), _p(b), int(threads)))


def apply_precond(G, r, eps: float = 0.0) -> np.ndarray:
    """s = G (G^T r) + eps r  (Eq. "major": M^-1 = G G^T + eps I)."""
    G = _mat(G)
    r = _c(r, np.float64)
    s = np.empty(G.n, np.float64)
    _load().or_apply_precond(G.n, _p(G.rowptr), _p(G.col), _p(G.val), float(eps), _p(r), _p(s))
    return s


@dataclass
class PCGResult:
    x: np.ndarray
    status: int
    iters: int
    restarts: int
    relres_rec: float
    relres_true: float
    rhist: np.ndarray | None = None
    xhist: np.ndarray | None = None


def pcg(A, G, b, x0=None, *, eps: float = 0.0, tol: float = 1e-8, maxit: int = 2000, rr_period: int = 50,
        delta_form: int = 0, stop_rule: int = 0, threads: int = 1, history: bool = False,
        x_history: bool = False) -> PCGResult:
    """Preconditioned CG, Algorithm 1 (Appendix A) with M^-1 = G G^T + eps I."""
    A = _mat(A)
    G = _mat(G)
    b = _c(b, np.float64)
    n = A.n
    x = np.zeros(n, np.float64) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    opts = _Opts(float(eps), float(tol), int(maxit), int(rr_period), int(delta_form), int(stop_rule), int(threads))
    res = _Res()
    rh = np.full(maxit + 1, np.nan) if history else None
    xh = np.full((maxit + 1, n), np.nan) if x_history else None
    _load().or_pcg(n, _p(A.rowptr), _p(A.col), _p(A.val), _p(G.rowptr), _p(G.col), _p(G.val), _p(b), _p(x),
                   ctypes.byref(opts), ctypes.byref(res), _p(rh), _p(xh))
    k = res.iters
    return PCGResult(x, res.status, k, res.restarts, res.relres_rec, res.relres_true,
                     None if rh is None else rh[: k + 1], None if xh is None else xh[: k + 1])


def tril_nnz(A) -> int:
    A = _mat(A)
    return int(_load().or_tril_nnz(A.n, _p(A.rowptr), _p(A.col)))


def fsai_lower(A, threads: int | None = None) -> Mat:
    """Classic FSAI G_L on tril(A)'s pattern (A^-1 ~ G_L^T G_L). Rows are
    independent; the thread count (default: all available) does not change
    the result."""
    A = _mat(A)
    m = tril_nnz(A)
    grp = np.empty(A.n + 1, np.int32)
    gci = np.empty(m, np.int32)
    gv = np.empty(m, np.float64)
    th = max_threads() if threads is None else int(threads)
    rc = _load().or_fsai_lower(A.n, _p(A.rowptr), _p(A.col), _p(A.val), _p(grp), _p(gci), _p(gv), th)
    if rc != OK:
        raise ValueError(f"or_fsai_lower failed with {rc}")
    return Mat(grp, gci, gv)


def fsai_g(A, threads: int | None = None) -> Mat:
    """G = G_L^T, so that M^-1 = G G^T = G_L^T G_L ~ A^-1."""
    return transpose(fsai_lower(A, threads))


def fsai_block_lower(A, b: int = 3, threads: int | None = None) -> Mat:
    """Block FSAI G_L (b x b blocks, block-lower on tril(A)'s block pattern,
    every block full) for an exactly b x b blocked A; A^-1 ~ G_L^T G_L."""
    A = _mat(A)
    grp = np.empty(A.n + 1, np.int32)
    m = int(_load().or_bfsai_pattern(A.n, _p(A.rowptr), _p(A.col), int(b), _p(grp)))
    if m < 0:
        raise ValueError("block FSAI needs an exactly b x b blocked matrix")
    gci = np.empty(m, np.int32)
    gv = np.empty(m, np.float64)
    th = max_threads() if threads is None else int(threads)
    rc = _load().or_fsai_block_lower(A.n, _p(A.rowptr), _p(A.col), _p(A.val), int(b), _p(grp), _p(gci), _p(gv), th)
    if rc != OK:
        raise ValueError(f"or_fsai_block_lower failed with {rc}")
    return Mat(grp, gci, gv)


def fsai_block_g(A, b: int = 3, threads: int | None = None) -> Mat:
    """G = G_L^T of the block FSAI, so that M^-1 = G G^T = G_L^T G_L."""
    return transpose(fsai_block_lower(A, b, threads))


def g_cfg1(A) -> Mat:
    A = _mat(A)
    m = tril_nnz(A)
    grp = np.empty(A.n + 1, np.int32)
    gci = np.empty(m, np.int32)
    gv = np.empty(m, np.float64)
    rc = _load().or_g_cfg1(A.n, _p(A.rowptr), _p(A.col), _p(A.val), _p(grp), _p(gci), _p(gv))
    if rc != OK:
        raise ValueError(f"or_g_cfg1 failed with {rc}")
    return Mat(grp, gci, gv)


def seeded_g(A, seed: int) -> Mat:
    """Seeded G on A's full pattern, a stand-in for a learned G of that shape
    (Sec. 3.2.2: the learned G keeps A's sparsity): G_ii = 1/sqrt(A_ii); for
    j != i, G_ij = 0.25 u_ij |A_ij| / sqrt(A_ii A_jj), u_ij = 2U - 1 with U the
    draw at index i*n + j of the preconditioner stream (taken from the shared
    input generator, which holds none of the method's arithmetic)."""
    from paper_2510_27517_amd import inputs

    A = _mat(A)
    n = A.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.rowptr))
    cols = A.col.astype(np.int64)
    diag = np.zeros(n)
    on = rows == cols
    diag[rows[on]] = A.val[on]
    if not np.all(diag > 0):
        raise ValueError("seeded_g needs a positive stored diagonal")
    u = 2.0 * inputs.u01_at(seed, inputs.STREAM_G, rows * n + cols) - 1.0
    val = 0.25 * u * np.abs(A.val) / np.sqrt(diag[rows] * diag[cols])
    val[on] = 1.0 / np.sqrt(diag[rows[on]])
    return Mat(A.rowptr.copy(), A.col.copy(), val)


def mean_norm(A) -> float:
    """||A|| of the SAI loss (Sec. 3.3): the mean of |A_ij| over the nonzero
    entries."""
    A = _mat(A)
    v = np.abs(A.val[A.val != 0.0])
    return float(np.mean(v)) if v.size else 1.0


def eps_shift(A, rel: float = 1e-4) -> float:
    """Absolute shift of M^-1 = G G^T + eps I for a G normalised to A's scale:
    the paper's relative shift (1e-4, Sec. 3.2.1) over the mean |A_ij|."""
    return rel / mean_norm(A)


def sai_losses(A, G, W, eps: float = 0.0):
    """Per-probe losses of Sec. 3.3 and its loss ablation, probe by probe:
    y = A M^-1 w with M^-1 = G G^T + eps I (Eq. "major"),
      sai = ||y / ||A|| - w||^2  (Eq. "our-loss"),  l2 = ||y - w||^2,
      cs  = w^T y / (||w|| ||y||).
    W is n x k (one probe per column). Their means over i.i.d. N(0,1) probes
    estimate the squared Frobenius norms of Eq. "loss-initial"."""
    W = np.asarray(W, dtype=np.float64)
    na = mean_norm(A)
    out = {"sai": np.zeros(W.shape[1]), "l2": np.zeros(W.shape[1]), "cs": np.zeros(W.shape[1])}
    for p in range(W.shape[1]):
        w = np.ascontiguousarray(W[:, p])
        y = spmv(A, apply_precond(G, w, eps))
        out["sai"][p] = float(np.sum((y / na - w) ** 2))
        out["l2"][p] = float(np.sum((y - w) ** 2))
        out["cs"][p] = float(np.dot(w, y) / (np.linalg.norm(w) * np.linalg.norm(y)))
    return out


# ------------------------------------------- mixed precision (FP64 emulation)

# (significand bits p, exponent of the smallest normal, largest finite value)
# of the storage formats: IEEE binary32, bfloat16 and IEEE binary16
_FORMATS = {
    "f32": (24, -126, (2.0 - 2.0 ** -23) * 2.0 ** 127),
    "bf16": (8, -126, (2.0 - 2.0 ** -7) * 2.0 ** 127),
    "f16": (11, -14, 65504.0),
}


def round_storage(x, fmt: str) -> np.ndarray:
    """x rounded once, to nearest with ties to even, onto the storage format
    fmt ("f64" keeps x). A value in [2^(e-1), 2^e) has the quantum 2^(e-p);
    below the smallest normal 2^emin the quantum stays 2^(emin-p+1)
    (subnormals); a result above the largest finite value is infinite."""
    x = np.array(x, dtype=np.float64, copy=True)
    if fmt == "f64":
        return x
    p, emin, vmax = _FORMATS[fmt]
    _, e = np.frexp(x)
    q = np.maximum(e - p, emin - p + 1)
    y = np.ldexp(np.rint(np.ldexp(x, -q)), q)
    return np.where(np.abs(y) > vmax, np.copysign(np.inf, x), y)


def g_storage_scale(G, fmt: str) -> float:
    """Power-of-two scale under which G is stored (reading of the mixed-
    precision setup): 1, except for binary16, whose narrow exponent range
    takes G times 2^(14-e), max |G| = m 2^e with m in [1/2, 1), so that the
    largest stored entry lies in [2^13, 2^14). PCG is invariant to the scale
    of M^-1 when eps is scaled alike (Algorithm 1: alpha and x are unchanged,
    delta and beta scale together)."""
    if fmt != "f16":
        return 1.0
    m = float(np.abs(_mat(G).val).max())
    if m == 0.0:
        return 1.0
    _, e = np.frexp(m)
    return float(2.0 ** (14 - int(e)))


def inner_tolerance(inner_tol: float, tol: float, nb: float, rn: float, step: int = 1) -> float:
    """Relative tolerance of inner solve number `step` (0 first; reading of the
    mixed-precision setup): inner_tol, or what brings ||r64|| from rn to a
    quarter of the target tol ||b|| when that is looser (never looser than
    1/2); after the first step, also that target when it is down to
    inner_tol / 10 (the step that can finish)."""
    target = 0.25 * tol * nb / rn
    if target >= inner_tol or (step > 0 and target >= 0.1 * inner_tol):
        return min(0.5, target)
    return inner_tol


@dataclass
class IRResult:
    x: np.ndarray
    status: int
    outer: int
    iters: int          # inner iterations over all outer steps
    relres_true: float  # ||b - A x|| / ||b|| in FP64 at exit
    rhist: np.ndarray   # ||r64|| / ||b|| before each outer step and at exit


def pcg_ir(A, G, b, *, tol: float = 1e-10, a_dtype: str = "f32", g_dtype: str = "bf16", vec_dtype: str = "f32",
           eps: float = 0.0, inner_tol: float = 1e-6, max_outer: int = 30, maxit: int = 2000) -> IRResult:
    """FP64 iterative refinement around a PCG on stored operands (the mixed-
    precision setting of Sec. 4: G in a 16-bit format, A and vectors in FP32,
    FP64 dot products), as an FP64 emulation. Storage is emulated by rounding
    (round_storage) A's values, G's values (times g_storage_scale) and the
    vectors the inner solve receives and returns; the inner PCG itself runs
    in FP64 on those rounded operands. The outer loop:
      r = b - A x in FP64 on the unrounded A; stop with OK once
      ||r|| <= tol ||b||; stop with NOT_CONVERGED after max_outer steps or
      when ||r|| fails to fall below 0.9 times its previous value;
      inner PCG (Algorithm 1 with M^-1 = G G^T + eps I, no residual
      replacement, stopping on its recurrence residual) on A_s c = r / ||r||
      from c = 0 to inner_tolerance(...); x += ||r|| c.
    b = 0 returns x = 0 after no outer step; an inner breakdown ends the
    solve with EBREAKDOWN."""
    A = _mat(A)
    G = _mat(G)
    b = np.asarray(b, np.float64)
    n = A.n
    sc = g_storage_scale(G, g_dtype)
    As = Mat(A.rowptr, A.col, round_storage(A.val, a_dtype))
    Gs = Mat(G.rowptr, G.col, round_storage(G.val * sc, g_dtype))
    x = np.zeros(n)
    nb = float(np.sqrt(dot(b, b)))
    if nb == 0.0:
        return IRResult(x, OK, 0, 0, 0.0, np.zeros(1))
    outer, iters, prev, status = 0, 0, np.inf, NOT_CONVERGED
    hist = []
    while True:
        r = b - spmv(A, x)
        rn = float(np.sqrt(dot(r, r)))
        hist.append(rn / nb)
        if rn <= tol * nb:
            status = OK
            break
        if not np.isfinite(rn):
            status = EBREAKDOWN
            break
        if outer >= max_outer or rn > 0.9 * prev:
            break
        prev = rn
        rhs = round_storage(r / rn, vec_dtype)
        inner = pcg(As, Gs, rhs, eps=eps * sc * sc, tol=inner_tolerance(inner_tol, tol, nb, rn, outer), maxit=maxit,
                    rr_period=0, delta_form=1, stop_rule=2)
        iters += inner.iters
        if inner.status == EBREAKDOWN:
            status = EBREAKDOWN
            break
        x = x + rn * round_storage(inner.x, vec_dtype)
        outer += 1
    return IRResult(x, status, outer, iters, hist[-1], np.array(hist))


def identity(n: int) -> Mat:
    return Mat(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))


def diag_inv_sqrt(A) -> Mat:
    """G = D^-1/2 (Jacobi: M^-1 = D^-1), D the stored diagonal of A. Pinned
    to 1/2 on constant 2D Poisson (A_ii = 4) and to the dense diagonal of a
    variable-coefficient matrix."""
    A = _mat(A)
    d = np.zeros(A.n)
    for i in range(A.n):
        for k in range(A.rowptr[i], A.rowptr[i + 1]):
            if A.col[k] == i:
                d[i] = A.val[k]
    return Mat(np.arange(A.n + 1, dtype=np.int32), np.arange(A.n, dtype=np.int32), 1.0 / np.sqrt(d))


def max_threads() -> int:
    return int(_load().or_max_threads())
