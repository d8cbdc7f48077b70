"""Python binding of the gfx950 PCG library (include/pcg.h).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels. Arrays may be numpy (host) or torch tensors on the GPU (device
pointers are passed straight through). Importing works anywhere; the first
call that needs the library raises if ``libpcg.so`` is missing, and creating
a solver raises if no GPU is usable. There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcg.so")

OK, PENDING, NOT_CONVERGED = 0, 1, 2
EINVAL, ESTATE, ENOMEM, EBREAKDOWN, EDEVICE = -1, -2, -3, -4, -5
F64, F32, BF16, F16 = 0, 1, 2, 3
G_FSAI, G_FIXED, G_JACOBI, G_IDENTITY, G_SEEDED, G_BFSAI = 1, 2, 3, 4, 5, 6
OP_A, OP_GT, OP_G, OP_MINV = 0, 1, 2, 3
LAYOUT_AUTO, LAYOUT_CSR, LAYOUT_SELL, LAYOUT_BSR3, LAYOUT_SDIA = 0, 1, 2, 3, 4
LAYOUTS = {"auto": LAYOUT_AUTO, "csr": LAYOUT_CSR, "sell": LAYOUT_SELL, "bsr3": LAYOUT_BSR3, "sdia": LAYOUT_SDIA}

DTYPES = {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16}

# every symbol include/pcg.h declares
EXPORTS = [
    "pcg_config_default", "pcg_create", "pcg_destroy", "pcg_set_matrix", "pcg_set_precond", "pcg_build_precond",
    "pcg_solve", "pcg_matvec", "pcg_sai_loss", "pcg_sai_loss_noalloc", "pcg_validate_csr", "pcg_g_nnz", "pcg_build_g_host", "pcg_bytes_per_iter",
    "pcg_last_error", "pcg_strerror", "pcg_time_kernels", "pcg_copy_bandwidth", "pcg_read_bandwidth",
    "pcg_submit_batch",
    "pcg_progress", "pcg_poll", "pcg_wait", "pcg_solve_batch", "pcg_pool_info", "pcg_estimate_bytes",
    "pcg_autotune", "pcg_batch_stats_get",
]


class Config(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("vec_dtype", ctypes.c_int),
        ("a_dtype", ctypes.c_int), ("g_dtype", ctypes.c_int), ("rr_period", ctypes.c_int),
        ("eps", ctypes.c_double), ("refine", ctypes.c_int), ("inner_tol", ctypes.c_double),
        ("max_outer", ctypes.c_int), ("graph_iters", ctypes.c_int), ("grid_mult", ctypes.c_int),
        ("mem_budget_mb", ctypes.c_int), ("layout", ctypes.c_int), ("g_device", ctypes.c_int),
        ("wide_index", ctypes.c_int), ("autotune", ctypes.c_int), ("cache_mb", ctypes.c_int),
        ("wg_max_n", ctypes.c_int), ("wg_max_n_batch", ctypes.c_int), ("rows_per_lane", ctypes.c_int),
        ("loads_in_flight", ctypes.c_int),
        ("alloc", ctypes.c_void_p), ("free", ctypes.c_void_p), ("alloc_user", ctypes.c_void_p),
    ]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class TorchAllocator:
    """Device allocator callbacks backed by PyTorch's caching allocator, for
    pcg_config.alloc / free (keeps the callback objects alive)."""

    def __init__(self, device: int = 0):
        import torch

        self.device = device
        self.live = {}

        def _alloc(nbytes, _user):
            try:
                p = int(torch.cuda.caching_allocator_alloc(int(nbytes), device))
            except Exception:
                return None
            self.live[p] = int(nbytes)
            return p

        def _free(ptr, _user):
            self.live.pop(int(ptr), None)
            torch.cuda.caching_allocator_delete(int(ptr))

        self.alloc_fn = ALLOC_FN(_alloc)
        self.free_fn = FREE_FN(_free)

    def install(self, cfg):
        cfg.alloc = ctypes.cast(self.alloc_fn, ctypes.c_void_p)
        cfg.free = ctypes.cast(self.free_fn, ctypes.c_void_p)
        return cfg


class TuneResult(ctypes.Structure):
    _fields_ = [
        ("layout_a", ctypes.c_int), ("layout_g", ctypes.c_int), ("grid_mult", ctypes.c_int),
        ("candidates", ctypes.c_int), ("fmt_a", ctypes.c_int), ("fmt_g", ctypes.c_int), ("fmt_gt", ctypes.c_int),
        ("idx16", ctypes.c_int), ("temporal", ctypes.c_int), ("rows_per_lane_gt", ctypes.c_int),
        ("loads_in_flight_a", ctypes.c_int), ("ms_per_iter", ctypes.c_double),
        ("ms_per_iter_auto", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchStats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64), ("step_ms", ctypes.c_double), ("step_bytes", ctypes.c_double),
        ("wg_launches", ctypes.c_int64), ("wg_ms", ctypes.c_double), ("wg_bytes", ctypes.c_double),
        ("host_prep_ms", ctypes.c_double), ("host_admit_ms", ctypes.c_double), ("host_step_ms", ctypes.c_double),
        ("host_retire_ms", ctypes.c_double), ("host_progress_ms", ctypes.c_double), ("host_idle_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("iters", ctypes.c_int), ("outer_iters", ctypes.c_int),
        ("restarts", ctypes.c_int), ("relres_true", ctypes.c_double), ("relres_rec", ctypes.c_double),
        ("t_solve_ms", ctypes.c_double), ("bytes_per_iter", ctypes.c_double),
        ("t_latency_ms", ctypes.c_double), ("t_queue_ms", ctypes.c_double),
        ("escalated", ctypes.c_int), ("reserved_", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class System(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("nnz_a", ctypes.c_int64), ("a_rowptr", ctypes.c_void_p),
        ("a_col", ctypes.c_void_p), ("a_val", ctypes.c_void_p), ("nnz_g", ctypes.c_int64),
        ("g_rowptr", ctypes.c_void_p), ("g_col", ctypes.c_void_p), ("g_val", ctypes.c_void_p),
        ("g_kind", ctypes.c_int), ("g_seed", ctypes.c_uint64), ("b", ctypes.c_void_p), ("x", ctypes.c_void_p), ("tol", ctypes.c_double),
        ("maxit", ctypes.c_int),
    ]


_lib = None


def load():
    """Load libpcg.so (raises RuntimeError when it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, dbl, c_int = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.pcg_config_default.argtypes = [ctypes.POINTER(Config)]
    lib.pcg_config_default.restype = None
    lib.pcg_create.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(P)]
    lib.pcg_destroy.argtypes = [P]
    lib.pcg_destroy.restype = None
    lib.pcg_set_matrix.argtypes = [P, i32, i64, P, P, P, c_int]
    lib.pcg_set_precond.argtypes = [P, i32, i64, P, P, P, c_int]
    lib.pcg_build_precond.argtypes = [P, c_int, ctypes.c_uint64]
    lib.pcg_sai_loss.argtypes = [P, i32, P, c_int, P, P, P]
    lib.pcg_sai_loss_noalloc.argtypes = [P, i32, P, P, P, P]
    lib.pcg_solve.argtypes = [P, P, P, dbl, c_int, c_int, ctypes.POINTER(Result)]
    lib.pcg_matvec.argtypes = [P, c_int, P, P, c_int]
    lib.pcg_validate_csr.argtypes = [i32, i64, P, P, c_int]
    lib.pcg_g_nnz.argtypes = [c_int, i32, P, P]
    lib.pcg_g_nnz.restype = i64
    lib.pcg_build_g_host.argtypes = [c_int, ctypes.c_uint64, i32, P, P, P, P, P, P]
    lib.pcg_bytes_per_iter.argtypes = [i32, i64, i64, c_int, c_int, c_int]
    lib.pcg_bytes_per_iter.restype = dbl
    lib.pcg_time_kernels.argtypes = [P, c_int, P, P]
    lib.pcg_copy_bandwidth.argtypes = [c_int, i64, c_int, P, P]
    lib.pcg_read_bandwidth.argtypes = [c_int, i64, c_int, P, P]
    lib.pcg_submit_batch.argtypes = [P, c_int, ctypes.POINTER(System), ctypes.POINTER(ctypes.c_uint64)]
    lib.pcg_progress.argtypes = [P, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]
    lib.pcg_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Result)]
    lib.pcg_wait.argtypes = [P, c_int, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(Result), dbl]
    lib.pcg_estimate_bytes.argtypes = [ctypes.POINTER(Config), i32, i64, i64, ctypes.POINTER(ctypes.c_size_t)]
    lib.pcg_autotune.argtypes = [P, c_int, ctypes.POINTER(TuneResult)]
    lib.pcg_solve_batch.argtypes = [P, c_int, ctypes.POINTER(System), ctypes.POINTER(Result), c_int]
    lib.pcg_pool_info.argtypes = [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    lib.pcg_batch_stats_get.argtypes = [P, ctypes.POINTER(BatchStats), c_int]
    lib.pcg_last_error.argtypes = [P]
    lib.pcg_last_error.restype = ctypes.c_char_p
    lib.pcg_strerror.argtypes = [c_int]
    lib.pcg_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


class PCGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def default_config(**kw) -> Config:
    cfg = Config()
    load().pcg_config_default(ctypes.byref(cfg))
    for k, v in kw.items():
        if k in ("vec_dtype", "a_dtype", "g_dtype") and isinstance(v, str):
            v = DTYPES[v]
        if k == "layout" and isinstance(v, str):
            v = LAYOUTS[v]
        setattr(cfg, k, v)
    return cfg


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a):
    """(pointer, on_device) of a numpy array or a torch tensor."""
    if _is_torch(a):
        return a.data_ptr(), int(a.is_cuda)
    return a.ctypes.data, 0


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------- host-only

def validate_csr(rowptr, col, n=None, require_diag=True) -> int:
    rp = _host(rowptr, np.int32)
    ci = _host(col, np.int32)
    n = rp.shape[0] - 1 if n is None else n
    return int(load().pcg_validate_csr(n, ci.shape[0], rp.ctypes.data, ci.ctypes.data, int(require_diag)))


def build_g_host(kind: int, A, seed: int = 0):
    """G of `kind` from A, built by the library's host code: (rowptr, col, val)."""
    lib = load()
    rp, ci, v = _host(A.rowptr, np.int32), _host(A.col, np.int32), _host(A.val, np.float64)
    n = rp.shape[0] - 1
    m = int(lib.pcg_g_nnz(kind, n, rp.ctypes.data, ci.ctypes.data))
    if m < 0:
        raise PCGError(EINVAL, "pcg_g_nnz")
    grp = np.empty(n + 1, np.int32)
    gci = np.empty(m, np.int32)
    gv = np.empty(m, np.float64)
    st = lib.pcg_build_g_host(kind, int(seed), n, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, grp.ctypes.data,
                              gci.ctypes.data, gv.ctypes.data)
    if st != OK:
        raise PCGError(st, "pcg_build_g_host")
    return grp, gci, gv


def copy_bandwidth(bytes_: int, reps: int = 20, device: int = 0):
    """(GB/s, ms per copy) of the library's device copy kernel."""
    g = np.zeros(1)
    m = np.zeros(1)
    st = load().pcg_copy_bandwidth(device, int(bytes_), int(reps), g.ctypes.data, m.ctypes.data)
    if st != OK:
        raise PCGError(st, "pcg_copy_bandwidth")
    return float(g[0]), float(m[0])


def read_bandwidth(bytes_: int, reps: int = 20, device: int = 0):
    """(GB/s, ms per read) of the library's read-only stream kernel."""
    g = np.zeros(1)
    m = np.zeros(1)
    st = load().pcg_read_bandwidth(device, int(bytes_), int(reps), g.ctypes.data, m.ctypes.data)
    if st != OK:
        raise PCGError(st, "pcg_read_bandwidth")
    return float(g[0]), float(m[0])


def estimate_bytes(cfg: Config, n: int, nnz_a: int, nnz_g: int) -> int:
    """Upper estimate of the device bytes one system takes under cfg."""
    out = ctypes.c_size_t()
    st = load().pcg_estimate_bytes(ctypes.byref(cfg), int(n), int(nnz_a), int(nnz_g), ctypes.byref(out))
    if st != OK:
        raise PCGError(st, "pcg_estimate_bytes")
    return int(out.value)


def bytes_per_iter(n, nnz_a, nnz_g, a_dtype=F64, g_dtype=F64, vec_dtype=F64) -> float:
    return float(load().pcg_bytes_per_iter(n, nnz_a, nnz_g, a_dtype, g_dtype, vec_dtype))


# ------------------------------------------------------------------ solver

@dataclass
class SolveOut:
    x: object
    status: int
    iters: int
    outer_iters: int
    restarts: int
    relres_true: float
    relres_rec: float
    t_solve_ms: float
    bytes_per_iter: float
    escalated: int = 0


class Solver:
    """One library context (one device, one stream)."""

    def __init__(self, config: Config | None = None, *, allocator=None, **kw):
        """allocator: None (hipMalloc), "torch" (PyTorch's caching allocator) or
        an object with install(cfg) such as TorchAllocator."""
        self._lib = load()
        self.cfg = config if config is not None else default_config(**kw)
        if allocator == "torch":
            allocator = TorchAllocator(self.cfg.device)
        self.allocator = allocator
        if allocator is not None:
            allocator.install(self.cfg)
        h = ctypes.c_void_p()
        st = self._lib.pcg_create(ctypes.byref(self.cfg), ctypes.byref(h))
        if st != OK:
            raise PCGError(st, "pcg_create: " + self._lib.pcg_strerror(st).decode())
        self._h = h
        self.n = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st, what, allow=(OK,)):
        if st not in allow:
            msg = self._lib.pcg_last_error(self._h).decode() or self._lib.pcg_strerror(st).decode()
            raise PCGError(st, msg if msg.startswith(what + ":") else f"{what}: {msg}")
        return st

    def _csr_args(self, rowptr, col, val):
        if _is_torch(rowptr):
            n = rowptr.shape[0] - 1
            return n, col.shape[0], rowptr.data_ptr(), col.data_ptr(), val.data_ptr(), int(rowptr.is_cuda), None
        rp, ci, v = _host(rowptr, np.int32), _host(col, np.int32), _host(val, np.float64)
        keep = (rp, ci, v)
        return rp.shape[0] - 1, ci.shape[0], rp.ctypes.data, ci.ctypes.data, v.ctypes.data, 0, keep

    def set_matrix(self, A=None, *, rowptr=None, col=None, val=None):
        if A is not None:
            rowptr, col, val = A.rowptr, A.col, A.val
        n, nnz, prp, pci, pv, dev, _keep = self._csr_args(rowptr, col, val)
        self._check(self._lib.pcg_set_matrix(self._h, n, nnz, prp, pci, pv, dev), "pcg_set_matrix")
        self.n = n

    def set_precond(self, G=None, *, rowptr=None, col=None, val=None):
        if G is not None:
            rowptr, col, val = G.rowptr, G.col, G.val
        n, nnz, prp, pci, pv, dev, _keep = self._csr_args(rowptr, col, val)
        self._check(self._lib.pcg_set_precond(self._h, n, nnz, prp, pci, pv, dev), "pcg_set_precond")

    def build_precond(self, kind: int = G_FSAI, seed: int = 0):
        self._check(self._lib.pcg_build_precond(self._h, kind, int(seed)), "pcg_build_precond")

    def solve(self, b, x0=None, *, tol=1e-8, maxit=2000, allow_failure=False) -> SolveOut:
        """Solve A x = b; returns the solution (same kind of array as b)."""
        if _is_torch(b):
            import torch

            x = torch.zeros_like(b, dtype=torch.float64) if x0 is None else x0.to(torch.float64).clone()
            bb = b.to(torch.float64).contiguous()
        else:
            bb = _host(b, np.float64)
            x = np.zeros(bb.shape[0]) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        pb, dev = _ptr(bb)
        px, _ = _ptr(x)
        res = Result()
        st = self._lib.pcg_solve(self._h, pb, px, float(tol), int(maxit), dev, ctypes.byref(res))
        allow = (OK, NOT_CONVERGED, EBREAKDOWN) if allow_failure else (OK, NOT_CONVERGED)
        self._check(st, "pcg_solve", allow)
        return SolveOut(x, res.status, res.iters, res.outer_iters, res.restarts, res.relres_true, res.relres_rec,
                        res.t_solve_ms, res.bytes_per_iter, res.escalated)

    def sai_loss(self, W):
        """Per-probe SAI, L2 and cosine-similarity losses of the stored A and
        M^-1 = G G^T + eps I for probes W (n x k; numpy or torch, FP64)."""
        if _is_torch(W):
            Wc = W.to(dtype=__import__("torch").float64).contiguous()
        else:
            Wc = np.ascontiguousarray(W, dtype=np.float64)
        if Wc.ndim != 2:
            raise PCGError(EINVAL, "sai_loss: W must be n x k")
        k = int(Wc.shape[1])
        pw, dev = _ptr(Wc)
        out = {name: np.zeros(k) for name in ("sai", "l2", "cs")}
        self._check(self._lib.pcg_sai_loss(self._h, k, pw, dev, out["sai"].ctypes.data, out["l2"].ctypes.data,
                                           out["cs"].ctypes.data), "pcg_sai_loss")
        return out

    def sai_loss_noalloc(self, W):
        """sai_loss with the library's static device scratch (no device
        allocation); W must be a contiguous FP64 n x k tensor on the GPU."""
        if not _is_torch(W) or not W.is_cuda or W.dtype != __import__("torch").float64 or W.ndim != 2 \
                or not W.is_contiguous():
            raise PCGError(EINVAL, "sai_loss_noalloc: W must be a contiguous float64 n x k GPU tensor")
        k = int(W.shape[1])
        out = {name: np.zeros(k) for name in ("sai", "l2", "cs")}
        self._check(self._lib.pcg_sai_loss_noalloc(self._h, k, W.data_ptr(), out["sai"].ctypes.data,
                                                   out["l2"].ctypes.data, out["cs"].ctypes.data),
                    "pcg_sai_loss_noalloc")
        return out

    def autotune(self, iters: int = 20):
        """Time the candidate layouts and grids of the set A and G and keep the
        fastest (see pcg_autotune); returns the choice as a dict."""
        out = TuneResult()
        self._check(self._lib.pcg_autotune(self._h, int(iters), ctypes.byref(out)), "pcg_autotune")
        return out.as_dict()

    def time_kernels(self, iters: int = 50):
        """{'ms': [A, GT, G, iteration], 'bytes': [A, GT, G, iteration]} per launch."""
        ms = np.zeros(4)
        by = np.zeros(4)
        self._check(self._lib.pcg_time_kernels(self._h, int(iters), ms.ctypes.data, by.ctypes.data),
                    "pcg_time_kernels")
        return {"ms": ms.tolist(), "bytes": by.tolist()}

    # ------------------------------------------------------- batch / serving

    def _system(self, A, b, x0=None, G=None, g_kind=G_FSAI, g_seed=0, tol=1e-8, maxit=2000):
        keep = [_host(A.rowptr, np.int32), _host(A.col, np.int32), _host(A.val, np.float64),
                _host(b, np.float64)]
        x = np.zeros(keep[0].shape[0] - 1) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        keep.append(x)
        sysd = System()
        sysd.n = keep[0].shape[0] - 1
        sysd.nnz_a = keep[1].shape[0]
        sysd.a_rowptr, sysd.a_col, sysd.a_val = keep[0].ctypes.data, keep[1].ctypes.data, keep[2].ctypes.data
        if G is not None:
            g = [_host(G.rowptr, np.int32), _host(G.col, np.int32), _host(G.val, np.float64)]
            keep += g
            sysd.nnz_g = g[1].shape[0]
            sysd.g_rowptr, sysd.g_col, sysd.g_val = g[0].ctypes.data, g[1].ctypes.data, g[2].ctypes.data
        sysd.g_kind = g_kind
        sysd.g_seed = int(g_seed)
        sysd.b = keep[3].ctypes.data
        sysd.x = x.ctypes.data
        sysd.tol = float(tol)
        sysd.maxit = int(maxit)
        return sysd, keep, x

    def submit(self, systems):
        """Queue systems (dicts with A, b and optional x0, G, g_kind, g_seed, tol,
        maxit); returns their tickets. Inputs are copied by the library; the
        solution arrays stay owned here until the ticket finishes."""
        if not hasattr(self, "_pending"):
            self._pending = {}
        built = [self._system(**sd) for sd in systems]
        arr = (System * len(built))(*[b[0] for b in built])
        tk = (ctypes.c_uint64 * len(built))()
        self._check(self._lib.pcg_submit_batch(self._h, len(built), arr, tk), "pcg_submit_batch")
        for i, b in enumerate(built):
            self._pending[int(tk[i])] = (b[1], b[2])
        return [int(t) for t in tk]

    def progress(self, iters=20):
        """One scheduler step; returns (active, queued)."""
        a, q = ctypes.c_int(), ctypes.c_int()
        self._check(self._lib.pcg_progress(self._h, int(iters), ctypes.byref(a), ctypes.byref(q)), "pcg_progress")
        return a.value, q.value

    def poll(self, ticket):
        """None while pending, else (x, result dict)."""
        res = Result()
        st = self._lib.pcg_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(res))
        if st == PENDING:
            return None
        if st == EINVAL and ticket not in self._pending:
            raise PCGError(st, "pcg_poll: unknown ticket")
        _keep, x = self._pending.pop(ticket)
        return x, res.as_dict()

    def wait(self, tickets, timeout_s=-1.0):
        """Block until all tickets finish: [(x, result dict)] in ticket order,
        or None when timeout_s (seconds, < 0: no limit) runs out first."""
        tickets = [int(t) for t in tickets]
        for t in tickets:
            if t not in getattr(self, "_pending", {}):
                raise PCGError(EINVAL, "wait: unknown ticket")
        tk = (ctypes.c_uint64 * len(tickets))(*tickets)
        res = (Result * len(tickets))()
        st = self._lib.pcg_wait(self._h, len(tickets), tk, res, float(timeout_s))
        if st == PENDING:
            return None
        self._check(st, "pcg_wait")
        out = [(self._pending[t][1], res[i].as_dict()) for i, t in enumerate(tickets)]
        for t in set(tickets):
            del self._pending[t]
        return out

    def solve_batch(self, systems, iters_per_step=20):
        """Solve all systems as one batch; returns [(x, result dict)]."""
        built = [self._system(**sd) for sd in systems]
        arr = (System * len(built))(*[b[0] for b in built])
        res = (Result * len(built))()
        self._check(self._lib.pcg_solve_batch(self._h, len(built), arr, res, int(iters_per_step)), "pcg_solve_batch")
        return [(b[2], res[i].as_dict()) for i, b in enumerate(built)]

    def batch_stats(self, reset: bool = False):
        """Device time and bytes of the batching scheduler's work (see
        pcg_batch_stats_get); reset zeroes the counters after reading."""
        out = BatchStats()
        self._check(self._lib.pcg_batch_stats_get(self._h, ctypes.byref(out), int(reset)), "pcg_batch_stats_get")
        return out.as_dict()

    def pool_info(self):
        cap, used = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(self._lib.pcg_pool_info(self._h, ctypes.byref(cap), ctypes.byref(used)), "pcg_pool_info")
        return cap.value, used.value

    def matvec(self, op: int, x):
        if _is_torch(x):
            import torch

            xx = x.to(torch.float64).contiguous()
            y = torch.empty_like(xx)
        else:
            xx = _host(x, np.float64)
            y = np.empty_like(xx)
        px, dev = _ptr(xx)
        py, _ = _ptr(y)
        self._check(self._lib.pcg_matvec(self._h, op, px, py, dev), "pcg_matvec")
        return y
