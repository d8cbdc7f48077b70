// Internal interface between the library driver (pcg.cpp) and the gfx950
// kernels (kernels.hip). Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime_api.h>
#include <cstdint>

namespace pcgk {

// Element storage types of a matrix or vector on the device.
enum Dtype : int { F64 = 0, F32 = 1, BF16 = 2, F16 = 3 };

inline size_t dtype_size(int dt) { return dt == F64 ? 8 : dt == F32 ? 4 : 2; }

// Device-resident solver scalars, kept in two slots: st[0] is written by the
// G-kernel (and by the host and single-workgroup helper kernels), st[1] by
// the G^T-kernel. A kernel never reads a slot it writes, so the workgroup that
// publishes new scalars cannot race the others reading the old ones. No
// host round trip is needed inside an iteration.
struct alignas(64) State {
  double delta;    // delta_i = r_i^T M^-1 r_i
  double alpha;    // alpha_i, pending in x until the next A-kernel applies it
  double beta;     // beta_{i+1}, used by the next A-kernel to form d
  double gamma;    // d_i^T A d_i
  double rr;       // ||r||^2 of the current residual
  double tt;       // ||G^T r||^2
  double tol_nb;   // tol * ||b||
  double eps;      // shift of M^-1 = G G^T + eps I
  double true_rr;  // ||b - A x||^2 from the last true-residual kernel
  double bb;       // ||b||^2
  double tol;
  double pad0;
  int32_t iter;       // completed iterations i
  int32_t maxit;
  int32_t status;     // Status below
  int32_t done;       // nonzero: every iteration kernel returns at once
  int32_t rr_period;  // residual replacement period (0 = off)
  int32_t pad1[3];
};

enum Status : int32_t {
  ST_RUNNING = 0,
  ST_CONV_REC = 1,     // recurrence residual met the tolerance (true residual still to confirm)
  ST_MAXIT = 2,
  ST_BREAK_GAMMA = 3,  // d^T A d <= 0 or not finite
  ST_BREAK_DELTA = 4,  // r^T M^-1 r < 0 or not finite
  ST_ZERO_B = 5,       // ||b|| = 0: x = 0
};

// A CSR matrix resident on the device, with its row-block partition: block k
// covers rows [blk[2k], blk[2k+2]) and nonzeros [blk[2k+1], blk[2k+3]),
// holding at most `lds_cap` nonzeros unless it is a single longer row.
struct DevCSR {
  int32_t n = 0;
  int64_t nnz = 0;
  int32_t *rp = nullptr, *ci = nullptr;
  void *val = nullptr;
  int dtype = F64;
  int32_t *blk = nullptr;  // nblk + 1 (row start, nonzero start) pairs
  int32_t nblk = 0;
  int32_t grid = 0;        // workgroups per launch (multiple of 8)
};

// Vector-kind launch geometry: which storage types one solver instance uses.
struct Types {
  int vec;  // F64 or F32 (accumulation type equals this)
  int a;    // F64 or F32
  int g;    // F64, F32, BF16 or F16
};

// Compile-time tuning of the CSR-stream kernels (defaults measured best on
// MI355X for 5-7 nonzeros per row).
#ifndef PCG_BLOCK_THREADS
#define PCG_BLOCK_THREADS 256
#endif
#ifndef PCG_LDS_BYTES
#define PCG_LDS_BYTES 16384
#endif
constexpr int kBlock = PCG_BLOCK_THREADS;  // threads per workgroup (waves of 64); also max rows per row block
constexpr int kLdsBytes = PCG_LDS_BYTES;   // LDS staging for row products per workgroup

inline int lds_cap(int vec_dtype) { return kLdsBytes / (int)dtype_size(vec_dtype); }

// ---- launchers (all asynchronous on `s`) ----------------------------------

// Iteration kernels. `v` holds the solver's vectors.
struct Vecs {
  void *x, *r0, *r1, *d0, *d1, *q, *t, *s, *b;
};

// Per-workgroup partial sums (one value per logical workgroup, value j of
// workgroup L at p[j * P + L]). Every workgroup of the consuming kernel adds
// them in the same fixed order, so each obtains the identical total without
// atomics or inter-workgroup synchronisation.
struct Partials {
  double *g;   // d^T A d          (written by the A-kernel)
  double *rt;  // ||r||^2, ||t||^2 (written by the G^T-kernel)
  double *b;   // ||b||^2
  double *tr;  // ||b - A x||^2
};

// r_slot = b - A (x [+ alpha d_i]);  slot = iter&1 (sel 0) or (iter+1)&1 (sel 1).
// with_d: add the pending alpha d_i; reduce: store ||r||^2 in st->true_rr;
// respect_done: return at once when st->done is set.
// with_d needs the A-kernel's partials (grid A.grid) to form alpha_i.
hipError_t launch_resid(const Types &ty, const DevCSR &A, const Vecs &v, State *st, const Partials &p,
                        int slot_sel, bool with_d, bool reduce, bool respect_done, hipStream_t s);

// A-kernel of iteration i: d_i = s + beta d_{i-1}; x += alpha_{i-1} d_{i-1};
// q = A d_i; gamma = d_i^T q; alpha_i = delta_i / gamma.
hipError_t launch_iter_A(const Types &ty, const DevCSR &A, const Vecs &v, State *st, const Partials &p,
                         hipStream_t s);

// G^T-kernel: mode 0 (update r_{i+1} = r_i - alpha q), 1 (r_{i+1} already
// replaced), 2 (start or restart: r_i given, no update, beta = 0).
// Reduces the A-kernel's partials (P_a workgroups) to gamma, alpha_i, or flags
// breakdown. t = G^T r; partials ||r||^2, ||t||^2. Publishes st[1].
hipError_t launch_iter_GT(const Types &ty, const DevCSR &GT, const Vecs &v, State *st, const Partials &p, int P_a,
                          int mode, hipStream_t s);

// G-kernel: reduces the G^T-kernel's partials (P_gt) to delta_{i+1},
// beta_{i+1}, the convergence / maxit / breakdown tests and iter; publishes
// st[0]; then s = G t + eps r unless stopped. `mode` as for the G^T-kernel.
hipError_t launch_iter_G(const Types &ty, const DevCSR &G, const Vecs &v, State *st, const Partials &p, int P_gt,
                         bool has_eps, int mode, hipStream_t s);

// x += alpha d_{iter-1} (the pending update), then alpha = 0.
hipError_t launch_finalize(const Types &ty, int32_t n, const Vecs &v, State *st, hipStream_t s);

// ||b||^2, ||b||, tol*||b|| into st[0]; ZERO_B status when b = 0.
hipError_t launch_norm_b(const Types &ty, int32_t n, const Vecs &v, State *st, const Partials &p, hipStream_t s);

// st[0].true_rr = sum of the true-residual partials (P workgroups).
hipError_t launch_reduce_true(State *st, const Partials &p, int P, hipStream_t s);

// Small state edits, ordered on the stream.
hipError_t launch_state_restart(State *st, hipStream_t s);  // done = 0, status = RUNNING, alpha = beta = 0

// y = op(x) for parity checks and the plain operator products: y = M x with M
// any stored CSR matrix (vector types = ty.vec).
hipError_t launch_spmv(const Types &ty, const DevCSR &M, int mdtype, const void *x, void *y, hipStream_t s);

// y = a*y + b*x (elementwise, vector type ty.vec).
hipError_t launch_axpby(int vec_dtype, int32_t n, double a, void *y, double b, const void *x, hipStream_t s);

// Conversions: dst[i] = (Tdst) (scale * src[i]).
hipError_t launch_convert(int src_dtype, const void *src, int dst_dtype, void *dst, int64_t n, double scale,
                          hipStream_t s);

hipError_t launch_fill(int dtype, void *p, int64_t n, double value, hipStream_t s);

// x64 += scale * (double) c  (iterative refinement update)
hipError_t launch_refine_update(int32_t n, double *x64, const void *c, int c_dtype, double scale, hipStream_t s);

// dst = src, `bytes` a multiple of 16.
hipError_t launch_copy(const void *src, void *dst, int64_t bytes, int grid, hipStream_t s);

}  // namespace pcgk
