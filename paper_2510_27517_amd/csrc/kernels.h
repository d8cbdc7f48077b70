// Internal interface between the library driver (pcg.cpp) and the gfx950
// kernels (kernels.hip). Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime_api.h>
#include <cstdint>

namespace pcgk {

// Element storage types of a matrix or vector on the device.
enum Dtype : int { F64 = 0, F32 = 1, BF16 = 2, F16 = 3 };

inline size_t dtype_size(int dt) { return dt == F64 ? 8 : dt == F32 ? 4 : 2; }

// Device-resident solver scalars. Kernels read them at launch and the last
// workgroup of each reducing kernel writes them, so no host round trip is
// needed inside an iteration.
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
  uint32_t ctr[8];    // arrival counters of the last-workgroup reductions
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
// covers rows [blk[k], blk[k+1]), holding at most `lds_cap` nonzeros unless it
// is a single longer row.
struct DevCSR {
  int32_t n = 0;
  int64_t nnz = 0;
  int32_t *rp = nullptr, *ci = nullptr;
  void *val = nullptr;
  int dtype = F64;
  int32_t *blk = nullptr;  // nblk + 1 row starts
  int32_t nblk = 0;
  int32_t grid = 0;        // workgroups per launch (multiple of 8)
};

// Vector-kind launch geometry: which storage types one solver instance uses.
struct Types {
  int vec;  // F64 or F32 (accumulation type equals this)
  int a;    // F64 or F32
  int g;    // F64, F32, BF16 or F16
};

constexpr int kBlock = 256;        // threads per workgroup (4 waves of 64)
constexpr int kLdsBytes = 16384;   // LDS staging for row products per workgroup

inline int lds_cap(int vec_dtype) { return kLdsBytes / (int)dtype_size(vec_dtype); }

// ---- launchers (all asynchronous on `s`) ----------------------------------

// Iteration kernels. `v` holds the solver's vectors.
struct Vecs {
  void *x, *r0, *r1, *d0, *d1, *q, *t, *s, *b;
};

// r_slot = b - A (x [+ alpha d_i]);  slot = iter&1 (sel 0) or (iter+1)&1 (sel 1).
// with_d: add the pending alpha d_i; reduce: store ||r||^2 in st->true_rr;
// respect_done: return at once when st->done is set.
hipError_t launch_resid(const Types &ty, const DevCSR &A, const Vecs &v, State *st, double *partials,
                        int slot_sel, bool with_d, bool reduce, bool respect_done, hipStream_t s);

// A-kernel of iteration i: d_i = s + beta d_{i-1}; x += alpha_{i-1} d_{i-1};
// q = A d_i; gamma = d_i^T q; alpha_i = delta_i / gamma.
hipError_t launch_iter_A(const Types &ty, const DevCSR &A, const Vecs &v, State *st, double *partials,
                         hipStream_t s);

// G^T-kernel: mode 0 (update r_{i+1} = r_i - alpha q), 1 (r_{i+1} already
// replaced), 2 (start or restart: r_i given, no update, beta = 0).
// t = G^T r; rr, tt; delta; beta; convergence / maxit / breakdown; iter++.
hipError_t launch_iter_GT(const Types &ty, const DevCSR &GT, const Vecs &v, State *st, double *partials,
                          int mode, hipStream_t s);

// G-kernel: s = G t + eps r.
hipError_t launch_iter_G(const Types &ty, const DevCSR &G, const Vecs &v, State *st, bool has_eps, hipStream_t s);

// x += alpha d_{iter-1} (the pending update), then alpha = 0.
hipError_t launch_finalize(const Types &ty, int32_t n, const Vecs &v, State *st, hipStream_t s);

// ||b||^2, ||b||, tol*||b||; ZERO_B status when b = 0.
hipError_t launch_norm_b(const Types &ty, int32_t n, const Vecs &v, State *st, double *partials, hipStream_t s);

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

}  // namespace pcgk
