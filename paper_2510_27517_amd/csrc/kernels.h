// Internal interface between the library driver (pcg.cpp) and the gfx950
// kernels (kernels.hip). Not part of the public C ABI.
//
// Every kernel works on a set of independent systems at once. A system is
// described by a SysDev record in a device-resident directory; a launch set
// lists the systems of one launch and, for each kind of kernel, maps every
// workgroup of the launch to (system, local workgroup). A system's share of a
// launch (its workgroup count, row blocks and reduction order) depends only
// on the system itself, so it computes bit for bit the same whether it is
// solved alone or inside any batch. A single-system solve is a set of one.
#pragma once
#include <hip/hip_runtime_api.h>
#include <cstdint>

namespace pcgk {

// Element storage types of a matrix or vector on the device.
enum Dtype : int { F64 = 0, F32 = 1, BF16 = 2, F16 = 3 };

inline size_t dtype_size(int dt) { return dt == F64 ? 8 : dt == F32 ? 4 : 2; }

// Device-resident solver scalars of one system, kept in two slots: st[0] is
// written by the G-kernel (and by the host and one-thread helper kernels),
// st[1] by the G^T-kernel. A kernel never reads a slot it writes, so the
// workgroup that publishes new scalars cannot race the others reading the
// old ones. No host round trip is needed inside an iteration.
struct alignas(64) State {
  double delta;    // delta_i = r_i^T M^-1 r_i
  double alpha;    // alpha_i (st[1], from the G^T-kernel); 0 in st[0] once the G-kernel applied it
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
  int32_t restarts;   // restarts from the true residual (one-workgroup solver)
  int32_t confirm;    // one-workgroup solver: confirm a converged recurrence on b - A x
  int32_t pad1;
};

enum Status : int32_t {
  ST_RUNNING = 0,
  ST_CONV_REC = 1,     // recurrence residual met the tolerance (true residual still to confirm)
  ST_MAXIT = 2,
  ST_BREAK_GAMMA = 3,  // d^T A d <= 0 or not finite
  ST_BREAK_DELTA = 4,  // r^T M^-1 r < 0 or not finite
  ST_ZERO_B = 5,       // ||b|| = 0: x = 0
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
// LDS the one-workgroup solver may take for a system's seven iteration
// vectors: in a launch of many systems (FP64 up to 512 rows, FP32 up to
// 1024), and for a single system (FP64 up to 2048 rows, FP32 up to 4096)
// where the device allows it beside the kernel's static LDS (below 20 KiB)
constexpr int kWgLdsVecBytes = 7 * 512 * 8;
constexpr int kWgLdsVecBytesOne = 7 * 2048 * 8;
constexpr int kWgStaticLdsBytes = 20480;

inline int lds_cap(int vec_dtype) { return kLdsBytes / (int)dtype_size(vec_dtype); }

// Storage layouts of a sparse matrix on the device.
enum Fmt : int32_t {
  FMT_CSR = 0,   // CSR with a row-block partition (any row lengths)
  FMT_SELL = 1,  // sliced ELL, slices of 64 rows (rows of similar length)
  FMT_BSR3 = 2,  // sliced 3x3 blocks, slices of 21 block rows (3x3-blocked matrices or block covers)
  FMT_SDIA = 3,  // sliced diagonals: slices of 64 rows, one column offset per slice entry (stencils)
};

// A sparse matrix resident on the device.
// FMT_CSR: rp/ci/val are CSR; block k covers rows [blk[2k], blk[2k+2]) and
//   nonzeros [blk[2k+1], blk[2k+3]), holding at most `lds_cap` nonzeros
//   unless it is a single longer row; nblk blocks.
// FMT_SELL: rp is unused; nblk slices of 64 rows; slice c has blk[c+1] -
//   blk[c] columns, entry k of row 64c + l at ci/val[(blk[c] + k) * 64 + l]
//   (rows keep their CSR order; padding has value 0 and a valid column).
// FMT_BSR3: rp is unused; nblk slices of 21 block rows (63 rows); slice c has
//   blk[c+1] - blk[c] blocks per block row; block k of block row 21c + r has
//   block column ci[(blk[c] + k) * 21 + r] and its row s, column j value at
//   val[((blk[c] + k) * 3 + j) * 63 + 21 s + r] for 8-byte values, at
//   val[9 ((blk[c] + k) * 21 + r) + 3 s + j] for 4- and 2-byte values
//   (padding: own block row, zeros; a block cover also holds explicit zeros).
// FMT_SDIA: rp is unused; nblk slices of 64 rows; slice c lists blk[c+1] -
//   blk[c] column offsets ci[blk[c] .. blk[c+1]) (ascending, column - row) and
//   holds the value of row 64c + l at offset k in val[(blk[c] + k) * 64 + l]
//   (0 where the row has no such entry; its column, clamped to [0, n), is
//   still gathered).
// `grid` is the system's workgroup count for products with this matrix (a
// multiple of 8, a function of nblk only). `nidx` counts the stored column
// indices (or offsets).
struct DevCSR {
  const int32_t *rp = nullptr, *ci = nullptr;
  const void *val = nullptr;
  const int32_t *blk = nullptr;
  int32_t nblk = 0;
  int32_t grid = 0;
  int64_t nnz = 0;
  int32_t n = 0;
  int32_t dtype = F64;
  int32_t fmt = FMT_CSR;
  int32_t idx16 = 0;     // FMT_SELL only: ci holds int16 column - row differences
  int32_t temporal = 0;  // 1: ordinary loads (kept in the memory-side cache); 0: nontemporal
  int64_t nidx = 0;
  int32_t rpl = 2;  // rows per lane over sliced diagonals where the kernel offers two (the G^T-kernel): 1 or 2
};

// Rows per slice of FMT_SELL; block rows per slice of FMT_BSR3.
constexpr int kSliceRows = 64;
constexpr int kBSliceRows = 21;

// Doubles per partial sum of an inner product (a double-double hi, lo).
constexpr int kAccWords = 2;

// One system in the directory (device-resident, POD). Partial sums: value j
// of a kernel with G workgroups keeps its workgroup L's hi at [2j G + L] and
// its lo at [(2j + 1) G + L].
struct SysDev {
  DevCSR A, GT, G;
  void *x, *r0, *r1, *d0, *d1, *q, *t, *s, *b;  // n entries of the vector type (s: FP64 views only)
  State *st;                                    // two slots
  double *pg;   // A.grid partials: d^T A d (kAccWords doubles each)
  double *prt;  // 2 * GT.grid partials: ||r||^2, ||t||^2
  double *pb;   // gB partials: ||b||^2
  double *ptr;  // A.grid partials: ||b - A x||^2
  int32_t n;
  int32_t gB;   // workgroups of the ||b|| kernel (multiple of 8)
};

// Storage types shared by all systems of a context.
struct Types {
  int vec;  // F64 or F32 (accumulation type equals this)
  int a;    // F64 or F32
  int g;    // F64, F32, BF16 or F16
};

// One launch over a set of systems. Workgroup w of an A-kind launch (A, resid,
// elementwise) works for system mapA[w].x as its local workgroup mapA[w].y;
// likewise mapGT, mapG, mapB. `set` lists the systems (for one-thread-per-
// system helpers). All arrays are device-resident.
struct LaunchSet {
  const SysDev *dir = nullptr;
  const int2 *mapA = nullptr, *mapGT = nullptr, *mapG = nullptr, *mapB = nullptr;
  const int32_t *set = nullptr;
  int32_t nA = 0, nGT = 0, nG = 0, nB = 0, nset = 0;  // workgroups of each kind, systems
  int32_t uw_a = 8;  // loads in flight per lane in the A-kernel's one-row sliced walks: 4 or 8
  // rows of the set's largest system whose seven iteration vectors fit in
  // the LDS cap with 8-byte and with 4-byte values (0: none): the
  // one-workgroup solver's dynamic LDS
  int32_t wg_lds_rows8 = 0, wg_lds_rows4 = 0;
};

// ---- launchers (all asynchronous on `s`) ----------------------------------

// r_slot = b - A (x [+ alpha_i d_i]), slot = iter&1 (sel 0) or (iter+1)&1
// (sel 1); sel 2: only for systems at a replacement iteration (i > 0,
// i % rr_period == 0), slot (iter+1)&1. with_d forms alpha_i from the A-kernel's partials; reduce writes
// ||r||^2 into st[0].true_rr; respect_done skips stopped systems.
hipError_t launch_resid(const Types &ty, const LaunchSet &L, int slot_sel, bool with_d, bool reduce,
                        bool respect_done, hipStream_t s);

// A-kernel of iteration i: q = A d_i; partials of d_i^T q.
// Optional events e0/e1 are attached to the dispatch itself (start and end
// of the kernel's execution), for timing.
hipError_t launch_iter_A(const Types &ty, const LaunchSet &L, hipStream_t s, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);

// G^T-kernel: mode 0 (r_{i+1} = r_i - alpha_i q), 1 (r_{i+1} already
// replaced), 2 (start or restart: r_i given, beta = 0), 3 (0 or 1 per system
// from its iteration count and replacement period). Forms gamma and
// alpha_i (or flags breakdown), t = G^T r, partials of ||r||^2 and ||t||^2;
// publishes st[1] (a copy of st[0] for a system that had already stopped).
hipError_t launch_iter_GT(const Types &ty, const LaunchSet &L, int mode, hipStream_t s, hipEvent_t e0 = nullptr,
                          hipEvent_t e1 = nullptr);

// G-kernel: delta_{i+1}, beta_{i+1}, convergence / maxit / breakdown, iter;
// publishes st[0]; then, unless stopped, d_{i+1} = (G t + eps r) + beta d_i
// (beta = 0 in mode 2), and x += alpha_i d_i (not in mode 2; also when the
// system stops at this iteration). Reads st[1] only.
hipError_t launch_iter_G(const Types &ty, const LaunchSet &L, bool has_eps, int mode, hipStream_t s,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Whole PCG solves, one workgroup per system of the set (persistent: the
// iteration loop, the residual replacement, the stopping test and, when
// st[0].confirm is set, the confirmation on b - A x with restarts all run in
// the kernel; no host round trip, no other launch). The states are set up as
// for the iteration kernels (tol, maxit, eps, rr_period, x holding x0); on
// return st[0] holds what the iteration kernels and the true-residual kernel
// would leave: iter, status, rr, tt, bb, tol_nb, true_rr, restarts, done = 1.
// Every row and every inner product is computed as by the iteration kernels
// (same row sums; exact inner products), so the results are theirs bit for
// bit. For small systems, where three launches per iteration dominate.
// Storage types it is built for: all FP64, or FP32 vectors and A with an
// FP32, BF16 or FP16 G (others: hipErrorInvalidValue).
bool solve_wg_supported(const Types &ty);
hipError_t launch_solve_wg(const Types &ty, const LaunchSet &L, bool has_eps, hipStream_t s);

// x += alpha d_{iter-1} if an update is still pending (alpha != 0), then
// alpha = 0. The G-kernel applies every update itself and leaves alpha = 0, so
// this only matters for states written by the host.
hipError_t launch_finalize(const Types &ty, const LaunchSet &L, hipStream_t s);

// ||b||^2, tol*||b|| into st[0]; ZERO_B status when b = 0.
hipError_t launch_norm_b(const Types &ty, const LaunchSet &L, hipStream_t s);

// Fill d0, d1 (and x when zero_x) of every system with zeros.
hipError_t launch_zero_dirs(const Types &ty, const LaunchSet &L, bool zero_x, hipStream_t s);

// Refinement over FP64 views (see k_outer): what 0: x64 += rn x_inner;
// what 1: b_inner = r64 / rn, with rn = sqrt(st[0].true_rr) of each view.
hipError_t launch_outer(int vec_dtype, const LaunchSet &L64, int what, hipStream_t s);

// done = 0, status = RUNNING, alpha = beta = 0 for every system of the set.
hipError_t launch_state_restart(const LaunchSet &L, hipStream_t s);

// y = M x for one stored matrix (plain product, vector type ty.vec).
hipError_t launch_spmv(const Types &ty, const DevCSR &M, const void *x, void *y, hipStream_t s);

// y = a*y + b*x (elementwise, vector type).
hipError_t launch_axpby(int vec_dtype, int32_t n, double a, void *y, double b, const void *x, hipStream_t s);

// Conversions: dst[i] = (Tdst) (scale * src[i]).
hipError_t launch_convert(int src_dtype, const void *src, int dst_dtype, void *dst, int64_t n, double scale,
                          hipStream_t s);

hipError_t launch_fill(int dtype, void *p, int64_t n, double value, hipStream_t s);

// x64 += scale * (double) c  (iterative refinement update)
hipError_t launch_refine_update(int32_t n, double *x64, const void *c, int c_dtype, double scale, hipStream_t s);

// ---- FSAI construction on the device (classic FSAI on tril(A), G = G_L^T)
//
// A in CSR with FP64 values; dpos[i] = position of row i's diagonal; lrp =
// row pointers of tril(A), the pattern of G_L. One wave per row i gathers
// A[J,J] (J = tril pattern of row i) into LDS, factors it A[J,J] = L L^T and
// writes row i of G_L = L^-T e_last into lv[lrp[i]..], with the arithmetic
// of the host builder in the same order. err[0] = 1 on a non-positive pivot.
// mmax (the longest tril row) sizes the LDS: at most kFsaiMaxRow.
constexpr int kFsaiMaxRow = 80;
hipError_t launch_fsai_rows(const int32_t *rp, const int32_t *ci, const double *v, const int32_t *dpos,
                            const int32_t *lrp, int32_t n, int32_t mmax, double *lv, int32_t *err, int grid,
                            hipStream_t s);

// part[b] = max |x[k]| over workgroup b's share (grid = 1024 workgroups).
hipError_t launch_absmax(const double *x, int64_t m, double *part, hipStream_t s);
constexpr int kAbsmaxGrid = 1024;

// Writes G_L (times scale, rounded to the storage type) into GT's storage and
// G_L^T into G's storage, each in its layout. G's row j holds the entries of
// A's row j from its diagonal on (A structurally symmetric); err[0] = 2 when
// an entry has no counterpart there.
hipError_t launch_fsai_place(const int32_t *rp, const int32_t *ci, const int32_t *dpos, const int32_t *lrp,
                             const double *lv, int32_t n, double scale, const DevCSR &GT, const DevCSR &G,
                             int32_t *err, hipStream_t s);

// ---- multi-probe products for the SAI loss (FP64 probes, n x k row-major)
//
// Y = c * (M X) + d * Z for a stored matrix M (either layout, any storage
// type; Z may be null): one wave per row, lane p for probes p, p+64, ...;
// each row summed left to right in CSR order.
hipError_t launch_spmm(const DevCSR &M, int32_t k, const double *X, double c, const double *Z, double d, double *Y,
                       hipStream_t s);

// Per-probe partial sums over rows for the losses: part[(b*5 + q)*k + p] for
// workgroup b < kLossGrid and q = 0..4: sum (y/na - w)^2, sum (y - w)^2,
// sum w y, sum y^2, sum w^2 (probe p's columns of Y and W).
constexpr int kLossGrid = 512;
hipError_t launch_loss_partials(int32_t n, int32_t k, const double *W, const double *Y, double na, double *part,
                                hipStream_t s);

// dst = src, `bytes` a multiple of 16 (nontemporal 16-byte accesses).
hipError_t launch_copy(const void *src, void *dst, int64_t bytes, int grid, hipStream_t s);
// Reads `bytes` (a multiple of 16) of src; sink has `grid` words and is
// written only for data no probe uses.
hipError_t launch_read(const void *src, int64_t bytes, uint32_t *sink, int grid, hipStream_t s);

// ---- the allocation-free loss entry point
//
// The library's file-scope device scratch: kStaticScratchBytes on every device
// the library runs on, held until the process ends, shared by every call on
// that device. static_scratch looks its address up on `device` (which must be
// the current device) the first time and returns the cached address after;
// the array's host-side name is never a device address.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
hipError_t static_scratch(int device, void **ptr);

// Final sums of the loss partials (kLossGrid x 5 x k, as launch_loss_partials
// writes them): for each probe p, the five sums over the workgroups in
// ascending order, then out[p] = sai, out[k + p] = l2 and
// out[2k + p] = cs = (w^T y) / (sqrt(w^T w) sqrt(y^T y)).
hipError_t launch_loss_final(int32_t k, const double *part, double *out, hipStream_t s);

}  // namespace pcgk
