/*
 * pcg.h - C ABI of the MI355X (gfx950) preconditioned conjugate-gradient
 * library with a factorized sparse approximate inverse preconditioner
 *
 *     M^-1 = G G^T + eps I                      (paper Sec. 3.2.1, Eq. "major")
 *
 * applied as two sparse matrix-vector products (t = G^T r, then
 * s = G t + eps r) with no triangular solve (Sec. 3.2.1, the paragraph after
 * Eq. "major"), inside the standard PCG iteration of Appendix A,
 * Algorithm 1. The solver's stopping metric is the relative residual
 * ||b - A x|| / ||b|| of Sec. 4.1.
 *
 * Conventions for every entry point
 *   - Return value: PCG_OK (0) or a status code below. No C++ exception
 *     crosses this interface. pcg_last_error() gives a message for the
 *     context's most recent failure.
 *   - Matrices are square CSR: int32 row pointers (n+1 entries, rowptr[0] = 0,
 *     non-decreasing), int32 column indices (nnz entries, strictly ascending
 *     within each row, in [0, n)), float64 values. nnz < 2^31.
 *   - Input pointers are borrowed for the duration of the call only: the
 *     library copies what it needs into its own device memory (cast to the
 *     storage types of pcg_config). `on_device` = 0 means host pointers,
 *     1 means device pointers of the context's GPU.
 *   - Vectors at the boundary are float64 (length n). The solution pointer x
 *     is owned by the caller; it is read as x0 and written before return.
 *   - One context serves one device and one HIP stream; calls on one context
 *     must not overlap, except that pcg_submit_batch, pcg_poll and
 *     pcg_pool_info may run on other threads while pcg_progress or pcg_wait
 *     runs.
 */
#ifndef PCG_H
#define PCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PCG_OK 0
#define PCG_PENDING 1        /* (batch) request queued or running */
#define PCG_NOT_CONVERGED 2  /* maxit reached; x holds the last iterate */
#define PCG_EINVAL (-1)      /* bad argument or malformed CSR */
#define PCG_ESTATE (-2)      /* call out of order (e.g. solve before set_matrix) or size mismatch */
#define PCG_ENOMEM (-3)      /* device allocation failed or budget exceeded */
#define PCG_EBREAKDOWN (-4)  /* d^T A d <= 0, r^T M^-1 r < 0, or NaN/Inf: A or M not SPD */
#define PCG_EDEVICE (-5)     /* HIP runtime error; the context must be destroyed */

/* storage types */
#define PCG_F64 0
#define PCG_F32 1
#define PCG_BF16 2
#define PCG_F16 3

/* preconditioner kinds for pcg_build_precond / pcg_build_g_host */
#define PCG_G_FSAI 1     /* classic FSAI (Kolotilina-Yeremin, cited in Sec. 3.2.1): G = G_L^T, G_L lower on tril(A) */
#define PCG_G_FIXED 2    /* lower G on tril(A): G_ii = 1/sqrt(A_ii), G_ij = -0.25 A_ij / sqrt(A_ii A_jj) */
#define PCG_G_JACOBI 3   /* G = D^-1/2, so M^-1 = D^-1 */
#define PCG_G_IDENTITY 4 /* G = I: plain CG */
/* Seeded G on A's full pattern, standing in for a learned G of that shape
 * (Sec. 3.2.2): G_ii = 1/sqrt(A_ii) and, for j != i,
 * G_ij = 0.25 u_ij |A_ij| / sqrt(A_ii A_jj) with u_ij = 2 U - 1, U the draw at
 * index i*n + j of stream 3 of the SplitMix64 counter generator keyed by the
 * seed (Steele, Lea and Flood 2014: key = mix(mix(seed + GAMMA) + 4 GAMMA),
 * draw k = mix(key + (k + 1) GAMMA), U = ((draw >> 11) + 1) 2^-53). G G^T is
 * not guaranteed SPD for every A: use it with eps > 0, e.g. 1e-4 / mean|A_ij|. */
#define PCG_G_SEEDED 5
/* Block FSAI for 3-dof systems (the blocked systems of Sec. 3.1, whose G has
 * one 3x3 block per nonzero block, Sec. 3.2.2): A must be exactly 3x3-blocked
 * (see PCG_LAYOUT_BSR3; else PCG_EINVAL). G = G_L^T with G_L block lower on
 * the block pattern of tril(A), every 3x3 block stored whole: for block row
 * I with tril blocks J, A[J,J] = L L^T and block row I of G_L is the last
 * three rows of L^-1, so each diagonal block of G_L A G_L^T is the identity
 * (M^-1 = G G^T does not depend on that choice within the block row).
 * G and G^T are then exactly 3x3-blocked and take the 3x3-block layout. */
#define PCG_G_BFSAI 6

/* operators for pcg_matvec */
#define PCG_OP_A 0    /* y = A x */
#define PCG_OP_GT 1   /* y = G^T x */
#define PCG_OP_G 2    /* y = G x */
#define PCG_OP_MINV 3 /* y = G (G^T x) + eps x  (the preconditioner apply, Eq. "major") */

typedef struct pcg_ctx pcg_ctx;

typedef struct {
  int device;        /* HIP device ordinal */
  void *stream;      /* hipStream_t to run on (kept alive by the caller until pcg_destroy; no other
                        thread may enqueue on it during a library call, which may capture HIP
                        graphs on it); NULL: the library creates its own */
  int vec_dtype;     /* PCG_F64 or PCG_F32: Krylov vectors and SpMV accumulation */
  int a_dtype;       /* PCG_F64 or PCG_F32: stored values of A (must equal vec_dtype) */
  int g_dtype;       /* PCG_F64, PCG_F32, PCG_BF16 or PCG_F16: stored values of G and G^T.
                        With F64 vectors any of them (G only preconditions: a rounded G is another
                        SPD M, and the FP64 iteration still reaches the FP64 tolerance); with F32
                        vectors F32, BF16 or F16. F16 values are stored times a power of two. */
  int rr_period;     /* recompute r = b - A x every rr_period iterations (Algorithm 1 uses 50); 0 = never */
  double eps;        /* shift of M^-1 = G G^T + eps I, absolute units (default 0) */
  int refine;        /* 1: FP64 iterative refinement around a vec_dtype = F32 inner PCG. A single
                        solve whose outer step gains less than 2x, or whose FP32 inner solve breaks
                        down, continues with FP64 inner solves (pcg_result.escalated) */
  double inner_tol;  /* relative tolerance of each inner solve under refinement (default 1e-6). A
                        step that can finish, i.e. whose target tol*||b|| / (4 ||r64||) is at least
                        inner_tol / 10, runs to min(1/2, that target) instead */
  int max_outer;     /* refinement steps at most (default 30) */
  int graph_iters;   /* iterations per captured HIP graph replay (default 10; 0 = plain launches) */
  int grid_mult;     /* workgroups per compute unit for the SpMV kernels (default 4: every consumer of a
                        kernel's partial sums reads all of them, so fewer, fuller workgroups pay) */
  int mem_budget_mb; /* device memory pool for batched / served systems, MiB (0: half the free memory at first use) */
  int layout;        /* storage of A, G, G^T: PCG_LAYOUT_AUTO (default), _CSR, _SELL, _BSR3 or _SDIA */
  int g_device;      /* 1: FSAI factored on the device (one wave per row; same arithmetic as the host
                        builder, bit-identical G): in pcg_build_precond(PCG_G_FSAI), and for batched
                        systems with FSAI at admission (the host lays out only the patterns; F16 G
                        is built on the host). Falls back to the host builder for tril rows longer
                        than 80 or a structurally unsymmetric A. 0 (default): on the host */
  int wide_index;    /* 0 (default): a sliced matrix whose every stored column lies within 32767 of its
                        row keeps 16-bit column - row differences (half the index bytes); 1: always
                        32-bit column indices */
  int autotune;      /* 1: pcg_set_precond and pcg_build_precond end with pcg_autotune(ctx, 20, NULL) */
  int cache_mb;      /* memory-side cache the single system's residency plan assumes, MiB (0: 256). The
                        matrices and iteration vectors all fit in 90% of it: all three matrices are read
                        with ordinary loads and stay cached across iterations; else the first of A, G
                        with G^T, G that fits in 75%; else none (nontemporal loads). Negative: always
                        nontemporal. Batched and served systems keep theirs while the whole active
                        set fits in 90% */
  int wg_max_n;      /* single solves of at most this many rows (FP64, or FP32 vectors and A with an
                        FP32/BF16/FP16 G, no refinement) run as one persistent workgroup: the whole
                        solve in one launch, with no per-iteration launches or host round trips, and
                        results bit for bit those of the three-kernel iteration. The iteration
                        vectors stay in the workgroup's LDS when they fit (up to 2048 FP64 or 4096
                        FP32 rows here, 512 or 1024 in a batch, where the device allows it). One
                        workgroup has far less memory parallelism than a full launch, so this pays
                        only for tiny systems. 0: the default (see pcg_config_default); -1: never */
  int wg_max_n_batch; /* the same for batched and served systems: those admitted in one scheduler
                        step run together, one workgroup each, in one launch on a second stream,
                        beside the iterations of the larger ones (many small systems keep the GPU
                        busy where one would not). 0: the default; -1: never */
  int rows_per_lane; /* rows per lane of the G^T- and G-kernels over sliced diagonals: 2 (every
                        operand, value and result access twice as wide; the default) or 1. 0: the
                        default. Results are the same bit for bit either way */
  int loads_in_flight; /* loads in flight per lane in the A-kernel's sliced rows of more than 4
                        entries: 8 (the default) or 4. 0: the default. Same results either way */
  /* Optional device allocator (for example a framework's caching allocator),
   * used for every device allocation of the context (matrices, vectors,
   * directory, serving pool, scratch): alloc returns at least `bytes` bytes of
   * device memory on cfg.device, 16-byte aligned (256 preferred), or NULL
   * (reported as PCG_ENOMEM); free releases a pointer alloc returned, after
   * the context's stream has been drained. Both or neither must be set (else
   * pcg_create returns PCG_EINVAL). NULL: hipMalloc / hipFree. */
  void *(*alloc)(size_t bytes, void *user);
  void (*free)(void *ptr, void *user);
  void *alloc_user; /* passed to alloc and free */
} pcg_config;

/* Matrix storage layouts (pcg_config.layout). All give bit-identical
 * products (each row is summed left to right in CSR order; stored zeros add
 * +0 to a sum that can never be -0, which changes nothing).
 *  CSR:  CSR plus a partition into blocks of up to 256 rows whose products
 *        fit the workgroup's LDS; any row lengths.
 *  SELL: sliced ELL, slices of 64 consecutive rows stored column-major and
 *        padded to the slice's longest row; coalesced loads without LDS.
 *  SDIA: sliced diagonals: slices of 64 rows store one int32 column offset
 *        (column - row) per distinct offset of the slice, and for each row
 *        one value per offset (0 where the row has none), in ascending
 *        column order. No per-entry index and contiguous gathers: for stencil
 *        and banded matrices.
 *  BSR3: for a matrix that is exactly 3x3-blocked (n % 3 == 0, each block
 *        row's three rows store the same complete column triples, as in
 *        node-major 3-dof systems): slices of 21 block rows, one column index
 *        per 3x3 block; products are still summed in CSR order. G and G^T,
 *        whose diagonal blocks are triangular, are stored as their 3x3-block
 *        cover (explicit zeros fill the missing entries) when the cover adds
 *        at most 1/8 of their nonzeros (at most 2x when BSR3 is forced).
 *  AUTO: BSR3 for such an A whose block padding stays within 1/8; otherwise
 *        SDIA when its stored values stay within 1/8 of the nonzeros, then
 *        SELL under the same rule, CSR otherwise. PCG_LAYOUT_SELL, _SDIA and
 *        _BSR3 still fall back above 2x. */
#define PCG_LAYOUT_AUTO 0
#define PCG_LAYOUT_CSR 1
#define PCG_LAYOUT_SELL 2
#define PCG_LAYOUT_BSR3 3
#define PCG_LAYOUT_SDIA 4

typedef struct {
  int status;          /* PCG_OK, PCG_NOT_CONVERGED or a negative code */
  int iters;           /* CG iterations (summed over refinement steps) */
  int outer_iters;     /* refinement steps (0 without refinement) */
  int restarts;        /* times the recurrence residual met tol but b - A x did not (restart from it) */
  double relres_true;  /* ||b - A x|| / ||b|| at exit, formed in the vector precision (FP64 under refinement) */
  double relres_rec;   /* recurrence ||r|| / ||b|| at exit */
  double t_solve_ms;   /* single solve: device time; batched: admission to completion (host clock) */
  double bytes_per_iter; /* device bytes of one iteration in the layouts in use: A, G^T and G once
                            as stored (values with their padding; column information at its stored
                            width: 4 or 2 bytes per slot, one index per 3x3 block, one offset per
                            sliced-diagonal entry; row or slice pointers), 11 vector streams */
  double t_latency_ms; /* batched: submission to completion (host clock) */
  double t_queue_ms;   /* batched: submission to admission (host clock) */
  int escalated;       /* single solve under refinement: 1 when the inner solves switched to FP64 */
  int reserved_;
} pcg_result;

/* One system of a batch (all pointers host memory, borrowed for the call). */
typedef struct {
  int32_t n;
  int64_t nnz_a;
  const int32_t *a_rowptr;
  const int32_t *a_col;
  const double *a_val;
  int64_t nnz_g;             /* G given explicitly (g_rowptr non-NULL) ... */
  const int32_t *g_rowptr;
  const int32_t *g_col;
  const double *g_val;
  int g_kind;                /* ... or built on the host by this kind (PCG_G_FSAI, ...) */
  uint64_t g_seed;           /* seed of PCG_G_SEEDED */
  const double *b;           /* right-hand side, n entries */
  double *x;                 /* x0 on submission (NULL: zeros); the solution is written here on completion */
  double tol;
  int maxit;
} pcg_system;

/* Fills cfg with the defaults: device 0, own stream, all FP64, rr_period 50,
 * eps 0, no refinement, inner_tol 1e-6, max_outer 30, graph_iters 10,
 * grid_mult 4, automatic layouts, no autotuning, wg_max_n 512,
 * wg_max_n_batch 16384, rows_per_lane 2, loads_in_flight 8, the default
 * allocator. */
void pcg_config_default(pcg_config *cfg);

/* Creates a context on cfg->device. Returns PCG_EDEVICE if no usable GPU,
 * PCG_EINVAL for an unsupported dtype combination (FP64 vectors need FP64 A
 * and no refinement; FP32 vectors need FP32 A and a G of FP32, BF16 or FP16),
 * a negative rr_period, graph_iters or mem_budget_mb, eps < 0 or NaN,
 * rows_per_lane other than 0, 1, 2, loads_in_flight other than 0, 4, 8, or
 * only one of alloc / free. *out is NULL on failure. */
int pcg_create(const pcg_config *cfg, pcg_ctx **out);
void pcg_destroy(pcg_ctx *ctx);

/* Sets the SPD matrix A (validated; see conventions). Replaces any previous A
 * and drops a preconditioner of another size. */
int pcg_set_matrix(pcg_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                   const double *val, int on_device);

/* Sets G of M^-1 = G G^T + eps I (Eq. "major"), any sparsity pattern
 * (the paper's learned G uses A's full pattern, Sec. 3.2.2). The library also
 * stores G^T explicitly, so both products are row-wise, each matrix in its
 * own layout. n must equal A's n. */
int pcg_set_precond(pcg_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                    const double *val, int on_device);

/* Builds G from the current A (PCG_G_FSAI, PCG_G_FIXED, PCG_G_JACOBI,
 * PCG_G_IDENTITY, PCG_G_SEEDED with `seed`; the seed is ignored by the other
 * kinds) and sets it: on the host, or for PCG_G_FSAI with g_device = 1 on the
 * device (same G bit for bit). A must have been set from host memory or will
 * be downloaded once. */
int pcg_build_precond(pcg_ctx *ctx, int kind, uint64_t seed);

/* Solves A x = b by PCG (Algorithm 1) to ||b - A x|| <= tol ||b||, at most
 * maxit iterations (per refinement step under refinement). x holds x0 on
 * entry. b = 0 gives x = 0. res may be NULL. Returns PCG_OK,
 * PCG_NOT_CONVERGED, PCG_EBREAKDOWN, or an error code. */
int pcg_solve(pcg_ctx *ctx, const double *b, double *x, double tol, int maxit, int on_device, pcg_result *res);

/* y = op(x) with the stored A, G or G^T, or the preconditioner apply, in the
 * context's vector precision (values at the boundary are float64). */
int pcg_matvec(pcg_ctx *ctx, int op, const double *x, double *y, int on_device);

/* Preconditioner-quality losses over k probe vectors (Sec. 3.3, the loss
 * function: the Hutchinson estimate of a Frobenius norm by products with
 * i.i.d. N(0,1) probes, Eq. "loss-initial"; the scale-invariant SAI loss of
 * Eq. "our-loss" with ||A|| = mean |A_ij| over the nonzeros; the L2 and
 * cosine-similarity losses of the loss ablation). With y = A M^-1 w and
 * M^-1 = G G^T + eps I for the context's stored A, G and eps, for each probe
 * p (column p of W):
 *   sai[p] = || y / ||A|| - w ||^2,   l2[p] = || y - w ||^2,
 *   cs[p]  = w^T y / (||w|| ||y||).
 * Their means over the probes estimate ||A M^-1 / ||A|| - I||_F^2 and
 * ||A M^-1 - I||_F^2. W: n x k, row-major (probe p of row i at W[i*k + p]),
 * FP64, host or device memory (on_device), borrowed for the call; sai, l2,
 * cs: host arrays of k doubles, each may be NULL. Products run in FP64 on the
 * stored values (rounded to their storage types); each row is summed in CSR
 * order. Uses 3 n k doubles of device scratch, allocated at the first call
 * that needs more and kept by the context until pcg_destroy.
 * PCG_EINVAL (k < 1, null W), PCG_ESTATE (A or G unset), PCG_ENOMEM. */
int pcg_sai_loss(pcg_ctx *ctx, int32_t k, const double *W, int on_device, double *sai, double *l2, double *cs);

/* Allocation-free variant of pcg_sai_loss, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation). Same losses, same kernels and summation order as
 * pcg_sai_loss, so the same values. W must be device memory of the context's
 * GPU (n x k row-major FP64, borrowed for the call); sai, l2, cs are host
 * arrays of k doubles, each may be NULL. Scratch (2 n k + 2563 k doubles,
 * each part 256-byte aligned) comes from the library's file-scope device
 * array of 64 MiB, one per GPU, held until the process ends; a larger need
 * returns PCG_EINVAL with a message, and nothing is allocated. Every call on
 * one GPU (from any context) shares that GPU's array, and it keeps the last
 * call's contents: calls that overlap on one GPU race. PCG_ESTATE (A or G
 * unset), PCG_EINVAL (k < 1, null W, too large), PCG_EDEVICE. */
int pcg_sai_loss_noalloc(pcg_ctx *ctx, int32_t k, const double *W, double *sai, double *l2, double *cs);

/* Measurement (not an operation of the paper, whose evaluation times whole
 * solves and splits them into construction, apply and CG time, Sec. 4.2 and
 * Tab. "time-decomposition": a facility of this library for per-kernel
 * bandwidth figures). Runs `iters` CG iterations of the stored system (a fresh
 * solve of the last right-hand side from x0 = 0 that never stops; the
 * context's vectors are overwritten) as plain launches on the context's
 * stream, each with start/stop events attached to its dispatch (the
 * kernel's own execution interval). ms[0..2]: average duration of the A-,
 * G^T- and G-kernel launches; ms[3]: average iteration (A start to G end).
 * bytes[0..3] (may be NULL): their device bytes per launch in the stored
 * layouts (A: A's values, column indices at their stored width and row
 * pointers, plus 2 vector streams; G^T: G^T plus 4; G: G plus 5, 6 with
 * eps). Needs one prior pcg_solve with b != 0 (or a nonzero stored b). */
int pcg_time_kernels(pcg_ctx *ctx, int iters, double *ms, double *bytes);

/* Measurement (not in the paper): the device's streaming ceilings.
 * pcg_copy_bandwidth: device-to-device copy of `bytes` (rounded down to 16)
 * repeated `reps` times (after two untimed copies) with 16-byte nontemporal
 * loads and stores, four in flight per lane; *gbps = 2 bytes reps / time
 * (read plus write), *ms_per_copy the average launch (may be NULL).
 * pcg_read_bandwidth: the same kernel shape reading `bytes` only;
 * *gbps = bytes reps / time. Both allocate and free their own buffers.
 * The measured HBM ceiling and the reference for calibrating memory-traffic
 * counters. PCG_EINVAL (bytes < 16, reps < 1, null gbps), PCG_ENOMEM,
 * PCG_EDEVICE. */
int pcg_copy_bandwidth(int device, int64_t bytes, int reps, double *gbps, double *ms_per_copy);
int pcg_read_bandwidth(int device, int64_t bytes, int reps, double *gbps, double *ms_per_read);

/* Batching and serving. The paper solves one system at a time (Sec. 4.1);
 * it defines no batched or served operation. These entry points are this
 * library's way to run many independent PCG solves (Algorithm 1 each) on one
 * GPU. Independent systems of any sizes are solved
 * together: each CG kernel is one launch over all admitted systems (each
 * system keeps its own row blocks, reductions and scalars, so its result is
 * bit for bit the one it gets alone). The context owns a device memory pool
 * (pcg_config.mem_budget_mb); a request is admitted when its storage fits and
 * refused with PCG_ENOMEM only if it exceeds the whole pool. Vector and
 * storage types are the context's; with pcg_config.refine each system runs
 * its own FP64 refinement (its outer steps taken between scheduler steps;
 * no escalation to FP64 inner solves here). If a device call fails while a
 * step admits requests, none of them starts: each finishes with that error
 * (PCG_ENOMEM for refused memory, else PCG_EDEVICE), its storage goes back
 * to the pool, and pcg_progress returns the error.
 *
 * pcg_submit_batch copies every input and returns at once with one ticket per
 * system (nothing is queued if any system is invalid). Host worker threads
 * build G (when not given) and stage the data. pcg_progress runs one
 * scheduler step on the calling thread: admit ready requests in arrival order
 * while the pool has room, run `iters` CG iterations over all admitted systems
 * (iteration-level continuous batching), and retire finished systems (x
 * written to the caller's pointer, device storage freed). *active and *queued
 * (may be NULL) report the systems admitted and those submitted but not yet
 * admitted (in host preparation or waiting for room). pcg_poll returns
 * PCG_PENDING until the ticket's request has finished, then its final status
 * (and fills *res); a finished ticket is released by the poll that reports
 * it. Submission may run concurrently with pcg_progress from another thread;
 * the caller must keep each system's x buffer alive until its ticket is done.
 * pcg_solve_batch submits `count` systems and progresses until all finish,
 * `iters_per_step` iterations per step (0: 20). pcg_wait drives pcg_progress
 * (graph_iters iterations per step, 0: 20) until every one of `count`
 * tickets has finished, then collects them as pcg_poll does (results may be
 * NULL; a ticket listed twice is reported twice); timeout_s < 0 waits
 * without limit. It returns PCG_PENDING, with no
 * ticket collected, when the time runs out first, and PCG_EINVAL for an
 * unknown or already collected ticket. The per-system status is in
 * results[i].status. */
int pcg_submit_batch(pcg_ctx *ctx, int count, const pcg_system *sys, uint64_t *tickets);
int pcg_progress(pcg_ctx *ctx, int iters, int *active, int *queued);
int pcg_poll(pcg_ctx *ctx, uint64_t ticket, pcg_result *res);
int pcg_wait(pcg_ctx *ctx, int count, const uint64_t *tickets, pcg_result *results, double timeout_s);
int pcg_solve_batch(pcg_ctx *ctx, int count, const pcg_system *sys, pcg_result *results, int iters_per_step);

/* Capacity and bytes in use of the batch pool (0 before first use). Not in
 * the paper: part of the batching facility above. */
int pcg_pool_info(pcg_ctx *ctx, size_t *capacity, size_t *in_use);

/* Measurement of the batching facility (not in the paper). Device time and
 * bytes of the scheduler's work since the context was created or the last
 * reset: each step's iterations over the active set are timed by events on
 * the context's stream around their launches (admission uploads and state
 * readbacks fall outside), and their bytes are, per system, the iterations
 * it ran in the step times its pcg_result.bytes_per_iter. One-workgroup
 * launches of small systems (second stream, overlapping the steps) are timed
 * from launch to completion, with each system's iterations times its bytes
 * per iteration. step_bytes / step_ms is the aggregate bandwidth over the
 * active set. reset != 0 zeroes the counters after reading them. Returns
 * PCG_EINVAL for a NULL pointer. */
typedef struct {
  int64_t steps;       /* scheduler steps that ran iterations */
  double step_ms;      /* their device time */
  double step_bytes;   /* bytes their iterations moved (layouts as stored) */
  int64_t wg_launches; /* one-workgroup launches */
  double wg_ms;        /* their device time */
  double wg_bytes;     /* bytes of their iterations */
  /* host time (wall clock) of the scheduler's phases and of the workers */
  double host_prep_ms;   /* worker threads preparing systems (G, layouts, images), summed over threads */
  double host_admit_ms;  /* scheduler: admission (pool blocks, uploads, first kernels) */
  double host_step_ms;   /* scheduler: launching the steps' iterations and reading the states back */
  double host_retire_ms; /* scheduler: finishing stopped systems (final residual, solution copies, refinement steps) */
  double host_progress_ms; /* scheduler: all of its steps (the three phases above and the rest of each step) */
  double host_idle_ms;     /* waiting callers (pcg_wait, pcg_solve_batch) asleep with nothing active */
} pcg_batch_stats;
int pcg_batch_stats_get(pcg_ctx *ctx, pcg_batch_stats *out, int reset);

/* Host-only helpers (no GPU needed). */

/* Checks a CSR matrix against the conventions above; require_diag = 1 also
 * demands a stored diagonal entry in every row. */
int pcg_validate_csr(int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col, int require_diag);

/* Number of nonzeros of G for kind on A's pattern (-1 on error). */
int64_t pcg_g_nnz(int kind, int32_t n, const int32_t *rowptr, const int32_t *col);

/* Builds G of kind (seed: PCG_G_SEEDED only) from A into caller arrays sized
 * n+1 / pcg_g_nnz. */
int pcg_build_g_host(int kind, uint64_t seed, int32_t n, const int32_t *rowptr, const int32_t *col,
                     const double *val, int32_t *g_rowptr, int32_t *g_col, double *g_val);

/* Autotuner (not in the paper: a facility of this library that picks storage
 * layouts, launch grid and load policy for the paper's iteration). Times one CG iteration of the single system (its three kernels
 * on b = 1: `iters` iterations for warm-up, then the smaller of two timings
 * of `iters` iterations) for each candidate storage of A (CSR row blocks,
 * sliced ELL, 3x3 blocks: each distinct format the matrix admits) and of G
 * and G^T (CSR, sliced ELL, and for a host-built G with n divisible by 3 its
 * 3x3-block cover), at the configured grid, then for the best layouts at
 * half and twice the grid, then the load policy (each subset of A, G, G^T
 * read with ordinary loads and kept in the memory-side cache, besides the
 * residency plan's choice), then two kernel knobs: rows per lane of the
 * G^T- and G-kernels over sliced diagonals (two rows make every access
 * twice as wide, or one) and loads in flight per lane in the A-kernel's sliced rows
 * (8 or 4), and keeps the fastest (a candidate must beat the current best
 * by 3%).
 * The matrices are laid out again with the same values, so products stay
 * bit-identical, and inner products are exact: every candidate gives the
 * same solve bit for bit. A layout forced in the configuration is kept; only
 * the grid, the load policy and the kernel knobs are tuned then.
 * The choice is cached per matrix signature (sizes, row-length structure, 3x3
 * blocking, storage types, options, compute units) for the process, and in
 * the file named by the environment variable PCG_TUNE_CACHE when set; a
 * cached signature is applied without search (candidates = 0). A new
 * pcg_set_matrix returns to the automatic layouts. Needs A and G set;
 * overwrites the stored right-hand side. iters <= 0: 20; above 1000:
 * PCG_EINVAL. On an error while laying the matrices out again (out of
 * memory, a HIP error) the context may have lost the matrix, the
 * preconditioner or both (solves then return PCG_ESTATE): set them again. */
typedef struct {
  int layout_a, layout_g; /* chosen PCG_LAYOUT_* (PCG_LAYOUT_AUTO: the automatic choice won) */
  int grid_mult;          /* chosen workgroups per compute unit */
  int candidates;         /* configurations timed (0: taken from the cache) */
  int fmt_a, fmt_g, fmt_gt; /* resulting storage: 0 CSR row blocks, 1 sliced ELL, 2 sliced 3x3 blocks,
                              3 sliced diagonals */
  int idx16;              /* bit 0/1/2: A / G / G^T keep 16-bit column differences */
  int temporal;           /* bit 0/1/2: A / G / G^T read with ordinary loads (cache-resident) */
  int rows_per_lane_gt;   /* rows per lane of the G^T- and G-kernels over sliced diagonals: 2 (default)
                             or 1 */
  int loads_in_flight_a;  /* loads in flight per lane of the A-kernel's sliced rows: 8 (default) or 4 */
  double ms_per_iter;      /* chosen configuration, one iteration */
  double ms_per_iter_auto; /* the automatic choice (NaN when taken from the cache) */
} pcg_tune_result;
int pcg_autotune(pcg_ctx *ctx, int iters, pcg_tune_result *res);

/* Admission planning for the batching facility (not in the paper). Upper estimate of the device memory one system (n unknowns, nnz_a entries
 * of A, nnz_g of G) takes from the serving pool of a context configured by
 * cfg: A, G and G^T as the automatic layout stores them (sliced layouts are
 * chosen only while their padding stays within 1/8; a forced sliced layout
 * may pad more), the vectors, staging, partial sums, and the FP64 view of A
 * under refinement. For admission planning; host only, no GPU needed.
 * Returns PCG_EINVAL for a NULL pointer, n <= 0 or negative counts. */
int pcg_estimate_bytes(const pcg_config *cfg, int32_t n, int64_t nnz_a, int64_t nnz_g, size_t *bytes);

/* Measurement (not in the paper, which reports no bandwidth). Algorithmic device bytes of one PCG iteration over int32 CSR: A, G^T and G
 * read once (values and 4-byte column indices), their row pointers, and 11
 * vector streams of n entries (vec bytes each). Results report the bytes of
 * the layouts actually used (pcg_result.bytes_per_iter), which store 16-bit
 * column differences, one index per 3x3 block or one offset per sliced-
 * diagonal entry where they can. */
double pcg_bytes_per_iter(int32_t n, int64_t nnz_a, int64_t nnz_g, int a_dtype, int g_dtype, int vec_dtype);

const char *pcg_last_error(const pcg_ctx *ctx);
const char *pcg_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* PCG_H */
