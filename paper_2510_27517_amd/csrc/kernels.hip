// gfx950 kernels for preconditioned CG with M^-1 = G G^T + eps I.
//
// Every operator product is a CSR sparse matrix-vector product ("CSR
// stream"): a workgroup owns a block of consecutive rows whose nonzeros fit
// in LDS; its threads load the block's column indices and values with
// coalesced loads, gather the vector entries (through L2), and stage the
// row products in LDS; then one thread per row adds its products in CSR
// order. The A, G^T and G products carry the CG vector updates in their
// gathers and epilogues, so one iteration is three launches:
//   A-kernel : d_i = s_i + beta_i d_{i-1}  (formed where it is gathered),
//              x += alpha_{i-1} d_{i-1}     (the update deferred from i-1),
//              q = A d_i,  gamma = d_i^T q, alpha_i = delta_i / gamma;
//   G^T-kernel: r_{i+1} = r_i - alpha_i q  (formed where it is gathered),
//              t = G^T r_{i+1}, ||r||^2, ||t||^2,
//              delta_{i+1} = ||t||^2 + eps ||r||^2 (= r^T M^-1 r),
//              beta_{i+1} = delta_{i+1} / delta_i, convergence test;
//   G-kernel : s_{i+1} = G t + eps r_{i+1}.
// d and r alternate between two buffers by iteration parity, so no
// workgroup overwrites a vector entry another one still gathers.
//
// Reductions are deterministic and need no atomics: each workgroup reduces
// its rows with wave shuffles and LDS and writes one partial per value; every
// workgroup of the next kernel adds all partials in the same fixed order
// (kernel boundaries make them visible), so all obtain the identical total.
// One workgroup publishes the updated scalars into a state slot that the
// kernel itself does not read.
//
// Work placement: each of the 8 XCDs (workgroup b runs on XCD b % 8) owns a
// contiguous eighth of the row blocks, and its workgroups take those blocks
// interleaved, so at any moment an XCD works on one window of consecutive
// rows whose gathered neighbourhoods stay in that XCD's L2.
//
// Built with floating-point contraction off: every product and sum rounds
// separately, in the order written (rows summed left to right from zero),
// which is also the order of the plain CSR definition.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace pcgk {

// Matrix values and column indices are read exactly once per product:
// nontemporal loads keep them from displacing the gathered vector entries in
// L2 (PCG_NT_MATRIX = 0 uses ordinary loads).
#ifndef PCG_NT_MATRIX
#define PCG_NT_MATRIX 1
#endif
#ifndef PCG_UNROLL
#define PCG_UNROLL 4
#endif

struct bf16_t { uint16_t bits; };

template <typename T>
__device__ __forceinline__ T ldstream(const T *p, int64_t k) {
#if PCG_NT_MATRIX
  return __builtin_nontemporal_load(p + k);
#else
  return p[k];
#endif
}

__device__ __forceinline__ double ldval(const double *p, int64_t k) { return ldstream(p, k); }
__device__ __forceinline__ float ldval(const float *p, int64_t k) { return ldstream(p, k); }
__device__ __forceinline__ float ldval(const bf16_t *p, int64_t k) {
  return __uint_as_float((uint32_t)ldstream((const uint16_t *)p, k) << 16);
}
__device__ __forceinline__ float ldval(const _Float16 *p, int64_t k) { return (float)ldstream(p, k); }

// Workgroup b is dispatched to XCD b % 8; give XCD x the logical ids
// [x*G/8, (x+1)*G/8) so its workgroups cover consecutive rows. G % 8 == 0.
__device__ __forceinline__ int xcd_remap(int b, int G) { return (b & 7) * (G >> 3) + (b >> 3); }

template <typename TM>
struct Mat {
  const int32_t *rp, *ci;
  const TM *val;
  const int32_t *blk;
  int32_t nblk;
};

template <typename TM>
static Mat<TM> mat(const DevCSR &m) {
  return Mat<TM>{m.rp, m.ci, (const TM *)m.val, m.blk, m.nblk};
}

// Operands of one row loaded before the row's products are staged.
template <typename TV>
struct RowVals {
  TV a, b, c;
};

// One row block: stage products in LDS, sum each row in CSR order. `pre(row)`
// loads the row's own operands early (overlapping the gathers), `epi(row,
// sum, pre_values)` consumes the row's sum.
template <typename TACC, typename TM, typename Pre, typename Gather, typename Epi>
__device__ __forceinline__ void stream_block(const Mat<TM> &M, int b, TACC *lds, Pre pre, Gather gather, Epi epi) {
  constexpr int cap = kLdsBytes / (int)sizeof(TACC);
  const int tid = threadIdx.x;
  const int r0 = M.blk[2 * b], k0 = M.blk[2 * b + 1], r1 = M.blk[2 * b + 2], k1 = M.blk[2 * b + 3];
  if (k1 - k0 <= cap) {
    const int row = r0 + tid;
    const bool has = row < r1;
    int a = 0, e = 0;
    RowVals<TACC> pv{};
    if (has) {
      a = M.rp[row] - k0;
      e = M.rp[row + 1] - k0;
      pv = pre(row);
    }
#pragma unroll PCG_UNROLL
    for (int k = k0 + tid; k < k1; k += kBlock) lds[k - k0] = (TACC)ldval(M.val, k) * gather(ldstream(M.ci, k));
    __syncthreads();
    if (has) {
      TACC sum = 0;
      for (int k = a; k < e; ++k) sum += lds[k];
      epi(row, sum, pv);
    }
    __syncthreads();
  } else {
    // a single row longer than the LDS window: chunks, summed in order by thread 0
    RowVals<TACC> pv{};
    if (tid == 0) pv = pre(r0);
    TACC sum = 0;
    for (int c0 = k0; c0 < k1; c0 += cap) {
      const int c1 = min(c0 + cap, k1);
      for (int k = c0 + tid; k < c1; k += kBlock) lds[k - c0] = (TACC)ldval(M.val, k) * gather(ldstream(M.ci, k));
      __syncthreads();
      if (tid == 0)
        for (int k = 0; k < c1 - c0; ++k) sum += lds[k];
      __syncthreads();
    }
    if (tid == 0) epi(r0, sum, pv);
  }
}

// This workgroup's row blocks: first, first + stride, ... < end; L is its
// logical index (the slot of its partial sums).
struct Sched {
  int first, end, stride, L;
};

__device__ __forceinline__ Sched sched(int nblk) {
  const int G = gridDim.x, W = G >> 3, x = blockIdx.x & 7, l = blockIdx.x >> 3;
  Sched sc;
  sc.first = (int)((int64_t)x * nblk / 8) + l;
  sc.end = (int)((int64_t)(x + 1) * nblk / 8);
  sc.stride = W;
  sc.L = x * W + l;
  return sc;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *sh) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] += __shfl_xor(v[j], off);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NW = kBlock / 64;
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) sh[j * NW + w] = v[j];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      double a = sh[j * NW];
      for (int q = 1; q < NW; ++q) a += sh[j * NW + q];
      v[j] = a;
    }
  __syncthreads();
}

// Write this workgroup's partial sums (value j at p[j * G + L]).
template <int NV>
__device__ __forceinline__ void put_partials(double (&v)[NV], double *p, int L, double *sh) {
  block_sum<NV>(v, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) p[(int64_t)j * gridDim.x + L] = v[j];
}

// Sum the P partials of each value in a fixed order; every thread gets the totals.
template <int NV>
__device__ __forceinline__ void sum_partials(const double *__restrict__ p, int P, double (&out)[NV], double *sh) {
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
#pragma unroll 8
  for (int k = threadIdx.x; k < P; k += kBlock)
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] += p[(int64_t)j * P + k];
  block_sum<NV>(acc, sh);
  __shared__ double tot[NV];
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) tot[j] = acc[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NV; ++j) out[j] = tot[j];
}

// ------------------------------------------------------------------ kernels

template <typename TV, typename TA>
__global__ __launch_bounds__(kBlock) void k_iter_A(Mat<TA> A, TV *__restrict__ x, const TV *__restrict__ s,
                                                   TV *__restrict__ d0, TV *__restrict__ d1, TV *__restrict__ q,
                                                   const State *__restrict__ st, double *__restrict__ pg) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  __shared__ double sh[4 * (kBlock / 64)];
  const State &S = st[0];
  if (S.done) return;
  const int it = S.iter;
  const TV beta = (TV)S.beta, ap = (TV)S.alpha;
  const TV *__restrict__ dold = (it & 1) ? d0 : d1;  // d_{i-1}
  TV *__restrict__ dnew = (it & 1) ? d1 : d0;        // d_i
  double part[1] = {0.0};
  const Sched sc = sched(A.nblk);
  for (int b = sc.first; b < sc.end; b += sc.stride)
    stream_block<TV>(
        A, b, lds, [&](int row) { return RowVals<TV>{s[row], dold[row], x[row]}; },
        [&](int j) -> TV { return s[j] + beta * dold[j]; },
        [&](int row, TV sum, const RowVals<TV> &pv) {
          const TV di = pv.a + beta * pv.b;
          dnew[row] = di;
          q[row] = sum;
          x[row] = pv.c + ap * pv.b;
          part[0] += (double)di * (double)sum;
        });
  put_partials<1>(part, pg, sc.L, sh);
}

template <typename TV, typename TG>
__global__ __launch_bounds__(kBlock) void k_iter_GT(Mat<TG> GT, TV *__restrict__ r0, TV *__restrict__ r1,
                                                    const TV *__restrict__ q, TV *__restrict__ t,
                                                    State *__restrict__ st, const double *__restrict__ pg, int P_a,
                                                    double *__restrict__ prt, int mode) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  __shared__ double sh[4 * (kBlock / 64)];
  const State &S = st[0];
  if (S.done) return;
  const int it = S.iter;
  double alpha = S.alpha, gamma = S.gamma;
  bool brk = false;
  if (mode != 2) {
    double g[1];
    sum_partials<1>(pg, P_a, g, sh);
    gamma = g[0];
    brk = !(gamma > 0.0) || !isfinite(gamma);
    alpha = brk ? 0.0 : S.delta / gamma;  // on breakdown x already holds x_i
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    State o = S;
    o.gamma = gamma;
    o.alpha = alpha;
    if (brk) {
      o.status = ST_BREAK_GAMMA;
      o.done = 1;
    }
    st[1] = o;
  }
  if (brk) return;
  const TV al = (mode == 0) ? (TV)alpha : (TV)0;
  const TV *__restrict__ src = (((mode == 1) ? it + 1 : it) & 1) ? r1 : r0;
  TV *__restrict__ dst = ((it + 1) & 1) ? r1 : r0;
  double part[2] = {0.0, 0.0};
  const Sched sc = sched(GT.nblk);
  if (mode == 0) {
    for (int b = sc.first; b < sc.end; b += sc.stride)
      stream_block<TV>(
          GT, b, lds, [&](int row) { return RowVals<TV>{src[row], q[row], (TV)0}; },
          [&](int j) -> TV { return src[j] - al * q[j]; },
          [&](int row, TV sum, const RowVals<TV> &pv) {
            const TV rn = pv.a - al * pv.b;
            dst[row] = rn;
            t[row] = sum;
            part[0] += (double)rn * (double)rn;
            part[1] += (double)sum * (double)sum;
          });
  } else {
    for (int b = sc.first; b < sc.end; b += sc.stride)
      stream_block<TV>(
          GT, b, lds, [&](int row) { return RowVals<TV>{src[row], (TV)0, (TV)0}; },
          [&](int j) -> TV { return src[j]; },
          [&](int row, TV sum, const RowVals<TV> &pv) {
            t[row] = sum;
            part[0] += (double)pv.a * (double)pv.a;
            part[1] += (double)sum * (double)sum;
          });
  }
  put_partials<2>(part, prt, sc.L, sh);
}

template <typename TV, typename TG, bool HAS_EPS>
__global__ __launch_bounds__(kBlock) void k_iter_G(Mat<TG> G, const TV *__restrict__ t, const TV *__restrict__ r0,
                                                   const TV *__restrict__ r1, TV *__restrict__ s,
                                                   State *__restrict__ st, const double *__restrict__ prt, int P_gt,
                                                   int mode) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  __shared__ double sh[4 * (kBlock / 64)];
  if (st[0].done) return;  // stopped before this iteration's G^T-kernel ran
  const State &S = st[1];
  if (S.done) {  // the G^T-kernel flagged a breakdown: publish it
    if (blockIdx.x == 0 && threadIdx.x == 0) st[0] = S;
    return;
  }
  const int it = S.iter;
  double v[2];
  sum_partials<2>(prt, P_gt, v, sh);
  const double rr = v[0], tt = v[1];
  const double dn = tt + S.eps * rr;
  State o = S;
  o.rr = rr;
  o.tt = tt;
  const int i1 = (mode == 2) ? it : it + 1;
  o.iter = i1;
  if (mode != 2 && (!(dn >= 0.0) || !isfinite(dn))) {
    o.status = ST_BREAK_DELTA;
    o.done = 1;
  } else {
    o.beta = (mode == 2) ? 0.0 : dn / S.delta;
    o.delta = dn;
    if (sqrt(rr) <= S.tol_nb) {
      o.status = ST_CONV_REC;
      o.done = 1;
    } else if (i1 >= S.maxit) {
      o.status = ST_MAXIT;
      o.done = 1;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st[0] = o;
  if (o.done) return;
  const TV *__restrict__ rc = (i1 & 1) ? r1 : r0;
  const TV eps = (TV)S.eps;
  const Sched sc = sched(G.nblk);
  for (int b = sc.first; b < sc.end; b += sc.stride)
    stream_block<TV>(
        G, b, lds, [&](int row) { return RowVals<TV>{HAS_EPS ? rc[row] : (TV)0, (TV)0, (TV)0}; },
        [&](int j) -> TV { return t[j]; },
        [&](int row, TV sum, const RowVals<TV> &pv) {
          if (HAS_EPS)
            s[row] = sum + eps * pv.a;
          else
            s[row] = sum;
        });
}

template <typename TV, typename TA>
__global__ __launch_bounds__(kBlock) void k_resid(Mat<TA> A, const TV *__restrict__ b, const TV *__restrict__ x,
                                                  const TV *__restrict__ d0, const TV *__restrict__ d1,
                                                  TV *__restrict__ r0, TV *__restrict__ r1,
                                                  const State *__restrict__ st, const double *__restrict__ pg,
                                                  int P_a, double *__restrict__ ptr, int slot_sel, int with_d,
                                                  int respect_done) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  __shared__ double sh[4 * (kBlock / 64)];
  const State &S = st[0];
  if (respect_done && S.done) return;
  const int it = S.iter;
  TV *__restrict__ rout = ((it + slot_sel) & 1) ? r1 : r0;
  const TV *__restrict__ dc = (it & 1) ? d1 : d0;  // d_i
  TV al = (TV)0;
  if (with_d) {
    double g[1];
    sum_partials<1>(pg, P_a, g, sh);
    if (!(g[0] > 0.0) || !isfinite(g[0])) return;  // the G^T-kernel reports the breakdown
    al = (TV)(S.delta / g[0]);
  }
  double part[1] = {0.0};
  const Sched sc = sched(A.nblk);
  auto pre = [&](int row) { return RowVals<TV>{b[row], (TV)0, (TV)0}; };
  auto epi = [&](int row, TV sum, const RowVals<TV> &pv) {
    const TV rv = pv.a - sum;
    rout[row] = rv;
    part[0] += (double)rv * (double)rv;
  };
  if (with_d) {
    for (int k = sc.first; k < sc.end; k += sc.stride)
      stream_block<TV>(A, k, lds, pre, [&](int j) -> TV { return x[j] + al * dc[j]; }, epi);
  } else {
    for (int k = sc.first; k < sc.end; k += sc.stride)
      stream_block<TV>(A, k, lds, pre, [&](int j) -> TV { return x[j]; }, epi);
  }
  if (ptr) put_partials<1>(part, ptr, sc.L, sh);
}

template <typename TV>
__global__ __launch_bounds__(kBlock) void k_finalize(int32_t n, TV *__restrict__ x, const TV *__restrict__ d0,
                                                     const TV *__restrict__ d1, const State *__restrict__ st) {
  const TV al = (TV)st[0].alpha;
  if (al == (TV)0) return;
  const TV *__restrict__ dc = ((st[0].iter - 1) & 1) ? d1 : d0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    x[i] = x[i] + al * dc[i];
}

__global__ void k_state_clear_alpha(State *st) { st[0].alpha = 0.0; }

__global__ void k_state_restart(State *st) {
  st[0].done = 0;
  st[0].status = ST_RUNNING;
  st[0].alpha = 0.0;
  st[0].beta = 0.0;
}

template <typename TV>
__global__ __launch_bounds__(kBlock) void k_norm_b(int32_t n, const TV *__restrict__ b, double *__restrict__ pb) {
  __shared__ double sh[4 * (kBlock / 64)];
  double part[1] = {0.0};
  // logical id -> contiguous slice, so the sum order is fixed
  const int G = gridDim.x, L = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  const int64_t i0 = (int64_t)L * n / G, i1 = (int64_t)(L + 1) * n / G;
#pragma unroll 8
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) part[0] += (double)b[i] * (double)b[i];
  put_partials<1>(part, pb, L, sh);
}

// Single workgroup: ||b||^2 (what = 0, also tol * ||b|| and the b = 0 test)
// or ||b - A x||^2 (what = 1) from P partials into st[0].
__global__ __launch_bounds__(kBlock) void k_reduce_state(const double *__restrict__ p, int P, State *st, int what) {
  __shared__ double sh[4 * (kBlock / 64)];
  double v[1];
  sum_partials<1>(p, P, v, sh);
  if (threadIdx.x != 0) return;
  if (what == 0) {
    st[0].bb = v[0];
    st[0].tol_nb = st[0].tol * sqrt(v[0]);
    if (v[0] == 0.0) {
      st[0].status = ST_ZERO_B;
      st[0].done = 1;
    }
  } else {
    st[0].true_rr = v[0];
  }
}

template <typename TV, typename TM>
__global__ __launch_bounds__(kBlock) void k_spmv(Mat<TM> M, const TV *__restrict__ x, TV *__restrict__ y) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  const Sched sc = sched(M.nblk);
  for (int b = sc.first; b < sc.end; b += sc.stride)
    stream_block<TV>(
        M, b, lds, [&](int) { return RowVals<TV>{}; }, [&](int j) -> TV { return x[j]; },
        [&](int row, TV sum, const RowVals<TV> &) { y[row] = sum; });
}

template <typename TV>
__global__ void k_axpby(int32_t n, TV a, TV *__restrict__ y, TV b, const TV *__restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * y[i] + b * x[i];
}

template <typename TS, typename TD>
__global__ void k_convert(const TS *__restrict__ src, TD *__restrict__ dst, int64_t n, double scale) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (TD)(scale * (double)src[i]);
}

template <typename T>
__global__ void k_fill(T *__restrict__ p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename TC>
__global__ void k_refine_update(int32_t n, double *__restrict__ x64, const TC *__restrict__ c, double scale) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x64[i] = x64[i] + scale * (double)c[i];
}

// Plain streaming copy (16-byte accesses): the reference for the HBM ceiling
// and for calibrating the memory-traffic counters.
__global__ __launch_bounds__(kBlock) void k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n16; i += (int64_t)gridDim.x * kBlock)
    dst[i] = src[i];
}

// ---------------------------------------------------------------- launchers

static inline int ew_grid(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 4096) g = 4096;
  return (int)(g < 1 ? 1 : g);
}

#define PCG_DISPATCH_G(gdt, TG, ...)                          \
  switch (gdt) {                                              \
    case F64: { using TG = double; __VA_ARGS__; break; }      \
    case F32: { using TG = float; __VA_ARGS__; break; }       \
    case BF16: { using TG = bf16_t; __VA_ARGS__; break; }     \
    case F16: { using TG = _Float16; __VA_ARGS__; break; }    \
    default: return hipErrorInvalidValue;                     \
  }

#define PCG_DISPATCH_V(vdt, TV, ...)                          \
  switch (vdt) {                                              \
    case F64: { using TV = double; __VA_ARGS__; break; }      \
    case F32: { using TV = float; __VA_ARGS__; break; }       \
    default: return hipErrorInvalidValue;                     \
  }

hipError_t launch_iter_A(const Types &ty, const DevCSR &A, const Vecs &v, State *st, const Partials &p,
                         hipStream_t s) {
  if (ty.vec == F64 && A.dtype == F64) {
    hipLaunchKernelGGL((k_iter_A<double, double>), dim3(A.grid), dim3(kBlock), 0, s, mat<double>(A), (double *)v.x,
                       (const double *)v.s, (double *)v.d0, (double *)v.d1, (double *)v.q, st, p.g);
  } else if (ty.vec == F32 && A.dtype == F32) {
    hipLaunchKernelGGL((k_iter_A<float, float>), dim3(A.grid), dim3(kBlock), 0, s, mat<float>(A), (float *)v.x,
                       (const float *)v.s, (float *)v.d0, (float *)v.d1, (float *)v.q, st, p.g);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_iter_GT(const Types &ty, const DevCSR &GT, const Vecs &v, State *st, const Partials &p, int P_a,
                          int mode, hipStream_t s) {
  PCG_DISPATCH_V(ty.vec, TV, PCG_DISPATCH_G(GT.dtype, TG, {
    hipLaunchKernelGGL((k_iter_GT<TV, TG>), dim3(GT.grid), dim3(kBlock), 0, s, mat<TG>(GT), (TV *)v.r0,
                       (TV *)v.r1, (const TV *)v.q, (TV *)v.t, st, p.g, P_a, p.rt, mode);
  }));
  return hipGetLastError();
}

hipError_t launch_iter_G(const Types &ty, const DevCSR &G, const Vecs &v, State *st, const Partials &p, int P_gt,
                         bool has_eps, int mode, hipStream_t s) {
  PCG_DISPATCH_V(ty.vec, TV, PCG_DISPATCH_G(G.dtype, TG, {
    if (has_eps)
      hipLaunchKernelGGL((k_iter_G<TV, TG, true>), dim3(G.grid), dim3(kBlock), 0, s, mat<TG>(G), (const TV *)v.t,
                         (const TV *)v.r0, (const TV *)v.r1, (TV *)v.s, st, p.rt, P_gt, mode);
    else
      hipLaunchKernelGGL((k_iter_G<TV, TG, false>), dim3(G.grid), dim3(kBlock), 0, s, mat<TG>(G), (const TV *)v.t,
                         (const TV *)v.r0, (const TV *)v.r1, (TV *)v.s, st, p.rt, P_gt, mode);
  }));
  return hipGetLastError();
}

hipError_t launch_resid(const Types &ty, const DevCSR &A, const Vecs &v, State *st, const Partials &p, int slot_sel,
                        bool with_d, bool reduce, bool respect_done, hipStream_t s) {
  double *ptr = reduce ? p.tr : nullptr;
  if (ty.vec == F64 && A.dtype == F64) {
    hipLaunchKernelGGL((k_resid<double, double>), dim3(A.grid), dim3(kBlock), 0, s, mat<double>(A),
                       (const double *)v.b, (const double *)v.x, (const double *)v.d0, (const double *)v.d1,
                       (double *)v.r0, (double *)v.r1, st, p.g, A.grid, ptr, slot_sel, (int)with_d,
                       (int)respect_done);
  } else if (ty.vec == F32 && A.dtype == F32) {
    hipLaunchKernelGGL((k_resid<float, float>), dim3(A.grid), dim3(kBlock), 0, s, mat<float>(A),
                       (const float *)v.b, (const float *)v.x, (const float *)v.d0, (const float *)v.d1,
                       (float *)v.r0, (float *)v.r1, st, p.g, A.grid, ptr, slot_sel, (int)with_d,
                       (int)respect_done);
  } else {
    return hipErrorInvalidValue;
  }
  if (reduce) hipLaunchKernelGGL(k_reduce_state, dim3(1), dim3(kBlock), 0, s, (const double *)p.tr, A.grid, st, 1);
  return hipGetLastError();
}

hipError_t launch_reduce_true(State *st, const Partials &p, int P, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_state, dim3(1), dim3(kBlock), 0, s, (const double *)p.tr, P, st, 1);
  return hipGetLastError();
}

hipError_t launch_finalize(const Types &ty, int32_t n, const Vecs &v, State *st, hipStream_t s) {
  PCG_DISPATCH_V(ty.vec, TV, {
    hipLaunchKernelGGL((k_finalize<TV>), dim3(ew_grid(n)), dim3(kBlock), 0, s, n, (TV *)v.x, (const TV *)v.d0,
                       (const TV *)v.d1, st);
  });
  hipLaunchKernelGGL(k_state_clear_alpha, dim3(1), dim3(1), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_norm_b(const Types &ty, int32_t n, const Vecs &v, State *st, const Partials &p, hipStream_t s) {
  // the grid must stay within the partial buffers (sized for at least 1024)
  int g = ew_grid(n);
  if (g > 1024) g = 1024;
  g = (g + 7) & ~7;
  PCG_DISPATCH_V(ty.vec, TV, {
    hipLaunchKernelGGL((k_norm_b<TV>), dim3(g), dim3(kBlock), 0, s, n, (const TV *)v.b, p.b);
  });
  hipLaunchKernelGGL(k_reduce_state, dim3(1), dim3(kBlock), 0, s, (const double *)p.b, g, st, 0);
  return hipGetLastError();
}

hipError_t launch_state_restart(State *st, hipStream_t s) {
  hipLaunchKernelGGL(k_state_restart, dim3(1), dim3(1), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_spmv(const Types &ty, const DevCSR &M, int mdtype, const void *x, void *y, hipStream_t s) {
  PCG_DISPATCH_V(ty.vec, TV, PCG_DISPATCH_G(mdtype, TM, {
    hipLaunchKernelGGL((k_spmv<TV, TM>), dim3(M.grid), dim3(kBlock), 0, s, mat<TM>(M), (const TV *)x, (TV *)y);
  }));
  return hipGetLastError();
}

hipError_t launch_axpby(int vec_dtype, int32_t n, double a, void *y, double b, const void *x, hipStream_t s) {
  PCG_DISPATCH_V(vec_dtype, TV, {
    hipLaunchKernelGGL((k_axpby<TV>), dim3(ew_grid(n)), dim3(kBlock), 0, s, n, (TV)a, (TV *)y, (TV)b,
                       (const TV *)x);
  });
  return hipGetLastError();
}

hipError_t launch_convert(int src_dtype, const void *src, int dst_dtype, void *dst, int64_t n, double scale,
                          hipStream_t s) {
  PCG_DISPATCH_V(src_dtype, TS, PCG_DISPATCH_V(dst_dtype, TD, {
    hipLaunchKernelGGL((k_convert<TS, TD>), dim3(ew_grid(n)), dim3(kBlock), 0, s, (const TS *)src, (TD *)dst, n,
                       scale);
  }));
  return hipGetLastError();
}

hipError_t launch_fill(int dtype, void *p, int64_t n, double value, hipStream_t s) {
  PCG_DISPATCH_V(dtype, TV, {
    hipLaunchKernelGGL((k_fill<TV>), dim3(ew_grid(n)), dim3(kBlock), 0, s, (TV *)p, n, (TV)value);
  });
  return hipGetLastError();
}

hipError_t launch_refine_update(int32_t n, double *x64, const void *c, int c_dtype, double scale, hipStream_t s) {
  PCG_DISPATCH_V(c_dtype, TC, {
    hipLaunchKernelGGL((k_refine_update<TC>), dim3(ew_grid(n)), dim3(kBlock), 0, s, n, x64, (const TC *)c, scale);
  });
  return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, int64_t bytes, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kBlock), 0, s, (const uint4 *)src, (uint4 *)dst, bytes / 16);
  return hipGetLastError();
}

}  // namespace pcgk
