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
// Reductions are deterministic: each workgroup reduces its rows with wave
// shuffles and LDS, writes one partial, and the last workgroup to arrive
// (arrival counter) adds the partials in a fixed order and updates the
// scalars in device memory. Workgroups are mapped so that each of the 8
// XCDs processes one contiguous eighth of the rows, keeping the gathered
// neighbourhoods inside that XCD's L2.
//
// Built with floating-point contraction off: every product and sum rounds
// separately, in the order written (rows summed left to right from zero),
// which is also the order of the plain CSR definition.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace pcgk {

struct bf16_t { uint16_t bits; };

__device__ __forceinline__ double ldval(const double *p, int64_t k) { return p[k]; }
__device__ __forceinline__ float ldval(const float *p, int64_t k) { return p[k]; }
__device__ __forceinline__ float ldval(const bf16_t *p, int64_t k) {
  return __uint_as_float((uint32_t)p[k].bits << 16);
}
__device__ __forceinline__ float ldval(const _Float16 *p, int64_t k) { return (float)p[k]; }

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

// One row block: stage products in LDS, sum each row in CSR order.
template <typename TACC, typename TM, typename Gather, typename Epi>
__device__ __forceinline__ void stream_block(int r0, int r1, const Mat<TM> &M, TACC *lds, Gather gather, Epi epi) {
  constexpr int cap = kLdsBytes / (int)sizeof(TACC);
  const int tid = threadIdx.x;
  const int k0 = M.rp[r0], k1 = M.rp[r1];
  if (k1 - k0 <= cap) {
#pragma unroll 4
    for (int k = k0 + tid; k < k1; k += kBlock) lds[k - k0] = (TACC)ldval(M.val, k) * gather(M.ci[k]);
    __syncthreads();
    const int row = r0 + tid;
    if (row < r1) {
      const int a = M.rp[row] - k0, e = M.rp[row + 1] - k0;
      TACC sum = 0;
      for (int k = a; k < e; ++k) sum += lds[k];
      epi(row, sum);
    }
    __syncthreads();
  } else {
    // a single row longer than the LDS window: chunks, summed in order by thread 0
    TACC sum = 0;
    for (int c0 = k0; c0 < k1; c0 += cap) {
      const int c1 = min(c0 + cap, k1);
      for (int k = c0 + tid; k < c1; k += kBlock) lds[k - c0] = (TACC)ldval(M.val, k) * gather(M.ci[k]);
      __syncthreads();
      if (tid == 0)
        for (int k = 0; k < c1 - c0; ++k) sum += lds[k];
      __syncthreads();
    }
    if (tid == 0) epi(r0, sum);
  }
}

// Row blocks [bstart, bend) of logical workgroup L out of G.
__device__ __forceinline__ void my_blocks(int nblk, int &bstart, int &bend) {
  const int G = gridDim.x;
  const int L = xcd_remap(blockIdx.x, G);
  bstart = (int)((int64_t)L * nblk / G);
  bend = (int)((int64_t)(L + 1) * nblk / G);
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

// Reduce v over the grid. Returns true in the last-arriving workgroup, where
// thread 0 then holds the grid totals (added in a fixed order).
template <int NV>
__device__ __forceinline__ bool grid_sum(double (&v)[NV], double *partials, uint32_t *ctr, double *sh) {
  __shared__ int is_last;
  const int G = gridDim.x;
  const int L = xcd_remap(blockIdx.x, G);
  block_sum<NV>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) partials[(int64_t)j * G + L] = v[j];
    __threadfence();
    const uint32_t prev = atomicAdd(ctr, 1u);
    is_last = (prev == (uint32_t)G - 1);
  }
  __syncthreads();
  if (!is_last) return false;
  __threadfence();
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  for (int k = threadIdx.x; k < G; k += kBlock)
#pragma unroll
    for (int j = 0; j < NV; ++j)
      acc[j] += __hip_atomic_load(&partials[(int64_t)j * G + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  block_sum<NV>(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = acc[j];
    *ctr = 0u;
  }
  return true;
}

// ------------------------------------------------------------------ kernels

template <typename TV, typename TA>
__global__ __launch_bounds__(kBlock) void k_iter_A(Mat<TA> A, TV *__restrict__ x, const TV *__restrict__ s,
                                                   TV *__restrict__ d0, TV *__restrict__ d1, TV *__restrict__ q,
                                                   State *__restrict__ st, double *__restrict__ partials) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  __shared__ double sh[4 * (kBlock / 64)];
  if (st->done) return;
  const int it = st->iter;
  const TV beta = (TV)st->beta, ap = (TV)st->alpha;
  const TV *__restrict__ dold = (it & 1) ? d0 : d1;  // d_{i-1}
  TV *__restrict__ dnew = (it & 1) ? d1 : d0;        // d_i
  double part[1] = {0.0};
  int b0, b1;
  my_blocks(A.nblk, b0, b1);
  for (int b = b0; b < b1; ++b)
    stream_block<TV>(
        A.blk[b], A.blk[b + 1], A, lds, [&](int j) -> TV { return s[j] + beta * dold[j]; },
        [&](int row, TV sum) {
          const TV dold_r = dold[row];
          const TV di = s[row] + beta * dold_r;
          dnew[row] = di;
          q[row] = sum;
          x[row] = x[row] + ap * dold_r;
          part[0] += (double)di * (double)sum;
        });
  if (grid_sum<1>(part, partials, &st->ctr[0], sh) && threadIdx.x == 0) {
    const double g = part[0];
    st->gamma = g;
    if (!(g > 0.0) || !isfinite(g)) {
      st->status = ST_BREAK_GAMMA;
      st->done = 1;
      st->alpha = 0.0;  // x already holds x_i
    } else {
      st->alpha = st->delta / g;
    }
  }
}

template <typename TV, typename TG>
__global__ __launch_bounds__(kBlock) void k_iter_GT(Mat<TG> GT, TV *__restrict__ r0, TV *__restrict__ r1,
                                                    const TV *__restrict__ q, TV *__restrict__ t,
                                                    State *__restrict__ st, double *__restrict__ partials,
                                                    int mode) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  __shared__ double sh[4 * (kBlock / 64)];
  if (st->done) return;
  const int it = st->iter;
  const TV al = (mode == 0) ? (TV)st->alpha : (TV)0;
  const TV *__restrict__ src = (((mode == 1) ? it + 1 : it) & 1) ? r1 : r0;
  TV *__restrict__ dst = ((it + 1) & 1) ? r1 : r0;
  double part[2] = {0.0, 0.0};
  int b0, b1;
  my_blocks(GT.nblk, b0, b1);
  if (mode == 0) {
    for (int b = b0; b < b1; ++b)
      stream_block<TV>(
          GT.blk[b], GT.blk[b + 1], GT, lds, [&](int j) -> TV { return src[j] - al * q[j]; },
          [&](int row, TV sum) {
            const TV rn = src[row] - al * q[row];
            dst[row] = rn;
            t[row] = sum;
            part[0] += (double)rn * (double)rn;
            part[1] += (double)sum * (double)sum;
          });
  } else {
    for (int b = b0; b < b1; ++b)
      stream_block<TV>(
          GT.blk[b], GT.blk[b + 1], GT, lds, [&](int j) -> TV { return src[j]; },
          [&](int row, TV sum) {
            const TV rn = src[row];
            t[row] = sum;
            part[0] += (double)rn * (double)rn;
            part[1] += (double)sum * (double)sum;
          });
  }
  if (grid_sum<2>(part, partials, &st->ctr[1], sh) && threadIdx.x == 0) {
    const double rr = part[0], tt = part[1];
    st->rr = rr;
    st->tt = tt;
    const double dn = tt + st->eps * rr;
    const int i1 = (mode == 2) ? it : it + 1;
    st->iter = i1;
    if (mode != 2 && (!(dn >= 0.0) || !isfinite(dn))) {
      st->status = ST_BREAK_DELTA;
      st->done = 1;
    } else {
      st->beta = (mode == 2) ? 0.0 : dn / st->delta;
      st->delta = dn;
      if (sqrt(rr) <= st->tol_nb) {
        st->status = ST_CONV_REC;
        st->done = 1;
      } else if (i1 >= st->maxit) {
        st->status = ST_MAXIT;
        st->done = 1;
      }
    }
  }
}

template <typename TV, typename TG, bool HAS_EPS>
__global__ __launch_bounds__(kBlock) void k_iter_G(Mat<TG> G, const TV *__restrict__ t, const TV *__restrict__ r0,
                                                   const TV *__restrict__ r1, TV *__restrict__ s,
                                                   State *__restrict__ st) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  if (st->done) return;
  const int it = st->iter;
  const TV *__restrict__ rc = (it & 1) ? r1 : r0;
  const TV eps = (TV)st->eps;
  int b0, b1;
  my_blocks(G.nblk, b0, b1);
  for (int b = b0; b < b1; ++b)
    stream_block<TV>(
        G.blk[b], G.blk[b + 1], G, lds, [&](int j) -> TV { return t[j]; },
        [&](int row, TV sum) {
          if (HAS_EPS)
            s[row] = sum + eps * rc[row];
          else
            s[row] = sum;
        });
}

template <typename TV, typename TA>
__global__ __launch_bounds__(kBlock) void k_resid(Mat<TA> A, const TV *__restrict__ b, const TV *__restrict__ x,
                                                  const TV *__restrict__ d0, const TV *__restrict__ d1,
                                                  TV *__restrict__ r0, TV *__restrict__ r1, State *__restrict__ st,
                                                  double *__restrict__ partials, int slot_sel, int with_d,
                                                  int reduce, int respect_done) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  __shared__ double sh[4 * (kBlock / 64)];
  if (respect_done && st->done) return;
  const int it = st->iter;
  TV *__restrict__ rout = ((it + slot_sel) & 1) ? r1 : r0;
  const TV *__restrict__ dc = (it & 1) ? d1 : d0;  // d_i
  const TV al = (TV)st->alpha;
  double part[1] = {0.0};
  int b0, b1;
  my_blocks(A.nblk, b0, b1);
  auto epi = [&](int row, TV sum) {
    const TV rv = b[row] - sum;
    rout[row] = rv;
    part[0] += (double)rv * (double)rv;
  };
  if (with_d) {
    for (int k = b0; k < b1; ++k)
      stream_block<TV>(A.blk[k], A.blk[k + 1], A, lds, [&](int j) -> TV { return x[j] + al * dc[j]; }, epi);
  } else {
    for (int k = b0; k < b1; ++k)
      stream_block<TV>(A.blk[k], A.blk[k + 1], A, lds, [&](int j) -> TV { return x[j]; }, epi);
  }
  if (reduce && grid_sum<1>(part, partials, &st->ctr[3], sh) && threadIdx.x == 0) st->true_rr = part[0];
}

template <typename TV>
__global__ __launch_bounds__(kBlock) void k_finalize(int32_t n, TV *__restrict__ x, const TV *__restrict__ d0,
                                                     const TV *__restrict__ d1, const State *__restrict__ st) {
  const TV al = (TV)st->alpha;
  if (al == (TV)0) return;
  const TV *__restrict__ dc = ((st->iter - 1) & 1) ? d1 : d0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    x[i] = x[i] + al * dc[i];
}

__global__ void k_state_clear_alpha(State *st) { st->alpha = 0.0; }

__global__ void k_state_restart(State *st) {
  st->done = 0;
  st->status = ST_RUNNING;
  st->alpha = 0.0;
  st->beta = 0.0;
}

template <typename TV>
__global__ __launch_bounds__(kBlock) void k_norm_b(int32_t n, const TV *__restrict__ b, State *__restrict__ st,
                                                   double *__restrict__ partials) {
  __shared__ double sh[4 * (kBlock / 64)];
  double part[1] = {0.0};
  // logical id -> contiguous slice, so the sum order is fixed
  const int G = gridDim.x, L = xcd_remap(blockIdx.x, G);
  const int64_t i0 = (int64_t)L * n / G, i1 = (int64_t)(L + 1) * n / G;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) part[0] += (double)b[i] * (double)b[i];
  if (grid_sum<1>(part, partials, &st->ctr[2], sh) && threadIdx.x == 0) {
    const double bb = part[0];
    st->bb = bb;
    const double nb = sqrt(bb);
    st->tol_nb = st->tol * nb;
    if (bb == 0.0) {
      st->status = ST_ZERO_B;
      st->done = 1;
    }
  }
}

template <typename TV, typename TM>
__global__ __launch_bounds__(kBlock) void k_spmv(Mat<TM> M, const TV *__restrict__ x, TV *__restrict__ y) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  int b0, b1;
  my_blocks(M.nblk, b0, b1);
  for (int b = b0; b < b1; ++b)
    stream_block<TV>(M.blk[b], M.blk[b + 1], M, lds, [&](int j) -> TV { return x[j]; },
                     [&](int row, TV sum) { y[row] = sum; });
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

hipError_t launch_iter_A(const Types &ty, const DevCSR &A, const Vecs &v, State *st, double *partials,
                         hipStream_t s) {
  if (ty.vec == F64 && A.dtype == F64) {
    hipLaunchKernelGGL((k_iter_A<double, double>), dim3(A.grid), dim3(kBlock), 0, s, mat<double>(A), (double *)v.x,
                       (const double *)v.s, (double *)v.d0, (double *)v.d1, (double *)v.q, st, partials);
  } else if (ty.vec == F32 && A.dtype == F32) {
    hipLaunchKernelGGL((k_iter_A<float, float>), dim3(A.grid), dim3(kBlock), 0, s, mat<float>(A), (float *)v.x,
                       (const float *)v.s, (float *)v.d0, (float *)v.d1, (float *)v.q, st, partials);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_iter_GT(const Types &ty, const DevCSR &GT, const Vecs &v, State *st, double *partials, int mode,
                          hipStream_t s) {
  PCG_DISPATCH_V(ty.vec, TV, PCG_DISPATCH_G(GT.dtype, TG, {
    hipLaunchKernelGGL((k_iter_GT<TV, TG>), dim3(GT.grid), dim3(kBlock), 0, s, mat<TG>(GT), (TV *)v.r0,
                       (TV *)v.r1, (const TV *)v.q, (TV *)v.t, st, partials, mode);
  }));
  return hipGetLastError();
}

hipError_t launch_iter_G(const Types &ty, const DevCSR &G, const Vecs &v, State *st, bool has_eps, hipStream_t s) {
  PCG_DISPATCH_V(ty.vec, TV, PCG_DISPATCH_G(G.dtype, TG, {
    if (has_eps)
      hipLaunchKernelGGL((k_iter_G<TV, TG, true>), dim3(G.grid), dim3(kBlock), 0, s, mat<TG>(G), (const TV *)v.t,
                         (const TV *)v.r0, (const TV *)v.r1, (TV *)v.s, st);
    else
      hipLaunchKernelGGL((k_iter_G<TV, TG, false>), dim3(G.grid), dim3(kBlock), 0, s, mat<TG>(G), (const TV *)v.t,
                         (const TV *)v.r0, (const TV *)v.r1, (TV *)v.s, st);
  }));
  return hipGetLastError();
}

hipError_t launch_resid(const Types &ty, const DevCSR &A, const Vecs &v, State *st, double *partials, int slot_sel,
                        bool with_d, bool reduce, bool respect_done, hipStream_t s) {
  if (ty.vec == F64 && A.dtype == F64) {
    hipLaunchKernelGGL((k_resid<double, double>), dim3(A.grid), dim3(kBlock), 0, s, mat<double>(A),
                       (const double *)v.b, (const double *)v.x, (const double *)v.d0, (const double *)v.d1,
                       (double *)v.r0, (double *)v.r1, st, partials, slot_sel, (int)with_d, (int)reduce,
                       (int)respect_done);
  } else if (ty.vec == F32 && A.dtype == F32) {
    hipLaunchKernelGGL((k_resid<float, float>), dim3(A.grid), dim3(kBlock), 0, s, mat<float>(A),
                       (const float *)v.b, (const float *)v.x, (const float *)v.d0, (const float *)v.d1,
                       (float *)v.r0, (float *)v.r1, st, partials, slot_sel, (int)with_d, (int)reduce,
                       (int)respect_done);
  } else {
    return hipErrorInvalidValue;
  }
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

hipError_t launch_norm_b(const Types &ty, int32_t n, const Vecs &v, State *st, double *partials, hipStream_t s) {
  // the grid must stay within the partial buffer sized for the matrices' grids
  int g = ew_grid(n);
  if (g > 1024) g = 1024;
  g = (g + 7) & ~7;
  PCG_DISPATCH_V(ty.vec, TV, {
    hipLaunchKernelGGL((k_norm_b<TV>), dim3(g), dim3(kBlock), 0, s, n, (const TV *)v.b, st, partials);
  });
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

}  // namespace pcgk
