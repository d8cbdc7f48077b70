// gfx950 kernels for preconditioned CG with M^-1 = G G^T + eps I.
//
// Every operator product is a sparse matrix-vector product in one of three
// layouts (DevCSR): sliced ELL (a wave owns slices of 64 rows, one lane per
// row, coalesced column and value loads, 32- or 16-bit column indices),
// sliced 3x3 blocks (one index per block), or CSR row blocks (a workgroup
// stages the products of a block of rows in LDS, then one thread per row
// adds them). In every layout each row's products are added left to right
// from zero in CSR order. Matrix loads are nontemporal, or ordinary for a
// matrix kept resident in the memory-side cache (DevCSR::temporal). The A,
// G^T and G products carry the CG vector updates in their gathers and
// epilogues, so one iteration is three launches:
//   A-kernel : q = A d_i,  partials of gamma = d_i^T q;
//   G^T-kernel: alpha_i = delta_i / gamma,
//              r_{i+1} = r_i - alpha_i q  (formed where it is gathered),
//              t = G^T r_{i+1}, partials of ||r||^2, ||t||^2;
//   G-kernel : delta_{i+1} = ||t||^2 + eps ||r||^2 (= r^T M^-1 r),
//              beta_{i+1} = delta_{i+1} / delta_i, convergence test,
//              x_{i+1} = x_i + alpha_i d_i (also on the last iteration),
//              d_{i+1} = (G t + eps r_{i+1}) + beta_{i+1} d_i.
// That is 11 vector streams of n entries per iteration: A reads d, writes
// q; G^T reads r and q, writes r and t; G reads t, d and x, writes x and d.
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
// contiguous eighth of the slices (or row blocks), and its workgroups take
// them interleaved, so at any moment an XCD works on one window of
// consecutive rows whose gathered neighbourhoods stay in that XCD's L2.
//
// Built with floating-point contraction off: every product and sum rounds
// separately, in the order written (rows summed left to right from zero),
// which is also the order of the plain CSR definition.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "kernels.h"

namespace pcgk {

// The SpMV kernels are memory-latency bound: they are compiled for 8 waves
// per SIMD (at most 64 VGPRs, checked free of scratch spills), which keeps
// twice the loads in flight of the 4-6 waves the compiler otherwise picks.
#ifndef PCG_WAVES_PER_EU
#define PCG_WAVES_PER_EU 8
#endif
#define PCG_OCCUPANCY __attribute__((amdgpu_waves_per_eu(PCG_WAVES_PER_EU)))
// The G^T-kernel takes two rows per lane over sliced diagonals (twice the
// operands per lane): compiled for 4 waves per SIMD (at most 128 VGPRs, no
// spills), the occupancy its default grid of 4 workgroups of 4 waves per CU
// gives anyway.
#define PCG_GT_OCCUPANCY __attribute__((amdgpu_waves_per_eu(4)))
// The G-kernel takes two rows per lane over sliced diagonals too and holds
// its first slice pair's operands while its workgroup reduces the partial
// sums of the G^T-kernel: compiled for 4 waves per SIMD like the G^T-kernel.
#define PCG_G_OCCUPANCY __attribute__((amdgpu_waves_per_eu(4)))

#ifndef PCG_UNROLL
#define PCG_UNROLL 4
#endif

struct bf16_t { uint16_t bits; };

// Pointers that come out of the device directory are not known to the
// compiler to address global memory, and accesses through them compile to
// flat instructions, which also count on the LDS wait counter and so stall
// every LDS wait of the staging loop behind outstanding gathers. Kernels
// therefore take every directory pointer into the global address space.
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T *gl(T *p) {
  return (GLOBAL T *)p;
}

// Layout metadata that a whole wave reads at one address (slice pointers,
// per-slice column offsets) is read through the constant address space, so
// that those reads compile to scalar loads: they wait on their own counter
// instead of behind the wave's outstanding vector loads and stores. Valid
// because no kernel writes a layout's metadata while it is being read.
#define CONSTANT __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ CONSTANT const T *ro(GLOBAL const T *p) {
  return (CONSTANT const T *)p;
}

// Matrix values and column indices are read once per product. NT = true:
// nontemporal loads, which stream past the caches (they neither displace the
// gathered vector entries in L2 nor stay in the memory-side cache); NT =
// false: ordinary loads, for a matrix meant to stay resident in the 256 MB
// memory-side cache from one iteration to the next (DevCSR::temporal).
template <bool NT = true, typename T>
__device__ __forceinline__ T ldstream(GLOBAL const T *p, int64_t k) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p + k);
  else
    return p[k];
}

template <bool NT = true>
__device__ __forceinline__ double ldval(GLOBAL const double *p, int64_t k) {
  return ldstream<NT>(p, k);
}
template <bool NT = true>
__device__ __forceinline__ float ldval(GLOBAL const float *p, int64_t k) {
  return ldstream<NT>(p, k);
}
template <bool NT = true>
__device__ __forceinline__ float ldval(GLOBAL const bf16_t *p, int64_t k) {
  return __uint_as_float((uint32_t)ldstream<NT>((GLOBAL const uint16_t *)p, k) << 16);
}
template <bool NT = true>
__device__ __forceinline__ float ldval(GLOBAL const _Float16 *p, int64_t k) {
  return (float)ldstream<NT>(p, k);
}

// Whole-record copies of a State (one thread publishes a slot), in 16-byte
// words of a builtin vector type (usable in any address space).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ State ld_state(GLOBAL const State *p) {
  constexpr int W = (int)(sizeof(State) / 16);
  u32x4 w[W];
  GLOBAL const u32x4 *q = (GLOBAL const u32x4 *)p;
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = q[i];
  State o;
  __builtin_memcpy(&o, w, sizeof(State));
  return o;
}

__device__ __forceinline__ void st_state(GLOBAL State *p, const State &o) {
  constexpr int W = (int)(sizeof(State) / 16);
  u32x4 w[W];
  __builtin_memcpy(w, &o, sizeof(State));
  GLOBAL u32x4 *q = (GLOBAL u32x4 *)p;
#pragma unroll
  for (int i = 0; i < W; ++i) q[i] = w[i];
}

template <typename TM>
struct Mat {
  GLOBAL const int32_t *rp;
  GLOBAL const int32_t *ci;
  GLOBAL const TM *val;
  GLOBAL const int32_t *blk;
  int32_t nblk;
  int32_t n;
  int32_t fmt;
  int32_t idx16;
  int32_t temporal;
  int32_t rpl;
};

template <typename TM>
__device__ __forceinline__ Mat<TM> mat(const DevCSR &m) {
  return Mat<TM>{gl(m.rp), gl(m.ci), gl((const TM *)m.val), gl(m.blk), m.nblk, m.n, m.fmt, m.idx16, m.temporal,
                 m.rpl};
}

// Column of stored entry q of `row`: an absolute int32 index, or (sliced
// layouts with 16-bit indices) an int16 difference from the row.
template <typename TI>
__device__ __forceinline__ int32_t col_at(GLOBAL const int32_t *ci, int64_t q, int32_t row) {
  if constexpr (sizeof(TI) == 2)
    return row + (int32_t)((GLOBAL const int16_t *)ci)[q];
  else
    return ci[q];
}

// Operands of one row loaded before the row's products are staged.
template <typename TV>
struct RowVals {
  TV a, b, c;
};

// Sum of lds[a..e) added left to right onto s0; eight reads are issued ahead
// of their adds, so long rows are not one LDS round trip per entry.
template <typename TACC>
__device__ __forceinline__ TACC lds_row_sum(const TACC *lds, int a, int e, TACC s0 = 0) {
  TACC sum = s0;
  int k = a;
  for (; k + 8 <= e; k += 8) {
    TACC v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = lds[k + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) sum += v[u];
  }
  for (; k < e; ++k) sum += lds[k];
  return sum;
}

// One row block: stage products in LDS, sum each row in CSR order. `pre(row)`
// loads the row's own operands early (overlapping the gathers), `epi(row,
// sum, pre_values)` consumes the row's sum.
template <typename TACC, bool NT, typename TM, typename Pre, typename Gather, typename Epi>
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
    for (int k = k0 + tid; k < k1; k += kBlock)
      lds[k - k0] = (TACC)ldval<NT>(M.val, k) * gather(ldstream<NT>(M.ci, k));
    __syncthreads();
    if (has) epi(row, lds_row_sum(lds, a, e), pv);
    __syncthreads();
  } else {
    // a single row longer than the LDS window: chunks, summed in order by thread 0
    RowVals<TACC> pv{};
    if (tid == 0) pv = pre(r0);
    TACC sum = 0;
    for (int c0 = k0; c0 < k1; c0 += cap) {
      const int c1 = min(c0 + cap, k1);
      for (int k = c0 + tid; k < c1; k += kBlock)
        lds[k - c0] = (TACC)ldval<NT>(M.val, k) * gather(ldstream<NT>(M.ci, k));
      __syncthreads();
      if (tid == 0) sum = lds_row_sum(lds, 0, c1 - c0, sum);
      __syncthreads();
    }
    if (tid == 0) epi(r0, sum, pv);
  }
}

// This workgroup's row blocks: first, first + stride, ... < end; L is its
// logical index (the slot of its partial sums). l is the workgroup's index
// among its system's G workgroups (G and the system's first workgroup are
// multiples of 8, so l % 8 is the XCD the workgroup runs on).
struct Sched {
  int first, end, stride, L;
};

__device__ __forceinline__ Sched sched(int nblk, int l, int G) {
  const int W = G >> 3, x = l & 7, w = l >> 3;
  Sched sc;
  sc.first = (int)((int64_t)x * nblk / 8) + w;
  sc.end = (int)((int64_t)(x + 1) * nblk / 8);
  sc.stride = W;
  sc.L = x * W + w;
  return sc;
}

// Slot of this workgroup's partial sums (the same for both layouts).
__device__ __forceinline__ int part_slot(int l, int G) { return (l & 7) * (G >> 3) + (l >> 3); }

// Column of a slice entry: an absolute int32 index, or an int16 difference
// from the lane's row.
template <bool NT>
__device__ __forceinline__ int32_t slice_col(GLOBAL const int32_t *cc, int64_t k, int32_t) {
  return ldstream<NT>(cc, k);
}
template <bool NT>
__device__ __forceinline__ int32_t slice_col(GLOBAL const int16_t *cc, int64_t k, int32_t row) {
  return row + (int32_t)ldstream<NT>(cc, k);
}

// One lane's row of a slice: products of its wd entries added left to right
// from zero, loads issued UNR at a time. The last wd % UNR entries form one
// more batch whose surplus loads repeat entry wd - 1 (in bounds) and whose
// surplus products are not added, so every load of a batch is in flight at
// once (wd is the same for the whole wave).
template <typename TACC, int UNR, bool NT, typename TM, typename TI, typename Gather>
__device__ __forceinline__ TACC slice_row_sum(GLOBAL const TM *vv, GLOBAL const TI *cc, int32_t row, int wd,
                                              Gather gather) {
  TACC sum = 0;
  int k = 0;
  for (; k + UNR <= wd; k += UNR) {
    TACC p[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      p[u] = (TACC)ldval<NT>(vv, (k + u) * kSliceRows) * gather(slice_col<NT>(cc, (k + u) * kSliceRows, row));
#pragma unroll
    for (int u = 0; u < UNR; ++u) sum += p[u];
  }
  const int rem = wd - k;
  if (rem > 0) {
    TACC p[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int e = k + min(u, rem - 1);
      p[u] = (TACC)ldval<NT>(vv, e * kSliceRows) * gather(slice_col<NT>(cc, e * kSliceRows, row));
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      if (u < rem) sum += p[u];
  }
  return sum;
}

template <typename TACC, int UW, bool NT, typename TM, typename TI, typename Gather>
__device__ __forceinline__ TACC slice_row(GLOBAL const TM *vv, GLOBAL const TI *cc, int32_t row, int wd,
                                          Gather gather) {
  return (UW > 4 && wd > 4) ? slice_row_sum<TACC, UW, NT>(vv, cc, row, wd, gather)
                            : slice_row_sum<TACC, 4, NT>(vv, cc, row, wd, gather);
}

// Sliced-ELL rows: each wave takes whole slices (64 rows, one per lane); a
// lane loads its row's entries with coalesced loads across the slice, gathers,
// and adds the products left to right from zero, the CSR order. No LDS and no
// barrier. The XCD slab split is the one of the row blocks.
// UW: loads in flight per lane for rows longer than 4 entries (8 pays where a
// row product gathers one vector and the epilogue holds few operands; under
// the 64-register budget kernels with two gathers per entry do better with 4).
// REV: each die walks its range of slices from the top down.
template <typename TACC, int UW, bool NT, bool REV, typename TM, typename Pre, typename Gather, typename Epi>
__device__ __forceinline__ void sell_rows(const Mat<TM> &M, int l, int G, Pre pre, Gather gather, Epi epi) {
  constexpr int NW = kBlock / 64;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int W = G >> 3, x = l & 7, w = l >> 3;
  const int s0 = (int)((int64_t)x * M.nblk / 8), s1 = (int)((int64_t)(x + 1) * M.nblk / 8);
  for (int k = w * NW + wv; k < s1 - s0; k += W * NW) {
    const int c = REV ? s1 - 1 - k : s0 + k;
    const int o0 = ro(M.blk)[c], wd = ro(M.blk)[c + 1] - o0;
    const int row = c * kSliceRows + lane;
    const bool has = row < M.n;
    RowVals<TACC> pv{};
    if (has) pv = pre(row);
    const int64_t o = (int64_t)o0 * kSliceRows + lane;
    GLOBAL const TM *vv = M.val + o;
    const TACC sum = M.idx16 ? slice_row<TACC, UW, NT>(vv, (GLOBAL const int16_t *)M.ci + o, row, wd, gather)
                             : slice_row<TACC, UW, NT>(vv, M.ci + o, row, wd, gather);
    if (has) epi(row, sum, pv);
  }
}

// One lane's row of a sliced-diagonal slice: value k of the row multiplies
// the gathered entry at column row + off[k] (clamped into [0, n): a stored
// zero's column may fall outside), added left to right from zero; loads
// issued UNR at a time as in slice_row_sum. off[] is the same for the whole
// wave (scalar loads).
template <typename TACC, int UNR, bool NT, bool DIAG = false, typename TM, typename Gather>
__device__ __forceinline__ TACC sdia_row_sum(GLOBAL const TM *vv, CONSTANT const int32_t *off, int32_t row, int32_t nmax,
                                             int wd, Gather gather, TACC dg = 0) {
  // DIAG: dg is the operand at the row's own column (offset 0), already
  // loaded by the caller, so that entry is not gathered again
  auto operand = [&](int32_t o) -> TACC {
    if constexpr (DIAG) {
      if (o == 0) return dg;
    }
    return gather(min(max(row + o, 0), nmax));
  };
  TACC sum = 0;
  int k = 0;
  for (; k + UNR <= wd; k += UNR) {
    TACC p[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) p[u] = (TACC)ldval<NT>(vv, (k + u) * kSliceRows) * operand(off[k + u]);
#pragma unroll
    for (int u = 0; u < UNR; ++u) sum += p[u];
  }
  const int rem = wd - k;
  if (rem > 0) {
    TACC p[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int e = k + min(u, rem - 1);
      p[u] = (TACC)ldval<NT>(vv, e * kSliceRows) * operand(off[e]);
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      if (u < rem) sum += p[u];
  }
  return sum;
}

// Sliced-diagonal rows: the walk of sell_rows (whole slices per wave, one
// lane per row, each die's eighth of the slices), with one column offset per
// slice entry instead of one index per lane.
template <typename TACC, int UW, bool NT, bool REV, bool DIAG = false, typename TM, typename Pre, typename Gather,
          typename Epi>
__device__ __forceinline__ void sdia_rows(const Mat<TM> &M, int l, int G, Pre pre, Gather gather, Epi epi) {
  constexpr int NW = kBlock / 64;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int W = G >> 3, x = l & 7, w = l >> 3;
  const int s0 = (int)((int64_t)x * M.nblk / 8), s1 = (int)((int64_t)(x + 1) * M.nblk / 8);
  for (int k = w * NW + wv; k < s1 - s0; k += W * NW) {
    const int c = REV ? s1 - 1 - k : s0 + k;
    const int o0 = ro(M.blk)[c], wd = ro(M.blk)[c + 1] - o0;
    const int row = c * kSliceRows + lane;
    const bool has = row < M.n;
    RowVals<TACC> pv{};
    if (has) pv = pre(row);
    GLOBAL const TM *vv = M.val + (int64_t)o0 * kSliceRows + lane;
    const TACC sum = (UW > 4 && wd > 4)
                         ? sdia_row_sum<TACC, UW, NT, DIAG>(vv, ro(M.ci) + o0, row, M.n - 1, wd, gather, pv.a)
                         : sdia_row_sum<TACC, 4, NT, DIAG>(vv, ro(M.ci) + o0, row, M.n - 1, wd, gather, pv.a);
    if (has) epi(row, sum, pv);
  }
}

// sdia_rows with a workgroup step between the first slice's products and its
// epilogue: every wave calls hook() exactly once (after the loop when it has
// no slice), so hook may hold barriers; its result, the same in every thread,
// says whether the walk goes on. A kernel that needs a reduction before its
// epilogue (the G-kernel's beta) issues its first slice's loads and products
// under that reduction's latency instead of after it.
template <typename TACC, int UW, bool NT, bool REV, typename TM, typename Pre, typename Gather, typename Epi,
          typename Hook>
__device__ __forceinline__ bool sdia_rows_h(const Mat<TM> &M, int l, int G, Pre pre, Gather gather, Epi epi,
                                            Hook hook) {
  constexpr int NW = kBlock / 64;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int W = G >> 3, x = l & 7, w = l >> 3;
  const int s0 = (int)((int64_t)x * M.nblk / 8), s1 = (int)((int64_t)(x + 1) * M.nblk / 8);
  // the first slice is peeled so that what hook needs is dead in the loop
  auto slice = [&](int k, auto first) -> bool {
    const int c = REV ? s1 - 1 - k : s0 + k;
    const int o0 = ro(M.blk)[c], wd = ro(M.blk)[c + 1] - o0;
    const int row = c * kSliceRows + lane;
    const bool has = row < M.n;
    RowVals<TACC> pv{};
    if (has) pv = pre(row);
    GLOBAL const TM *vv = M.val + (int64_t)o0 * kSliceRows + lane;
    const TACC sum = (UW > 4 && wd > 4) ? sdia_row_sum<TACC, UW, NT>(vv, ro(M.ci) + o0, row, M.n - 1, wd, gather)
                                        : sdia_row_sum<TACC, 4, NT>(vv, ro(M.ci) + o0, row, M.n - 1, wd, gather);
    if constexpr (decltype(first)::value)
      if (!hook()) return false;
    if (has) epi(row, sum, pv);
    return true;
  };
  int k = w * NW + wv;
  if (k >= s1 - s0) return hook();
  if (!slice(k, std::true_type{})) return false;
  for (k += W * NW; k < s1 - s0; k += W * NW) slice(k, std::false_type{});
  return true;
}

// ---- two rows per lane over sliced diagonals
//
// Rows r and r + 1 of a slice read their operands at one offset o from the
// adjacent entries r + o and r + 1 + o, their values from adjacent slots,
// and write adjacent results: a lane that owns both rows makes one access of
// twice the width for each, half the memory instructions of one row per
// lane (gathers, the bulk of them, are unaligned 8- or 16-byte loads).

// Two adjacent entries of a vector (any alignment of the element type).
template <typename T>
struct Pair {
  T x, y;
};
template <typename T>
__device__ __forceinline__ Pair<T> ld_pair(GLOBAL const T *p, int64_t i) {
  Pair<T> v;
  __builtin_memcpy(&v, p + i, sizeof(v));
  return v;
}
template <typename T>
__device__ __forceinline__ void st_pair(GLOBAL T *p, int64_t i, T a, T b) {
  const Pair<T> v{a, b};
  __builtin_memcpy(p + i, &v, sizeof(v));
}

// The operands of rows r0 and r0 + 1 at column offset o, j0 = r0 + o: the
// entries at j0 and j0 + 1, each clamped into [0, n) as the one-row walk
// clamps it, from one load of [lo, lo + 1] (n >= 2).
template <typename T>
__device__ __forceinline__ Pair<T> gather_pair(GLOBAL const T *x, int32_t j0, int32_t n) {
  const int32_t lo = min(max(j0, 0), n - 2);
  const Pair<T> v = ld_pair(x, lo);
  return Pair<T>{j0 > n - 2 ? v.y : v.x, j0 < 0 ? v.x : v.y};
}

// Values of two adjacent slots (an even slot of a 64-slot slice entry:
// aligned to twice the value size), with the matrix's load policy.
typedef double v2f64 __attribute__((ext_vector_type(2)));
typedef float v2f32 __attribute__((ext_vector_type(2)));
typedef _Float16 v2f16 __attribute__((ext_vector_type(2)));
template <bool NT, typename V>
__device__ __forceinline__ V ld_aligned(GLOBAL const V *p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <bool NT, typename TACC>
__device__ __forceinline__ void ldval_pair(GLOBAL const double *p, int64_t k, TACC &a, TACC &b) {
  const v2f64 v = ld_aligned<NT>((GLOBAL const v2f64 *)(p + k));
  a = (TACC)v.x;
  b = (TACC)v.y;
}
template <bool NT, typename TACC>
__device__ __forceinline__ void ldval_pair(GLOBAL const float *p, int64_t k, TACC &a, TACC &b) {
  const v2f32 v = ld_aligned<NT>((GLOBAL const v2f32 *)(p + k));
  a = (TACC)v.x;
  b = (TACC)v.y;
}
template <bool NT, typename TACC>
__device__ __forceinline__ void ldval_pair(GLOBAL const bf16_t *p, int64_t k, TACC &a, TACC &b) {
  const uint32_t v = ld_aligned<NT>((GLOBAL const uint32_t *)(p + k));
  a = (TACC)__uint_as_float(v << 16);
  b = (TACC)__uint_as_float(v & 0xffff0000u);
}
template <bool NT, typename TACC>
__device__ __forceinline__ void ldval_pair(GLOBAL const _Float16 *p, int64_t k, TACC &a, TACC &b) {
  const v2f16 v = ld_aligned<NT>((GLOBAL const v2f16 *)(p + k));
  a = (TACC)(float)v.x;
  b = (TACC)(float)v.y;
}

// Sliced-diagonal rows, two per lane: a wave takes two slices at once (lanes
// 0-31 the first, 32-63 the second; in each die's range, pairs of slices
// from the bottom up, or the top down with REV), lane L rows 2 (L mod 32)
// and 2 (L mod 32) + 1 of its slice. Each row's products are added left to
// right from zero, as in the one-row walk, so both walks give the same bits.
// The kernel's functors work on row pairs:
//   pre2(r0, h0, h1) -> the pair's own operands (rows r0, r0 + 1; h0, h1:
//                       whether each row exists),
//   load2(j0)        -> what the operands at columns j0, j0 + 1 are made of
//                       (clamped loads, gather_pair),
//   comb2(loaded)    -> Pair<TACC>, those operands,
//   epi2(r0, h0, h1, sum0, sum1, pre_values),
// PRE_AT_DIAG: pre2 returns what load2(r0) would, on every row the epilogue
// keeps, so a leading entry at offset 0 (a diagonal) reuses it instead of
// loading the same operands again.
//   hook()           -> a workgroup step, called by every wave exactly once:
//                       after its first slice pair's loads are issued and
//                       before anything uses them (after the loop when the
//                       wave has no slice), so it may hold barriers and
//                       compute what comb2 needs; its result, the same in
//                       every thread, says whether the walk goes on.
// n >= 2.
template <typename TACC, bool NT, bool REV, bool PRE_AT_DIAG, typename TM, typename Pre2, typename Load2,
          typename Comb2, typename Epi2, typename Hook>
__device__ __forceinline__ bool sdia_rows2(const Mat<TM> &M, int l, int G, Pre2 pre2, Load2 load2, Comb2 comb2,
                                           Epi2 epi2, Hook hook) {
  constexpr int NW = kBlock / 64, U = 4;
  const int lane = threadIdx.x & 63, half = lane >> 5, lr = 2 * (lane & 31);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int W = G >> 3, x = l & 7, w = l >> 3;
  const int s0 = (int)((int64_t)x * M.nblk / 8), s1 = (int)((int64_t)(x + 1) * M.nblk / 8);
  const int npairs = (s1 - s0 + 1) / 2;
  // the first pair and its first chunk of entries are peeled so that what
  // hook needs is dead in the loops
  auto pair = [&](int p, auto first) -> bool {
    // slices ca (lanes 0-31) and cb = ca + 1 (lanes 32-63); at an odd end of
    // the range one of them lies outside it and its lanes idle on the other
    const int ca = REV ? s1 - 2 - 2 * p : s0 + 2 * p, cb = ca + 1;
    const bool va = ca >= s0, vb = cb < s1;
    // both slices' pointers and offsets are read whole-wave (scalar loads);
    // each half selects its own slice (cb <= s1 <= nblk, so blk[cb] exists)
    CONSTANT const int32_t *blk = ro(M.blk), *ci = ro(M.ci);
    const int ob = blk[cb], oa = va ? blk[ca] : ob, oe = vb ? blk[cb + 1] : ob;
    const int wa = ob - oa, wb = oe - ob;
    const bool useb = half ? vb : !va;
    const bool live = half ? vb : va;
    const int cs = useb ? cb : ca, o0 = useb ? ob : oa, wd = useb ? wb : wa;
    const int wmax = max(wa, wb);
    const int r0 = cs * kSliceRows + lr;
    const bool h0 = live && r0 < M.n, h1 = live && r0 + 1 < M.n;
    const auto pv = pre2(r0, h0, h1);
    GLOBAL const TM *vv = M.val + (int64_t)o0 * kSliceRows + lr;
    TACC sa = 0, sb = 0;
    auto chunk = [&](int e0, auto hk) -> bool {
      decltype(load2(0)) g[U];
      TACC va_[U], vb_[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // entries past this slice's width repeat its last (in bounds) and are not added
        const int e = max(min(e0 + u, wd - 1), 0);
        const int offa = wa > 0 ? ci[oa + max(min(e0 + u, wa - 1), 0)] : 0;
        const int offb = wb > 0 ? ci[ob + max(min(e0 + u, wb - 1), 0)] : 0;
        const int o = useb ? offb : offa;
        if constexpr (PRE_AT_DIAG) {
          if (e0 + u == 0 && o == 0)
            g[u] = pv;  // a leading diagonal: the pair's own operands, already loaded
          else
            g[u] = load2(r0 + o);
        } else {
          g[u] = load2(r0 + o);
        }
        ldval_pair<NT>(vv, (int64_t)e * kSliceRows, va_[u], vb_[u]);
      }
      if constexpr (decltype(hk)::value)
        if (!hook()) return false;
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (e0 + u < wd) {
          const Pair<TACC> o = comb2(g[u]);
          sa += va_[u] * o.x;
          sb += vb_[u] * o.y;
        }
      return true;
    };
    int e0 = 0;
    if constexpr (decltype(first)::value) {
      if (wmax > 0) {
        if (!chunk(0, std::true_type{})) return false;
        e0 = U;
      } else if (!hook()) {
        return false;
      }
    }
    for (; e0 < wmax; e0 += U) chunk(e0, std::false_type{});
    epi2(r0, h0, h1, sa, sb, pv);
    return true;
  };
  int p = w * NW + wv;
  if (p >= npairs) return hook();
  if (!pair(p, std::true_type{})) return false;
  for (p += W * NW; p < npairs; p += W * NW) pair(p, std::false_type{});
  return true;
}

// The two-row walk applies to a sliced-diagonal matrix of at least 2 rows
// placed with two rows per lane.
template <typename TM>
__device__ __forceinline__ bool rows2(const Mat<TM> &M) {
  return M.fmt == FMT_SDIA && M.n >= 2 && M.rpl == 2;
}

template <typename TACC, bool REV = false, bool PRE_AT_DIAG = false, typename TM, typename Pre2, typename Load2,
          typename Comb2, typename Epi2, typename Hook>
__device__ __forceinline__ bool for_rows2(const Mat<TM> &M, int l, int G, Pre2 pre2, Load2 load2, Comb2 comb2,
                                          Epi2 epi2, Hook hook) {
  if (M.temporal) return sdia_rows2<TACC, false, REV, PRE_AT_DIAG>(M, l, G, pre2, load2, comb2, epi2, hook);
  return sdia_rows2<TACC, true, REV, PRE_AT_DIAG>(M, l, G, pre2, load2, comb2, epi2, hook);
}

// Sliced 3x3-block rows: each wave takes whole slices of 21 block rows, one
// lane per row (lane 63 idle); the three lanes of a block row read the same
// block column. 8-byte values are stored column-major within the slice (lane
// 21 s + r for row s of block row r), so each column's values are one
// coalesced load; 4-byte values keep each row's three values contiguous
// (lane 3 r + s), one 12-byte load per lane. Each lane adds its row's three
// products block by block: the CSR order.
template <typename TM>
struct BsrLanes {
  static constexpr bool kColMajor = sizeof(TM) == 8;
  __device__ static int sub(int lane) { return kColMajor ? lane / kBSliceRows : lane % 3; }
  __device__ static int blockrow(int lane) { return kColMajor ? lane % kBSliceRows : lane / 3; }
  // offset of block k's column-j value for this lane, relative to the slice's first block
  __device__ static int64_t at(int lane, int k, int j) {
    return kColMajor ? ((int64_t)k * 3 + j) * (3 * kBSliceRows) + lane
                     : ((int64_t)k * kBSliceRows + lane / 3) * 9 + 3 * (lane % 3) + j;
  }
};

template <typename TACC, bool NT, typename TM, typename Pre, typename Gather, typename Epi>
__device__ __forceinline__ void bsr_rows(const Mat<TM> &M, int l, int G, Pre pre, Gather gather, Epi epi) {
  constexpr int NW = kBlock / 64;
  constexpr int SR = 3 * kBSliceRows;  // rows per slice
  using BL = BsrLanes<TM>;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int W = G >> 3, x = l & 7, w = l >> 3;
  const int s0 = (int)((int64_t)x * M.nblk / 8), s1 = (int)((int64_t)(x + 1) * M.nblk / 8);
  const int sub = BL::sub(lane), r = BL::blockrow(lane);
  for (int c = s0 + w * NW + wv; c < s1; c += W * NW) {
    const int o0 = ro(M.blk)[c], wd = ro(M.blk)[c + 1] - o0;
    const int row = (c * kBSliceRows + r) * 3 + sub;
    const bool has = lane < SR && row < M.n;
    if (!has) continue;
    const RowVals<TACC> pv = pre(row);
    GLOBAL const int32_t *bc = M.ci + (int64_t)o0 * kBSliceRows + r;
    GLOBAL const TM *bv = M.val + (int64_t)o0 * 9 * kBSliceRows;
    TACC sum = 0;
    int k = 0;
    for (; k + 2 <= wd; k += 2) {
      const int32_t c0 = 3 * ldstream<NT>(bc, (int64_t)k * kBSliceRows);
      const int32_t c1 = 3 * ldstream<NT>(bc, (int64_t)(k + 1) * kBSliceRows);
      TACC p[6];
#pragma unroll
      for (int j = 0; j < 3; ++j) p[j] = (TACC)ldval<NT>(bv, BL::at(lane, k, j)) * gather(c0 + j);
#pragma unroll
      for (int j = 0; j < 3; ++j) p[3 + j] = (TACC)ldval<NT>(bv, BL::at(lane, k + 1, j)) * gather(c1 + j);
#pragma unroll
      for (int u = 0; u < 6; ++u) sum += p[u];
    }
    if (k < wd) {
      const int32_t c0 = 3 * ldstream<NT>(bc, (int64_t)k * kBSliceRows);
#pragma unroll
      for (int j = 0; j < 3; ++j) sum += (TACC)ldval<NT>(bv, BL::at(lane, k, j)) * gather(c0 + j);
    }
    epi(row, sum, pv);
  }
}

// All rows of this workgroup (local index l of the system's G workgroups),
// in any layout, with the matrix's load policy.
// DIAG: pre(row).a is the gathered operand at column row (the sliced-diagonal
// walk then reuses it for a diagonal entry).
template <typename TACC, int UW, bool NT, bool REV, bool DIAG = false, typename TM, typename Pre, typename Gather,
          typename Epi>
__device__ __forceinline__ void for_rows_as(const Mat<TM> &M, int l, int G, TACC *lds, Pre pre, Gather gather,
                                            Epi epi) {
  if (M.fmt == FMT_SELL) {
    sell_rows<TACC, UW, NT, REV>(M, l, G, pre, gather, epi);
  } else if (M.fmt == FMT_SDIA) {
    sdia_rows<TACC, UW, NT, REV, DIAG>(M, l, G, pre, gather, epi);
  } else if (M.fmt == FMT_BSR3) {
    bsr_rows<TACC, NT>(M, l, G, pre, gather, epi);
  } else {
    const Sched sc = sched(M.nblk, l, G);
    for (int b = sc.first; b < sc.end; b += sc.stride) stream_block<TACC, NT>(M, b, lds, pre, gather, epi);
  }
}

template <typename TACC, int UW = 4, bool REV = false, bool DIAG = false, typename TM, typename Pre, typename Gather,
          typename Epi>
__device__ __forceinline__ void for_rows(const Mat<TM> &M, int l, int G, TACC *lds, Pre pre, Gather gather, Epi epi) {
  if (M.temporal)
    for_rows_as<TACC, UW, false, REV, DIAG>(M, l, G, lds, pre, gather, epi);
  else
    for_rows_as<TACC, UW, true, REV, DIAG>(M, l, G, lds, pre, gather, epi);
}

// for_rows with a workgroup step (hook, as in sdia_rows_h) before the first
// epilogue: over sliced diagonals after the first slice's products, in the
// other layouts before the walk. Returns hook's result.
template <typename TACC, int UW = 4, typename TM, typename Pre, typename Gather, typename Epi, typename Hook>
__device__ __forceinline__ bool for_rows_h(const Mat<TM> &M, int l, int G, TACC *lds, Pre pre, Gather gather,
                                           Epi epi, Hook hook) {
  if (M.fmt == FMT_SDIA) {
    if (M.temporal) return sdia_rows_h<TACC, UW, false, false>(M, l, G, pre, gather, epi, hook);
    return sdia_rows_h<TACC, UW, true, false>(M, l, G, pre, gather, epi, hook);
  }
  if (!hook()) return false;
  for_rows<TACC, UW>(M, l, G, lds, pre, gather, epi);
  return true;
}

// ---- inner products
//
// Every dot product and norm is its exact value rounded once to FP64, the
// value that does not depend on how the sum is split over lanes, waves and
// workgroups. Each lane accumulates its products as an unevaluated double-
// double hi + lo (the product's rounding error from an FMA, the additions'
// from TwoSum: Ogita, Rump and Oishi's Dot2); partial sums are combined as
// double-doubles in any order and rounded once at the end. The result is the
// correctly rounded inner product unless the exact value lies within about
// n u^2 sum|a_i b_i| of a rounding boundary (u = 2^-53), which for the sizes
// here is far below one chance in a billion per dot product.
struct Acc {
  double hi, lo;
};

// s + e = a + b exactly, s = fl(a + b) (Knuth's TwoSum; needs no ordering
// of |a|, |b|, and no contraction or reassociation, which the build forbids)
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// x += a b: the product's exact error from an FMA (FP64 operands); the
// product of two FP32 values is exact in FP64
__device__ __forceinline__ void acc_prod(Acc &x, double a, double b) {
  const double p = a * b;
  const double pe = __builtin_fma(a, b, -p);
  double s, e;
  two_sum(x.hi, p, s, e);
  x.hi = s;
  x.lo = x.lo + (e + pe);
}
__device__ __forceinline__ void acc_prod(Acc &x, float a, float b) {
  const double p = (double)a * (double)b;
  double s, e;
  two_sum(x.hi, p, s, e);
  x.hi = s;
  x.lo = x.lo + e;
}

// a + b, normalised (hi = fl(hi + lo))
__device__ __forceinline__ Acc acc_add(Acc a, Acc b) {
  double s, e;
  two_sum(a.hi, b.hi, s, e);
  const double t = (a.lo + b.lo) + e;
  Acc r;
  two_sum(s, t, r.hi, r.lo);
  return r;
}

// One DPP move of a double (two 32-bit moves); lanes of rows outside
// ROW_MASK receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROW_MASK, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ Acc acc_dpp(Acc a) {
  return Acc{dpp_f64<CTRL, ROW_MASK>(a.hi), dpp_f64<CTRL, ROW_MASK>(a.lo)};
}

// Wave total of a double-double by DPP row operations, with no LDS traffic.
// The two quad exchanges, the half-row mirror and the row mirror leave each
// 16-lane row's total in all of its lanes. Two row broadcasts then carry
// rows 0 to 2 into row 3, so lanes 48-63 hold the total.
__device__ __forceinline__ Acc wave_total(Acc v) {
  v = acc_add(v, acc_dpp<0xB1, 0xF>(v));   // quad_perm [1,0,3,2]
  v = acc_add(v, acc_dpp<0x4E, 0xF>(v));   // quad_perm [2,3,0,1]
  v = acc_add(v, acc_dpp<0x141, 0xF>(v));  // row_half_mirror
  v = acc_add(v, acc_dpp<0x140, 0xF>(v));  // row_mirror
  v = acc_add(v, acc_dpp<0x142, 0xA>(v));  // row_bcast:15 into rows 1 and 3
  v = acc_add(v, acc_dpp<0x143, 0xC>(v));  // row_bcast:31 into rows 2 and 3
  return v;
}

// Workgroup total of each value, in thread 0 (normalised); sh[0, NV NW).
template <int NV>
__device__ __forceinline__ void block_sum(Acc (&v)[NV], Acc *sh) {
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = wave_total(v[j]);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NW = kBlock / 64;
  if (lane == 63)
#pragma unroll
    for (int j = 0; j < NV; ++j) sh[j * NW + w] = v[j];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      Acc a = sh[j * NW];
      for (int q = 1; q < NW; ++q) a = acc_add(a, sh[j * NW + q]);
      v[j] = a;
    }
  __syncthreads();
}

// Write this workgroup's partial sums: value j's hi at p[2j G + L], its lo at
// p[(2j + 1) G + L] (kAccWords doubles per partial).
template <int NV>
__device__ __forceinline__ void put_partials(Acc (&v)[NV], GLOBAL double *p, int L, int G, Acc *sh) {
  block_sum<NV>(v, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      p[(int64_t)(2 * j) * G + L] = v[j].hi;
      p[(int64_t)(2 * j + 1) * G + L] = v[j].lo;
    }
}

// Total of the P partials of each value; every thread gets the totals,
// rounded once to FP64. load_partials adds this thread's share (no barrier,
// so a kernel can issue it before it reads its state); reduce_partials
// finishes the sums.
template <int NV>
__device__ __forceinline__ void load_partials(GLOBAL const double *__restrict__ p, int P, Acc (&acc)[NV]) {
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = Acc{0.0, 0.0};
#pragma unroll 4
  for (int k = threadIdx.x; k < P; k += kBlock)
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = acc_add(acc[j], Acc{p[(int64_t)(2 * j) * P + k], p[(int64_t)(2 * j + 1) * P + k]});
}

// A value every lane holds alike, as a wave-uniform (scalar) value.
__device__ __forceinline__ double uniform(double v) {
  const uint64_t b = __double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b), hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// The wave totals meet in LDS after one barrier, and every thread adds them
// in the same order. They sit in sh[2 NW, 2 NW + NV NW), apart from
// block_sum's slots, so that a block_sum later in the kernel cannot
// overwrite them while a slower wave still reads them; callers put a barrier
// between two calls.
template <int NV>
__device__ __forceinline__ void reduce_partials(Acc (&acc)[NV], double (&out)[NV], Acc *sh) {
  static_assert(NV <= 2, "reduction slots");
  constexpr int NW = kBlock / 64;
  Acc *shr = sh + 2 * NW;
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = wave_total(acc[j]);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 63)
#pragma unroll
    for (int j = 0; j < NV; ++j) shr[j * NW + w] = acc[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    Acc a = shr[j * NW];
    for (int q = 1; q < NW; ++q) a = acc_add(a, shr[j * NW + q]);
    out[j] = uniform(a.hi + a.lo);
  }
}

template <int NV>
__device__ __forceinline__ void sum_partials(GLOBAL const double *__restrict__ p, int P, double (&out)[NV],
                                             Acc *sh) {
  Acc acc[NV];
  load_partials<NV>(p, P, acc);
  reduce_partials<NV>(acc, out, sh);
}

// ------------------------------------------------------------------ kernels

// Rows [l n / G, (l+1) n / G) of a system: local workgroup l's share of
// elementwise work over G workgroups.
__device__ __forceinline__ void ew_rows(int n, int l, int G, int64_t &i0, int64_t &i1) {
  i0 = (int64_t)l * n / G;
  i1 = (int64_t)(l + 1) * n / G;
}

// UW: loads in flight per lane in the one-row sliced walks (rows longer
// than 4 entries), a tuning knob.
template <typename TV, typename TA, int UW>
__global__ __launch_bounds__(kBlock) PCG_OCCUPANCY void k_iter_A(const SysDev *__restrict__ dir, const int2 *__restrict__ map) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  __shared__ Acc sh[4 * (kBlock / 64)];
  const int2 m = map[blockIdx.x];
  const SysDev &D = dir[m.x];
  GLOBAL const State &S = gl(D.st)[0];
  if (S.done) return;
  const Mat<TA> A = mat<TA>(D.A);
  const int it = S.iter;
  GLOBAL TV *__restrict__ q = gl((TV *)D.q);
  GLOBAL const TV *__restrict__ dcur = gl((const TV *)((it & 1) ? D.d1 : D.d0));  // d_i
  Acc part[1] = {{0.0, 0.0}};
  // pre's d_i[row] is the operand of A's diagonal
  for_rows<TV, UW, false, true>(
      A, m.y, D.A.grid, lds, [&](int row) { return RowVals<TV>{dcur[row], (TV)0, (TV)0}; },
      [&](int j) -> TV { return dcur[j]; },
      [&](int row, TV sum, const RowVals<TV> &pv) {
        q[row] = sum;
        acc_prod(part[0], pv.a, sum);
      });
  put_partials<1>(part, gl(D.pg), part_slot(m.y, D.A.grid), D.A.grid, sh);
}

template <typename TV, typename TG>
__global__ __launch_bounds__(kBlock) PCG_GT_OCCUPANCY void k_iter_GT(const SysDev *__restrict__ dir, const int2 *__restrict__ map,
                                                    int mode) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  __shared__ Acc sh[4 * (kBlock / 64)];
  const int2 m = map[blockIdx.x];
  const SysDev &D = dir[m.x];
  GLOBAL State *st = gl(D.st);
  GLOBAL const State &S = st[0];
  Acc g[1];
  load_partials<1>(gl(D.pg), D.A.grid, g);  // in flight while the state is read
  if (S.done) {  // stopped earlier: st[1] mirrors st[0], so the G-kernel need not read st[0]
    if (m.y == 0 && threadIdx.x == 0) st_state(st + 1, ld_state(&S));
    return;
  }
  const int it = S.iter;
  if (mode == 3) mode = (S.rr_period > 0 && it > 0 && it % S.rr_period == 0) ? 1 : 0;
  const double delta = S.delta, alpha0 = S.alpha, gamma0 = S.gamma;
  const Mat<TG> GT = mat<TG>(D.GT);
  GLOBAL const TV *__restrict__ q = gl((const TV *)D.q);
  GLOBAL TV *__restrict__ t = gl((TV *)D.t);
  GLOBAL const TV *__restrict__ src = gl((const TV *)((((mode == 1) ? it + 1 : it) & 1) ? D.r1 : D.r0));
  GLOBAL TV *__restrict__ dst = gl((TV *)(((it + 1) & 1) ? D.r1 : D.r0));
  // alpha_i = delta_i / gamma_i (published in st[1] after the walk); false
  // on breakdown
  double alpha = alpha0, gamma = gamma0;
  bool brk = false;
  TV al = (TV)0;
  auto step = [&]() -> bool {
    if (mode != 2) {
      double gv[1];
      reduce_partials<1>(g, gv, sh);
      gamma = gv[0];
      brk = !(gamma > 0.0) || !isfinite(gamma);
      alpha = brk ? 0.0 : delta / gamma;  // on breakdown x already holds x_i
    }
    al = (mode == 0) ? (TV)alpha : (TV)0;
    return !brk;
  };
  auto publish = [&]() {
    if (m.y == 0 && threadIdx.x == 0) {
      State o = ld_state(&S);
      o.gamma = gamma;
      o.alpha = alpha;
      if (brk) {
        o.status = ST_BREAK_GAMMA;
        o.done = 1;
      }
      st_state(st + 1, o);
    }
  };
  Acc part[2] = {{0.0, 0.0}, {0.0, 0.0}};
  // each die walks its slices from the top down (measured slightly faster);
  // two rows per lane over sliced diagonals where the operand is the
  // difference of two gathered vectors (the other kernels, with one, are
  // faster one row per lane), with the first slice pair's loads in flight
  // while alpha is reduced
  if (mode == 0 && rows2(GT)) {
    const int32_t n = GT.n;
    struct PV {
      Pair<TV> s, q;
    };
    // pre2's pair equals gather_pair at offset 0 on every row that exists
    const bool go = for_rows2<TV, true, true>(
        GT, m.y, D.GT.grid,
        [&](int r0, bool h0, bool h1) -> PV {
          PV o{{(TV)0, (TV)0}, {(TV)0, (TV)0}};
          if (h1) {
            o.s = ld_pair(src, r0);
            o.q = ld_pair(q, r0);
          } else if (h0) {
            o.s.x = src[r0];
            o.q.x = q[r0];
          }
          return o;
        },
        [&](int32_t j0) -> PV { return PV{gather_pair(src, j0, n), gather_pair(q, j0, n)}; },
        [&](const PV &v) -> Pair<TV> { return Pair<TV>{v.s.x - al * v.q.x, v.s.y - al * v.q.y}; },
        [&](int r0, bool h0, bool h1, TV s0, TV s1, const PV &pv) {
          const TV ra = pv.s.x - al * pv.q.x, rb = pv.s.y - al * pv.q.y;
          if (h1) {
            st_pair(dst, r0, ra, rb);
            st_pair(t, r0, s0, s1);
            acc_prod(part[0], ra, ra);
            acc_prod(part[1], s0, s0);
            acc_prod(part[0], rb, rb);
            acc_prod(part[1], s1, s1);
          } else if (h0) {
            dst[r0] = ra;
            t[r0] = s0;
            acc_prod(part[0], ra, ra);
            acc_prod(part[1], s0, s0);
          }
        },
        step);
    publish();
    if (!go) return;
  } else if (!step()) {
    publish();
    return;
  } else if (mode == 0) {
    publish();
    for_rows<TV, 4, true>(
        GT, m.y, D.GT.grid, lds, [&](int row) { return RowVals<TV>{src[row], q[row], (TV)0}; },
        [&](int j) -> TV { return src[j] - al * q[j]; },
        [&](int row, TV sum, const RowVals<TV> &pv) {
          const TV rn = pv.a - al * pv.b;
          dst[row] = rn;
          t[row] = sum;
          acc_prod(part[0], rn, rn);
          acc_prod(part[1], sum, sum);
        });
  } else {
    publish();
    for_rows<TV, 4, true>(
        GT, m.y, D.GT.grid, lds, [&](int row) { return RowVals<TV>{src[row], (TV)0, (TV)0}; },
        [&](int j) -> TV { return src[j]; },
        [&](int row, TV sum, const RowVals<TV> &pv) {
          t[row] = sum;
          acc_prod(part[0], pv.a, pv.a);
          acc_prod(part[1], sum, sum);
        });
  }
  put_partials<2>(part, gl(D.prt), part_slot(m.y, D.GT.grid), D.GT.grid, sh);
}

template <typename TV, typename TG, bool HAS_EPS>
__global__ __launch_bounds__(kBlock) PCG_G_OCCUPANCY void k_iter_G(const SysDev *__restrict__ dir, const int2 *__restrict__ map,
                                                   int mode) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  __shared__ Acc sh[4 * (kBlock / 64)];
  const int2 m = map[blockIdx.x];
  const SysDev &D = dir[m.x];
  GLOBAL State *st = gl(D.st);
  // st[1] is the G^T-kernel's publication for this iteration; st[0] is written
  // below by workgroup 0 and must not be read by the others
  GLOBAL const State &S = st[1];
  Acc va[2];
  load_partials<2>(gl(D.prt), D.GT.grid, va);  // in flight while the state is read
  if (S.done) {  // stopped earlier, or the G^T-kernel flagged a breakdown
    if (m.y == 0 && threadIdx.x == 0) st_state(st, ld_state(&S));
    return;
  }
  const int it = S.iter;
  const double delta = S.delta, eps_d = S.eps, tol_nb = S.tol_nb;
  const int maxit = S.maxit;
  const int i1 = (mode == 2) ? it : it + 1;
  // x_{i+1} = x_i + alpha_i d_i (not at a start or restart, mode 2)
  const bool upd = mode != 2;
  const TV ap = (TV)S.alpha;
  GLOBAL TV *__restrict__ x = gl((TV *)D.x);
  GLOBAL const TV *__restrict__ dprev = gl((const TV *)((i1 & 1) ? D.d0 : D.d1));  // d_i
  // s = G t + eps r, and the next direction d_{i+1} = s + beta d_i (at a
  // start or restart beta = 0, d = s)
  const Mat<TG> G = mat<TG>(D.G);
  GLOBAL const TV *__restrict__ t = gl((const TV *)D.t);
  GLOBAL const TV *__restrict__ rc = gl((const TV *)((i1 & 1) ? D.r1 : D.r0));
  GLOBAL TV *__restrict__ dnext = gl((TV *)((i1 & 1) ? D.d1 : D.d0));
  const TV eps = (TV)eps_d;
  // delta_{i+1}, beta_i and the stopping tests, published in st[0]; false
  // once the solve stops (then only x is updated)
  TV beta = (TV)0;
  double rr = 0.0, tt = 0.0, dn = 0.0;
  int status = ST_RUNNING;
  auto step = [&]() -> bool {
    double v[2];
    reduce_partials<2>(va, v, sh);
    rr = v[0];
    tt = v[1];
    dn = tt + eps_d * rr;
    if (mode != 2 && (!(dn >= 0.0) || !isfinite(dn)))
      status = ST_BREAK_DELTA;
    else if (sqrt(rr) <= tol_nb)
      status = ST_CONV_REC;
    else if (i1 >= maxit)
      status = ST_MAXIT;
    beta = (TV)((mode == 2) ? 0.0 : dn / delta);
    return status == ST_RUNNING;
  };
  // the first slice's products are formed while the partials are reduced;
  // two rows per lane over sliced diagonals (as in the G^T-kernel: one
  // access of twice the width for each operand, value and result), one
  // otherwise and at a start or restart
  bool go;
  if (upd && rows2(G)) {
    const int32_t n = G.n;
    struct PV {
      Pair<TV> r, d, x;
    };
    go = for_rows2<TV, false, false>(
        G, m.y, D.G.grid,
        [&](int r0, bool h0, bool h1) -> PV {
          PV o{{(TV)0, (TV)0}, {(TV)0, (TV)0}, {(TV)0, (TV)0}};
          if (h1) {
            if (HAS_EPS) o.r = ld_pair(rc, r0);
            o.d = ld_pair(dprev, r0);
            o.x = ld_pair(x, r0);
          } else if (h0) {
            if (HAS_EPS) o.r.x = rc[r0];
            o.d.x = dprev[r0];
            o.x.x = x[r0];
          }
          return o;
        },
        [&](int32_t j0) -> Pair<TV> { return gather_pair(t, j0, n); },
        [&](const Pair<TV> &v) -> Pair<TV> { return v; },
        [&](int r0, bool h0, bool h1, TV s0, TV s1, const PV &pv) {
          const TV sv0 = HAS_EPS ? s0 + eps * pv.r.x : s0, sv1 = HAS_EPS ? s1 + eps * pv.r.y : s1;
          const TV dn0 = sv0 + beta * pv.d.x, dn1 = sv1 + beta * pv.d.y;
          const TV x0 = pv.x.x + ap * pv.d.x, x1 = pv.x.y + ap * pv.d.y;
          if (h1) {
            st_pair(dnext, r0, dn0, dn1);
            st_pair(x, r0, x0, x1);
          } else if (h0) {
            dnext[r0] = dn0;
            x[r0] = x0;
          }
        },
        step);
  } else if (upd)
    go = for_rows_h<TV>(
        G, m.y, D.G.grid, lds,
        [&](int row) { return RowVals<TV>{HAS_EPS ? rc[row] : (TV)0, dprev[row], x[row]}; },
        [&](int j) -> TV { return t[j]; },
        [&](int row, TV sum, const RowVals<TV> &pv) {
          const TV sv = HAS_EPS ? sum + eps * pv.a : sum;
          dnext[row] = sv + beta * pv.b;
          x[row] = pv.c + ap * pv.b;
        },
        step);
  else
    go = for_rows_h<TV>(
        G, m.y, D.G.grid, lds, [&](int row) { return RowVals<TV>{HAS_EPS ? rc[row] : (TV)0, dprev[row], (TV)0}; },
        [&](int j) -> TV { return t[j]; },
        [&](int row, TV sum, const RowVals<TV> &pv) {
          const TV sv = HAS_EPS ? sum + eps * pv.a : sum;
          dnext[row] = sv + beta * pv.b;
        },
        step);
  if (m.y == 0 && threadIdx.x == 0) {
    State o = ld_state(&S);
    o.rr = rr;
    o.tt = tt;
    o.iter = i1;
    o.alpha = 0.0;  // x += alpha_i d_i is applied in this kernel, whatever the status
    if (status != ST_BREAK_DELTA) {
      o.beta = (mode == 2) ? 0.0 : dn / delta;
      o.delta = dn;
    }
    if (status != ST_RUNNING) {
      o.status = status;
      o.done = 1;
    }
    st_state(st, o);
  }
  if (!go && upd) {  // stopped: x_{i+1} only
    int64_t i0, i1r;
    ew_rows(D.n, m.y, D.G.grid, i0, i1r);
    for (int64_t i = i0 + threadIdx.x; i < i1r; i += kBlock) x[i] = x[i] + ap * dprev[i];
  }
}

template <typename TV, typename TA>
__global__ __launch_bounds__(kBlock) PCG_OCCUPANCY void k_resid(const SysDev *__restrict__ dir, const int2 *__restrict__ map,
                                                  int slot_sel, int with_d, int reduce, int respect_done) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  __shared__ Acc sh[4 * (kBlock / 64)];
  const int2 m = map[blockIdx.x];
  const SysDev &D = dir[m.x];
  GLOBAL const State &S = gl(D.st)[0];
  if (respect_done && S.done) return;
  const int it = S.iter;
  if (slot_sel == 2) {  // replacement decided per system
    if (!(S.rr_period > 0 && it > 0 && it % S.rr_period == 0)) return;
    slot_sel = 1;
  }
  const Mat<TA> A = mat<TA>(D.A);
  GLOBAL const TV *__restrict__ b = gl((const TV *)D.b);
  GLOBAL const TV *__restrict__ x = gl((const TV *)D.x);
  GLOBAL TV *__restrict__ rout = gl((TV *)(((it + slot_sel) & 1) ? D.r1 : D.r0));
  GLOBAL const TV *__restrict__ dc = gl((const TV *)((it & 1) ? D.d1 : D.d0));  // d_i
  TV al = (TV)0;
  if (with_d) {
    double g[1];
    sum_partials<1>(gl(D.pg), D.A.grid, g, sh);
    if (!(g[0] > 0.0) || !isfinite(g[0])) return;  // the G^T-kernel reports the breakdown
    al = (TV)(S.delta / g[0]);
  }
  Acc part[1] = {{0.0, 0.0}};
  auto pre = [&](int row) { return RowVals<TV>{b[row], (TV)0, (TV)0}; };
  auto epi = [&](int row, TV sum, const RowVals<TV> &pv) {
    const TV rv = pv.a - sum;
    rout[row] = rv;
    acc_prod(part[0], rv, rv);
  };
  if (with_d)
    for_rows<TV>(A, m.y, D.A.grid, lds, pre, [&](int j) -> TV { return x[j] + al * dc[j]; }, epi);
  else
    for_rows<TV>(A, m.y, D.A.grid, lds, pre, [&](int j) -> TV { return x[j]; }, epi);
  if (reduce) put_partials<1>(part, gl(D.ptr), part_slot(m.y, D.A.grid), D.A.grid, sh);
}


// ------------------------------------------------ one-workgroup solver

// Totals of a workgroup's double-double sums, rounded once, in every thread.
template <int NV>
__device__ __forceinline__ void wg_totals(Acc (&v)[NV], double (&out)[NV], Acc *sh) {
  reduce_partials<NV>(v, out, sh);
}

// Every row of M by this one workgroup: the eight die-slabs of the
// iteration kernels' partition, one after the other, then a barrier (the
// vector written is read by the next phase). Ordinary loads: a small
// system's matrices stay in L2 from one iteration to the next.
template <typename TACC, int UW, bool REV, typename TM, typename Pre, typename Gather, typename Epi>
__device__ __forceinline__ void wg_rows(const Mat<TM> &M, TACC *lds, Pre pre, Gather gather, Epi epi) {
  for (int l = 0; l < 8; ++l) for_rows_as<TACC, UW, false, REV>(M, l, 8, lds, pre, gather, epi);
  __syncthreads();
}

// Elementwise over all rows by this workgroup, then a barrier.
template <typename F>
__device__ __forceinline__ void wg_elementwise(int n, F f) {
  for (int64_t i = threadIdx.x; i < n; i += kBlock) f(i);
  __syncthreads();
}

// The solve of one system by this workgroup. The iteration vectors x, q, t,
// r (two slots) and d (two slots) are reached through VP: global memory, or
// the workgroup's LDS for a system small enough (then x is copied in and out
// by the kernel). b, the matrices and the state stay in global memory. Both
// placements run the same operations in the same order.
template <typename TV, typename TA, typename TG, bool HAS_EPS, typename VP>
__device__ __forceinline__ void solve_wg(const SysDev &D, GLOBAL State *st, const State &S0, TV *lds, Acc *sh, VP __restrict__ x,
                                         VP __restrict__ q, VP __restrict__ t, VP r0, VP r1, VP d0, VP d1) {
  const int n = D.n;
  const Mat<TA> A = mat<TA>(D.A);
  const Mat<TG> GT = mat<TG>(D.GT), G = mat<TG>(D.G);
  GLOBAL const TV *__restrict__ b = gl((const TV *)D.b);
  VP rv[2] = {r0, r1};
  VP dv[2] = {d0, d1};
  const double eps = S0.eps;
  const TV epsv = (TV)eps;
  // ||b||^2, tol ||b||
  double bb;
  {
    Acc a[1] = {{0.0, 0.0}};
    for (int64_t i = threadIdx.x; i < n; i += kBlock) acc_prod(a[0], b[i], b[i]);
    double v[1];
    wg_totals<1>(a, v, sh);
    bb = v[0];
  }
  const double tol_nb = S0.tol * sqrt(bb);
  State o = S0;
  o.bb = bb;
  o.tol_nb = tol_nb;
  o.alpha = o.beta = 0.0;
  o.restarts = 0;
  if (bb == 0.0) {
    wg_elementwise(n, [&](int64_t i) { x[i] = (TV)0; });
    o.status = ST_ZERO_B;
    o.done = 1;
    o.iter = 0;
    o.rr = o.tt = o.true_rr = 0.0;
    if (threadIdx.x == 0) st_state(st, o);
    return;
  }
  wg_elementwise(n, [&](int64_t i) { dv[0][i] = (TV)0; dv[1][i] = (TV)0; });
  int it = 0;
  int status = ST_RUNNING;
  double delta = 0.0, rr = 0.0, tt = 0.0, true_rr = 0.0;
  // r_it = b - A x (true residual), its norm when `reduce`
  auto residual = [&](VP rout, bool reduce) {
    Acc a[1] = {{0.0, 0.0}};
    wg_rows<TV, 4, false>(
        A, lds, [&](int row) { return RowVals<TV>{b[row], (TV)0, (TV)0}; }, [&](int j) -> TV { return x[j]; },
        [&](int row, TV sum, const RowVals<TV> &pv) {
          const TV r = pv.a - sum;
          rout[row] = r;
          acc_prod(a[0], r, r);
        });
    double v[1];
    wg_totals<1>(a, v, sh);
    if (reduce) true_rr = v[0];
  };
  // start or restart from r_it: t = G^T r, rr, tt, delta, d_it = G t + eps r
  // (beta = 0 against the zeroed or previous direction buffer), stop tests
  auto restart = [&]() {
    const VP src = rv[it & 1];
    Acc a[2] = {{0.0, 0.0}, {0.0, 0.0}};
    wg_rows<TV, 4, true>(
        GT, lds, [&](int row) { return RowVals<TV>{src[row], (TV)0, (TV)0}; }, [&](int j) -> TV { return src[j]; },
        [&](int row, TV sum, const RowVals<TV> &pv) {
          t[row] = sum;
          acc_prod(a[0], pv.a, pv.a);
          acc_prod(a[1], sum, sum);
        });
    double v[2];
    wg_totals<2>(a, v, sh);
    rr = v[0];
    tt = v[1];
    const double dn = tt + eps * rr;
    if (sqrt(rr) <= tol_nb)
      status = ST_CONV_REC;
    else if (it >= S0.maxit)
      status = ST_MAXIT;
    delta = dn;
    if (status != ST_RUNNING) return;
    const VP dnext = dv[it & 1];
    const VP dprev = dv[(it + 1) & 1];
    const TV beta = (TV)0.0;
    wg_rows<TV, 4, false>(
        G, lds, [&](int row) { return RowVals<TV>{HAS_EPS ? src[row] : (TV)0, dprev[row], (TV)0}; },
        [&](int j) -> TV { return t[j]; },
        [&](int row, TV sum, const RowVals<TV> &pv) {
          const TV sv = HAS_EPS ? sum + epsv * pv.a : sum;
          dnext[row] = sv + beta * pv.b;
        });
  };
  residual(rv[0], false);
  restart();
  for (;;) {
    while (status == ST_RUNNING) {
      const VP dcur = dv[it & 1];
      // q = A d_i, gamma = d_i^T q
      double gamma;
      {
        Acc a[1] = {{0.0, 0.0}};
        wg_rows<TV, 8, false>(
            A, lds, [&](int row) { return RowVals<TV>{dcur[row], (TV)0, (TV)0}; },
            [&](int j) -> TV { return dcur[j]; },
            [&](int row, TV sum, const RowVals<TV> &pv) {
              q[row] = sum;
              acc_prod(a[0], pv.a, sum);
            });
        double v[1];
        wg_totals<1>(a, v, sh);
        gamma = v[0];
      }
      if (!(gamma > 0.0) || !isfinite(gamma)) {  // x stays x_i
        status = ST_BREAK_GAMMA;
        break;
      }
      const double alpha = delta / gamma;
      const TV al = (TV)alpha;
      const VP rnext = rv[(it + 1) & 1];
      const bool replace = S0.rr_period > 0 && it > 0 && it % S0.rr_period == 0;
      Acc a[2] = {{0.0, 0.0}, {0.0, 0.0}};
      if (replace) {  // r_{i+1} = b - A (x_i + alpha_i d_i), then t = G^T r_{i+1}
        wg_rows<TV, 4, false>(
            A, lds, [&](int row) { return RowVals<TV>{b[row], (TV)0, (TV)0}; },
            [&](int j) -> TV { return x[j] + al * dcur[j]; },
            [&](int row, TV sum, const RowVals<TV> &pv) { rnext[row] = pv.a - sum; });
        wg_rows<TV, 4, true>(
            GT, lds, [&](int row) { return RowVals<TV>{rnext[row], (TV)0, (TV)0}; },
            [&](int j) -> TV { return rnext[j]; },
            [&](int row, TV sum, const RowVals<TV> &pv) {
              t[row] = sum;
              acc_prod(a[0], pv.a, pv.a);
              acc_prod(a[1], sum, sum);
            });
      } else {  // r_{i+1} = r_i - alpha_i q, formed where it is gathered
        const VP src = rv[it & 1];
        wg_rows<TV, 4, true>(
            GT, lds, [&](int row) { return RowVals<TV>{src[row], q[row], (TV)0}; },
            [&](int j) -> TV { return src[j] - al * q[j]; },
            [&](int row, TV sum, const RowVals<TV> &pv) {
              const TV rn = pv.a - al * pv.b;
              rnext[row] = rn;
              t[row] = sum;
              acc_prod(a[0], rn, rn);
              acc_prod(a[1], sum, sum);
            });
      }
      double v[2];
      wg_totals<2>(a, v, sh);
      rr = v[0];
      tt = v[1];
      const double dn = tt + eps * rr;
      const int i1 = it + 1;
      if (!(dn >= 0.0) || !isfinite(dn))
        status = ST_BREAK_DELTA;
      else if (sqrt(rr) <= tol_nb)
        status = ST_CONV_REC;
      else if (i1 >= S0.maxit)
        status = ST_MAXIT;
      const TV ap = (TV)alpha;
      if (status != ST_RUNNING) {  // x_{i+1} = x_i + alpha_i d_i
        wg_elementwise(n, [&](int64_t i) { x[i] = x[i] + ap * dcur[i]; });
        if (status != ST_BREAK_DELTA) delta = dn;
        it = i1;
        break;
      }
      const TV beta = (TV)(dn / delta);
      delta = dn;
      const VP dnext = dv[i1 & 1];
      wg_rows<TV, 4, false>(
          G, lds, [&](int row) { return RowVals<TV>{HAS_EPS ? rnext[row] : (TV)0, dcur[row], x[row]}; },
          [&](int j) -> TV { return t[j]; },
          [&](int row, TV sum, const RowVals<TV> &pv) {
            const TV sv = HAS_EPS ? sum + epsv * pv.a : sum;
            dnext[row] = sv + beta * pv.b;
            x[row] = pv.c + ap * pv.b;
          });
      it = i1;
    }
    if (status == ST_BREAK_GAMMA || status == ST_BREAK_DELTA) break;
    // the true residual b - A x into the current r slot
    residual(rv[it & 1], true);
    if (status == ST_CONV_REC && S0.confirm && !(sqrt(true_rr) <= tol_nb)) {
      ++o.restarts;  // the recurrence drifted: restart from the true residual
      status = ST_RUNNING;
      restart();
      continue;
    }
    break;
  }
  o.iter = it;
  o.status = status;
  o.done = 1;
  o.rr = rr;
  o.tt = tt;
  o.delta = delta;
  o.true_rr = true_rr;
  if (threadIdx.x == 0) st_state(st, o);
}

// Iteration vectors in LDS: 7 n values (x, q, t, r0, r1, d0, d1).
#define LDSP __attribute__((address_space(3)))
constexpr int kWgVectors = 7;
// the host sizes the dynamic LDS assuming at most this much static LDS
static_assert(kLdsBytes + 4 * (kBlock / 64) * sizeof(Acc) + 2 * 8 * sizeof(double) <= kWgStaticLdsBytes,
              "static LDS of the one-workgroup solver");

// One workgroup per system of the set solves it whole. lds_vec_bytes: the
// dynamic LDS of the launch; a system whose seven iteration vectors fit in it
// keeps them there (a phase's gathers and stores then stay on the CU instead
// of going through L2), any other keeps them in global memory.
template <typename TV, typename TA, typename TG, bool HAS_EPS>
__global__ __launch_bounds__(kBlock) void k_solve_wg(const SysDev *__restrict__ dir, const int32_t *__restrict__ set,
                                                     int lds_vec_bytes) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  __shared__ Acc sh[4 * (kBlock / 64)];
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  const SysDev &D = dir[set[blockIdx.x]];
  GLOBAL State *st = gl(D.st);
  const State S0 = ld_state(st);
  const int n = D.n;
  GLOBAL TV *__restrict__ xg = gl((TV *)D.x);
  if ((int64_t)kWgVectors * n * (int64_t)sizeof(TV) <= lds_vec_bytes) {
    LDSP TV *v = (LDSP TV *)dyn_lds;
    wg_elementwise(n, [&](int64_t i) { v[i] = xg[i]; });
    solve_wg<TV, TA, TG, HAS_EPS>(D, st, S0, lds, sh, v, v + n, v + 2 * n, v + 3 * n, v + 4 * n, v + 5 * n,
                                  v + 6 * n);
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += kBlock) xg[i] = v[i];
  } else {
    solve_wg<TV, TA, TG, HAS_EPS>(D, st, S0, lds, sh, xg, gl((TV *)D.q), gl((TV *)D.t), gl((TV *)D.r0),
                                  gl((TV *)D.r1), gl((TV *)D.d0), gl((TV *)D.d1));
  }
}

template <typename TV>
__global__ __launch_bounds__(kBlock) void k_finalize(const SysDev *__restrict__ dir, const int2 *__restrict__ map) {
  const int2 m = map[blockIdx.x];
  const SysDev &D = dir[m.x];
  GLOBAL const State &S = gl(D.st)[0];
  const TV al = (TV)S.alpha;
  if (al == (TV)0) return;
  GLOBAL TV *__restrict__ x = gl((TV *)D.x);
  GLOBAL const TV *__restrict__ dc = gl((const TV *)(((S.iter - 1) & 1) ? D.d1 : D.d0));
  int64_t i0, i1;
  ew_rows(D.n, m.y, D.A.grid, i0, i1);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) x[i] = x[i] + al * dc[i];
}

template <typename TV>
__global__ __launch_bounds__(kBlock) void k_zero_dirs(const SysDev *__restrict__ dir, const int2 *__restrict__ map,
                                                      int zero_x) {
  const int2 m = map[blockIdx.x];
  const SysDev &D = dir[m.x];
  GLOBAL TV *__restrict__ d0 = gl((TV *)D.d0);
  GLOBAL TV *__restrict__ d1 = gl((TV *)D.d1);
  GLOBAL TV *__restrict__ x = gl((TV *)D.x);
  int64_t i0, i1;
  ew_rows(D.n, m.y, D.A.grid, i0, i1);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
    d0[i] = (TV)0;
    d1[i] = (TV)0;
    if (zero_x) x[i] = (TV)0;
  }
}

// Refinement steps over FP64 system views (A = FP64 copy, x = x64, b = b64,
// r0 = r64; s points at the inner solve's x and t at its right-hand side, both
// in the vector type), with rn = sqrt(st[0].true_rr) of each view:
//   update: x64 += rn * x_inner;   rhs: b_inner = (1 / rn) * r64.
template <typename TV>
__global__ __launch_bounds__(kBlock) void k_outer(const SysDev *__restrict__ dir, const int2 *__restrict__ map,
                                                  int what) {
  const int2 m = map[blockIdx.x];
  const SysDev &D = dir[m.x];
  const double rn = sqrt(gl(D.st)[0].true_rr);
  int64_t i0, i1;
  ew_rows(D.n, m.y, D.A.grid, i0, i1);
  if (what == 0) {
    GLOBAL double *__restrict__ x64 = gl((double *)D.x);
    GLOBAL const TV *__restrict__ c = gl((const TV *)D.s);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) x64[i] = x64[i] + rn * (double)c[i];
  } else {
    const double sc = 1.0 / rn;
    GLOBAL const double *__restrict__ r64 = gl((const double *)D.r0);
    GLOBAL TV *__restrict__ bi = gl((TV *)D.t);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) bi[i] = (TV)(sc * r64[i]);
  }
}

// One thread per system of the set.
__global__ void k_state_clear_alpha(const SysDev *__restrict__ dir, const int32_t *__restrict__ set, int nset) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nset) gl(dir[set[k]].st)[0].alpha = 0.0;
}

__global__ void k_state_restart(const SysDev *__restrict__ dir, const int32_t *__restrict__ set, int nset) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nset) return;
  GLOBAL State &S = gl(dir[set[k]].st)[0];
  S.done = 0;
  S.status = ST_RUNNING;
  S.alpha = 0.0;
  S.beta = 0.0;
}

template <typename TV>
__global__ __launch_bounds__(kBlock) void k_norm_b(const SysDev *__restrict__ dir, const int2 *__restrict__ map) {
  __shared__ Acc sh[4 * (kBlock / 64)];
  const int2 m = map[blockIdx.x];
  const SysDev &D = dir[m.x];
  GLOBAL const TV *__restrict__ b = gl((const TV *)D.b);
  Acc part[1] = {{0.0, 0.0}};
  // local workgroup l adds the contiguous slice l of b
  const int G = D.gB, l = m.y;
  const int64_t i0 = (int64_t)l * D.n / G, i1 = (int64_t)(l + 1) * D.n / G;
#pragma unroll 4
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) acc_prod(part[0], b[i], b[i]);
  put_partials<1>(part, gl(D.pb), l, G, sh);
}

// One workgroup per system of the set: ||b||^2 (what = 0, also tol * ||b||
// and the b = 0 test) or ||b - A x||^2 (what = 1) from its partials into st[0].
__global__ __launch_bounds__(kBlock) void k_reduce_state(const SysDev *__restrict__ dir,
                                                         const int32_t *__restrict__ set, int what) {
  __shared__ Acc sh[4 * (kBlock / 64)];
  const SysDev &D = dir[set[blockIdx.x]];
  double v[1];
  if (what == 0)
    sum_partials<1>(gl(D.pb), D.gB, v, sh);
  else
    sum_partials<1>(gl(D.ptr), D.A.grid, v, sh);
  if (threadIdx.x != 0) return;
  GLOBAL State &S = gl(D.st)[0];
  if (what == 0) {
    S.bb = v[0];
    S.tol_nb = S.tol * sqrt(v[0]);
    if (v[0] == 0.0) {
      S.status = ST_ZERO_B;
      S.done = 1;
    }
  } else {
    S.true_rr = v[0];
  }
}

template <typename TV, typename TM>
__global__ __launch_bounds__(kBlock) PCG_OCCUPANCY void k_spmv(DevCSR Md, const TV *__restrict__ x, TV *__restrict__ y) {
  __shared__ TV lds[kLdsBytes / sizeof(TV)];
  const Mat<TM> M = mat<TM>(Md);
  for_rows<TV, 8>(
      M, blockIdx.x, gridDim.x, lds, [&](int) { return RowVals<TV>{}; }, [&](int j) -> TV { return x[j]; },
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

// Streaming probes of the HBM ceiling (and the reference for calibrating the
// memory-traffic counters): 16-byte nontemporal accesses, four per lane in
// flight (all loads of a round issued before its stores), grid-stride rounds.
constexpr int kStreamUnroll = 4;

__global__ __launch_bounds__(kBlock) void k_copy(const u32x4 *__restrict__ src_, u32x4 *__restrict__ dst_, int64_t n16) {
  GLOBAL const u32x4 *src = gl(src_);
  GLOBAL u32x4 *dst = gl(dst_);
  constexpr int U = kStreamUnroll;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  for (; i + (U - 1) * stride < n16; i += U * stride) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
  for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Read-only stream: the words are folded with xor, and a workgroup writes its
// fold only if it equals a value no test data produces (so the loads stay).
__global__ __launch_bounds__(kBlock) void k_read(const u32x4 *__restrict__ src_, int64_t n16,
                                                 uint32_t *__restrict__ sink_) {
  GLOBAL const u32x4 *src = gl(src_);
  constexpr int U = kStreamUnroll;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  u32x4 acc = {0u, 0u, 0u, 0u};
  for (; i + (U - 1) * stride < n16; i += U * stride) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u];
  }
  for (; i < n16; i += stride) acc ^= __builtin_nontemporal_load(src + i);
  if (acc.x == 0x9e3779b9u && acc.y == 0x7f4a7c15u && acc.z == 0x85ebca6bu && acc.w == 0xc2b2ae35u)
    gl(sink_)[blockIdx.x] = acc.x;
}

// ------------------------------------------------ FSAI construction on the device

// One wave (the whole workgroup) per row; LDS holds S = A[J,J] (m x m,
// row-major), g (m) and J (m).
__global__ __launch_bounds__(64) void k_fsai_rows(const int32_t *__restrict__ rp_, const int32_t *__restrict__ ci_,
                                                  const double *__restrict__ v_, const int32_t *__restrict__ dpos_,
                                                  const int32_t *__restrict__ lrp_, int32_t n, int32_t mmax,
                                                  double *__restrict__ lv_, int32_t *__restrict__ err_) {
  extern __shared__ double smem[];
  GLOBAL const int32_t *rp = gl(rp_), *ci = gl(ci_), *dpos = gl(dpos_), *lrp = gl(lrp_);
  GLOBAL const double *v = gl(v_);
  GLOBAL double *lv = gl(lv_);
  GLOBAL int32_t *err = gl(err_);
  double *S = smem;
  double *g = smem + (size_t)mmax * mmax;
  int32_t *J = (int32_t *)(g + mmax);
  const int lane = threadIdx.x;
  for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int32_t r0 = rp[i];
    const int m = dpos[i] - r0 + 1;
    for (int a = lane; a < m; a += 64) J[a] = ci[r0 + a];
    __syncthreads();
    // lower part of S: S[a][b] = A[J[a], J[b]] (b <= a), merging row J[a]'s
    // columns up to its diagonal with J
    for (int a = lane; a < m; a += 64) {
      const int32_t row = J[a];
      int32_t k = rp[row];
      const int32_t kend = dpos[row];
      double *Sa = S + (size_t)a * m;
      int b = 0;
      while (b <= a) {
        if (k > kend) {
          Sa[b++] = 0.0;
          continue;
        }
        const int32_t c = ci[k], jb = J[b];
        if (c == jb) {
          Sa[b++] = v[k++];
        } else if (c < jb) {
          ++k;
        } else {
          Sa[b++] = 0.0;
        }
      }
    }
    __syncthreads();
    // Cholesky, column by column: the pivot by lane 0, the column below it by
    // one lane per entry, each sum left to right
    for (int c = 0; c < m; ++c) {
      if (lane == 0) {
        double dsum = S[(size_t)c * m + c];
        for (int k = 0; k < c; ++k) dsum -= S[(size_t)c * m + k] * S[(size_t)c * m + k];
        if (!(dsum > 0.0)) {
          err[0] = 1;
          dsum = 1.0;
        }
        S[(size_t)c * m + c] = sqrt(dsum);
      }
      __syncthreads();
      const double l = S[(size_t)c * m + c];
      for (int a = c + 1 + lane; a < m; a += 64) {
        double e = S[(size_t)a * m + c];
        for (int k = 0; k < c; ++k) e -= S[(size_t)a * m + k] * S[(size_t)c * m + k];
        S[(size_t)a * m + c] = e / l;
      }
      __syncthreads();
    }
    // back substitution L^T g = e_last
    if (lane == 0) {
      const int32_t base = lrp[i];
      for (int a = m - 1; a >= 0; --a) {
        double e = (a == m - 1) ? 1.0 : 0.0;
        for (int k = a + 1; k < m; ++k) e -= S[(size_t)k * m + a] * g[k];
        g[a] = e / S[(size_t)a * m + a];
        lv[base + a] = g[a];
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_absmax(const double *__restrict__ x, int64_t m, double *__restrict__ part) {
  __shared__ double sh[kBlock / 64];
  double a = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < m; k += (int64_t)gridDim.x * kBlock)
    a = fmax(a, fabs(x[k]));
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) a = fmax(a, __shfl_xor(a, off));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) a = fmax(a, sh[w]);
    part[blockIdx.x] = a;
  }
}

// Rounding to nearest even onto a format with `sig` significant bits, least
// normal exponent emin and largest finite value vmax (subnormals included,
// beyond vmax: infinity); every step is exact.
__device__ double round_sig(double v, int sig, int emin, double vmax) {
  if (v == 0.0 || !isfinite(v)) return v;
  int e;
  frexp(fabs(v), &e);
  int q = e - sig;
  if (e - 1 < emin) q = emin - (sig - 1);
  double r = ldexp(rint(ldexp(fabs(v), -q)), q);
  if (r > vmax) r = INFINITY;
  return copysign(r, v);
}

__device__ uint16_t bf16_bits(double v) {
  return (uint16_t)(__float_as_uint((float)round_sig(v, 8, -126, 3.3895313892515355e38)) >> 16);
}

__device__ uint16_t f16_bits(double v) {
  const double r = round_sig(v, 11, -14, 65504.0);
  if (isinf(r)) return r > 0 ? 0x7C00 : 0xFC00;
  if (isnan(r)) return 0x7E00;
  const uint16_t sign = signbit(r) ? 0x8000 : 0;
  const double a = fabs(r);
  if (a == 0.0) return sign;
  int e;
  const double mnt = frexp(a, &e);  // a = mnt 2^e, mnt in [0.5, 1)
  if (e - 1 >= -14) return sign | (uint16_t)((e - 1 + 15) << 10) | (uint16_t)rint((mnt * 2.0 - 1.0) * 1024.0);
  return sign | (uint16_t)rint(a * 16777216.0);  // subnormal: multiples of 2^-24
}

// Store entry idx of `row` (column col) in M's layout: CSR, sliced ELL, or
// sliced diagonals (the slot of offset col - row among the slice's offsets).
__device__ __forceinline__ void store_val(const DevCSR &M, int32_t row, int32_t idx, int32_t col, double x) {
  int64_t p;
  if (M.fmt == FMT_SELL) {
    p = ((int64_t)gl(M.blk)[row / kSliceRows] + idx) * kSliceRows + row % kSliceRows;
  } else if (M.fmt == FMT_SDIA) {
    GLOBAL const int32_t *off = gl(M.ci);
    int32_t lo = gl(M.blk)[row / kSliceRows], hi = gl(M.blk)[row / kSliceRows + 1] - 1;
    const int32_t d = col - row;
    while (lo < hi) {  // the slice lists every offset of its rows, so d is found
      const int32_t mid = lo + (hi - lo) / 2;
      if (off[mid] < d)
        lo = mid + 1;
      else
        hi = mid;
    }
    p = (int64_t)lo * kSliceRows + row % kSliceRows;
  } else {
    p = (int64_t)gl(M.rp)[row] + idx;
  }
  switch (M.dtype) {
    case F64: gl((double *)M.val)[p] = x; break;
    case F32: gl((float *)M.val)[p] = (float)x; break;
    case BF16: gl((uint16_t *)M.val)[p] = bf16_bits(x); break;
    default: gl((uint16_t *)M.val)[p] = f16_bits(x); break;
  }
}

__global__ __launch_bounds__(kBlock) void k_fsai_place(const int32_t *__restrict__ rp_, const int32_t *__restrict__ ci_,
                                                       const int32_t *__restrict__ dpos_,
                                                       const int32_t *__restrict__ lrp_, const double *__restrict__ lv_,
                                                       int32_t n, double scale, DevCSR GT, DevCSR G,
                                                       int32_t *__restrict__ err_) {
  GLOBAL const int32_t *rp = gl(rp_), *ci = gl(ci_), *dpos = gl(dpos_), *lrp = gl(lrp_);
  GLOBAL const double *lv = gl(lv_);
  for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const int32_t r0 = rp[i], m = dpos[i] - r0 + 1, base = lrp[i];
    for (int32_t k = 0; k < m; ++k) {
      const int32_t j = ci[r0 + k];
      const double x = lv[base + k] * scale;
      store_val(GT, i, k, j, x);
      // entry (j, i) of G = G_L^T: its rank in the upper part of A's row j
      int32_t lo = dpos[j], hi = rp[j + 1] - 1;
      while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (ci[mid] < i)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo > rp[j + 1] - 1 || ci[lo] != i) {
        gl(err_)[0] = 2;
        continue;
      }
      store_val(G, j, lo - dpos[j], i, x);
    }
  }
}

// ------------------------------------------------ multi-probe products (SAI loss)

template <typename TM>
__device__ __forceinline__ double ld64(GLOBAL const TM *p, int64_t k) {
  return (double)ldval(p, k);
}
__device__ __forceinline__ double ld64(GLOBAL const double *p, int64_t k) { return p[k]; }

// LPR lanes per row (a power of two >= the probe count, up to 64): a wave
// works on 64 / LPR rows at once, lane p of a group on probes p, p + LPR, ...
// Each group loads four entries' columns and values ahead of their gathers;
// the products are still added left to right.
template <typename TM, int LPR, typename TI>
__global__ __launch_bounds__(kBlock) PCG_OCCUPANCY void k_spmm(DevCSR Md, int32_t k, const double *__restrict__ X_,
                                                              double c, const double *__restrict__ Z_, double d,
                                                              double *__restrict__ Y_) {
  const Mat<TM> M = mat<TM>(Md);
  GLOBAL const double *X = gl(X_);
  GLOBAL const double *Z = Z_ ? gl(Z_) : nullptr;
  GLOBAL double *Y = gl(Y_);
  constexpr int RPW = 64 / LPR;  // rows per wave
  constexpr int NW = kBlock / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int grp = lane / LPR, pl = lane % LPR;
  const int64_t rows_per_block = (int64_t)NW * RPW;
  for (int64_t base = (int64_t)blockIdx.x * rows_per_block; base < M.n; base += (int64_t)gridDim.x * rows_per_block) {
    const int64_t r = base + (int64_t)wv * RPW + grp;
    const bool has = r < M.n;
    const int32_t row = has ? (int32_t)r : 0;
    int64_t e0 = 0, stride = 1;
    int32_t len = 0;
    if (has && M.fmt == FMT_SDIA) {  // one offset per slice entry; stored zeros add +0
      const int32_t sl = row / kSliceRows, o0 = M.blk[sl], wd = M.blk[sl + 1] - o0;
      GLOBAL const TM *vv = M.val + (int64_t)o0 * kSliceRows + row % kSliceRows;
      for (int32_t p0 = 0; p0 < k; p0 += LPR) {
        const int32_t p = p0 + pl;
        double sum = 0.0;
        for (int32_t e = 0; e < wd; ++e) {
          const int32_t col = min(max(row + M.ci[o0 + e], 0), M.n - 1);
          sum += ld64(vv, (int64_t)e * kSliceRows) * (p < k ? X[(int64_t)col * k + p] : 0.0);
        }
        if (p < k) {
          double y = c * sum;
          if (Z) y = y + d * Z[(int64_t)row * k + p];
          Y[(int64_t)row * k + p] = y;
        }
      }
      continue;
    }
    if (has && M.fmt == FMT_BSR3) {  // whole blocks: three entries of the row per block
      const int32_t R = row / 3, sub = row % 3, sl = R / kBSliceRows, rr = R % kBSliceRows;
      const int32_t o0 = M.blk[sl], wd = M.blk[sl + 1] - o0;
      for (int32_t p0 = 0; p0 < k; p0 += LPR) {
        const int32_t p = p0 + pl;
        double sum = 0.0;
        for (int32_t b = 0; b < wd; ++b) {
          const int64_t blk = ((int64_t)o0 + b) * kBSliceRows + rr;
          const int32_t c0 = 3 * M.ci[blk];
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const int64_t vi = sizeof(TM) == 8 ? (((int64_t)o0 + b) * 3 + j) * (3 * kBSliceRows) + sub * kBSliceRows + rr
                                               : (((int64_t)o0 + b) * kBSliceRows + rr) * 9 + 3 * sub + j;
            const double a = ld64(M.val, vi);
            sum += a * (p < k ? X[(int64_t)(c0 + j) * k + p] : 0.0);
          }
        }
        if (p < k) {
          double y = c * sum;
          if (Z) y = y + d * Z[(int64_t)row * k + p];
          Y[(int64_t)row * k + p] = y;
        }
      }
      continue;
    }
    if (has) {
      if (M.fmt == FMT_SELL) {  // padded entries add +0 (value 0, valid column)
        const int32_t sl = row / kSliceRows;
        e0 = (int64_t)M.blk[sl] * kSliceRows + row % kSliceRows;
        stride = kSliceRows;
        len = M.blk[sl + 1] - M.blk[sl];
      } else {
        e0 = M.rp[row];
        len = M.rp[row + 1] - M.rp[row];
      }
    }
    for (int32_t p0 = 0; p0 < k; p0 += LPR) {
      const int32_t p = p0 + pl;
      const bool act = has && p < k;
      double sum = 0.0;
      int32_t e = 0;
      for (; e + 4 <= len; e += 4) {
        int32_t col[4];
        double a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t q = e0 + (int64_t)(e + u) * stride;
          col[u] = col_at<TI>(M.ci, q, row);
          a[u] = ld64(M.val, q);
        }
        double x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = act ? X[(int64_t)col[u] * k + p] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) sum += a[u] * x[u];
      }
      for (; e < len; ++e) {
        const int64_t q = e0 + (int64_t)e * stride;
        const int32_t col = col_at<TI>(M.ci, q, row);
        const double a = ld64(M.val, q);
        sum += a * (act ? X[(int64_t)col * k + p] : 0.0);
      }
      if (act) {
        double y = c * sum;
        if (Z) y = y + d * Z[(int64_t)row * k + p];
        Y[(int64_t)row * k + p] = y;
      }
    }
  }
}

// Partial sums per workgroup (rows split in contiguous ranges), one lane per
// probe, each sum in row order.
__global__ __launch_bounds__(kBlock) void k_loss_partials(int32_t n, int32_t k, const double *__restrict__ W_,
                                                          const double *__restrict__ Y_, double na,
                                                          double *__restrict__ part_) {
  __shared__ double sh[5 * kBlock];
  GLOBAL const double *W = gl(W_), *Y = gl(Y_);
  GLOBAL double *part = gl(part_);
  const int64_t r0 = (int64_t)blockIdx.x * n / gridDim.x, r1 = (int64_t)(blockIdx.x + 1) * n / gridDim.x;
  const int t = threadIdx.x;
  const int lanes = kBlock;
  for (int32_t p0 = 0; p0 < k; p0 += lanes) {
    // thread t of group g = t / k2 handles probe p0 + t % k2 over rows r0 + g, r0 + g + ng, ...
    const int32_t kk = min(lanes, k - p0);
    const int ng = lanes / kk;
    const int g = t / kk, p = p0 + t % kk;
    double acc[5] = {0, 0, 0, 0, 0};
    if (g < ng)
      for (int64_t r = r0 + g; r < r1; r += ng) {
        const double w = W[r * k + p], y = Y[r * k + p];
        const double e = y / na - w, f = y - w;
        acc[0] += e * e;
        acc[1] += f * f;
        acc[2] += w * y;
        acc[3] += y * y;
        acc[4] += w * w;
      }
#pragma unroll
    for (int q = 0; q < 5; ++q) sh[q * kBlock + t] = (g < ng) ? acc[q] : 0.0;
    __syncthreads();
    if (t < kk) {  // fixed order over the groups
      for (int q = 0; q < 5; ++q) {
        double a = 0.0;
        for (int gg = 0; gg < ng; ++gg) a += sh[q * kBlock + gg * kk + t];
        part[((int64_t)blockIdx.x * 5 + q) * k + p0 + t] = a;
      }
    }
    __syncthreads();
  }
}

// One thread per probe: the workgroups' partial sums added in ascending
// workgroup order, then the three losses.
__global__ __launch_bounds__(kBlock) void k_loss_final(int32_t k, const double *__restrict__ part_,
                                                       double *__restrict__ out_) {
  const int32_t p = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
  if (p >= k) return;
  GLOBAL const double *part = gl(part_);
  GLOBAL double *out = gl(out_);
  double q[5] = {0, 0, 0, 0, 0};
  for (int b = 0; b < kLossGrid; ++b)
#pragma unroll
    for (int j = 0; j < 5; ++j) q[j] += part[((int64_t)b * 5 + j) * k + p];
  out[p] = q[0];
  out[(int64_t)k + p] = q[1];
  out[2 * (int64_t)k + p] = q[2] / (sqrt(q[4]) * sqrt(q[3]));
}

// The allocation-free entry point's scratch: one copy per device, allocated
// by the runtime with the code object. Host code uses only the per-device
// address that hipGetSymbolAddress returns for it.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(int device, void **ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
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

// Plain launch, or with events on the dispatch when timing.
#define PCG_LAUNCH(kern, grid, s, e0, e1, ...)                                                  \
  do {                                                                                          \
    if ((e0) || (e1))                                                                           \
      hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, e0, e1, 0, __VA_ARGS__);     \
    else                                                                                        \
      hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, __VA_ARGS__);                   \
  } while (0)

hipError_t launch_iter_A(const Types &ty, const LaunchSet &L, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (L.nA == 0) return hipSuccess;
  const bool u4 = L.uw_a == 4;
  if (ty.vec == F64 && ty.a == F64) {
    if (u4)
      PCG_LAUNCH((k_iter_A<double, double, 4>), L.nA, s, e0, e1, L.dir, L.mapA);
    else
      PCG_LAUNCH((k_iter_A<double, double, 8>), L.nA, s, e0, e1, L.dir, L.mapA);
  } else if (ty.vec == F32 && ty.a == F32) {
    if (u4)
      PCG_LAUNCH((k_iter_A<float, float, 4>), L.nA, s, e0, e1, L.dir, L.mapA);
    else
      PCG_LAUNCH((k_iter_A<float, float, 8>), L.nA, s, e0, e1, L.dir, L.mapA);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_iter_GT(const Types &ty, const LaunchSet &L, int mode, hipStream_t s, hipEvent_t e0,
                          hipEvent_t e1) {
  if (L.nGT == 0) return hipSuccess;
  PCG_DISPATCH_V(ty.vec, TV, PCG_DISPATCH_G(ty.g, TG, {
    PCG_LAUNCH((k_iter_GT<TV, TG>), L.nGT, s, e0, e1, L.dir, L.mapGT, mode);
  }));
  return hipGetLastError();
}

hipError_t launch_iter_G(const Types &ty, const LaunchSet &L, bool has_eps, int mode, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1) {
  if (L.nG == 0) return hipSuccess;
  PCG_DISPATCH_V(ty.vec, TV, PCG_DISPATCH_G(ty.g, TG, {
    if (has_eps)
      PCG_LAUNCH((k_iter_G<TV, TG, true>), L.nG, s, e0, e1, L.dir, L.mapG, mode);
    else
      PCG_LAUNCH((k_iter_G<TV, TG, false>), L.nG, s, e0, e1, L.dir, L.mapG, mode);
  }));
  return hipGetLastError();
}

hipError_t launch_resid(const Types &ty, const LaunchSet &L, int slot_sel, bool with_d, bool reduce,
                        bool respect_done, hipStream_t s) {
  if (L.nA == 0) return hipSuccess;
  if (ty.vec == F64 && ty.a == F64) {
    hipLaunchKernelGGL((k_resid<double, double>), dim3(L.nA), dim3(kBlock), 0, s, L.dir, L.mapA, slot_sel,
                       (int)with_d, (int)reduce, (int)respect_done);
  } else if (ty.vec == F32 && ty.a == F32) {
    hipLaunchKernelGGL((k_resid<float, float>), dim3(L.nA), dim3(kBlock), 0, s, L.dir, L.mapA, slot_sel,
                       (int)with_d, (int)reduce, (int)respect_done);
  } else {
    return hipErrorInvalidValue;
  }
  if (reduce) hipLaunchKernelGGL(k_reduce_state, dim3(L.nset), dim3(kBlock), 0, s, L.dir, L.set, 1);
  return hipGetLastError();
}

bool solve_wg_supported(const Types &ty) {
  return (ty.vec == F64 && ty.a == F64 && ty.g == F64) ||
         (ty.vec == F32 && ty.a == F32 && (ty.g == F32 || ty.g == BF16 || ty.g == F16));
}

hipError_t launch_solve_wg(const Types &ty, const LaunchSet &L, bool has_eps, hipStream_t s) {
  if (L.nset == 0) return hipSuccess;
#define PCG_SOLVE_WG(TV, TG)                                                                                   \
  do {                                                                                                         \
    if (has_eps)                                                                                               \
      hipLaunchKernelGGL((k_solve_wg<TV, TV, TG, true>), dim3(L.nset), dim3(kBlock), vec_bytes, s, L.dir,      \
                         L.set, vec_bytes);                                                                    \
    else                                                                                                       \
      hipLaunchKernelGGL((k_solve_wg<TV, TV, TG, false>), dim3(L.nset), dim3(kBlock), vec_bytes, s, L.dir,     \
                         L.set, vec_bytes);                                                                    \
  } while (0)
  if (!solve_wg_supported(ty)) return hipErrorInvalidValue;
  const int vec_bytes = ty.vec == F64 ? kWgVectors * 8 * L.wg_lds_rows8 : kWgVectors * 4 * L.wg_lds_rows4;
  if (ty.vec == F64)
    PCG_SOLVE_WG(double, double);
  else if (ty.g == F32)
    PCG_SOLVE_WG(float, float);
  else if (ty.g == BF16)
    PCG_SOLVE_WG(float, bf16_t);
  else
    PCG_SOLVE_WG(float, _Float16);
#undef PCG_SOLVE_WG
  return hipGetLastError();
}

hipError_t launch_finalize(const Types &ty, const LaunchSet &L, hipStream_t s) {
  if (L.nA == 0) return hipSuccess;
  PCG_DISPATCH_V(ty.vec, TV, {
    hipLaunchKernelGGL((k_finalize<TV>), dim3(L.nA), dim3(kBlock), 0, s, L.dir, L.mapA);
  });
  hipLaunchKernelGGL(k_state_clear_alpha, dim3((L.nset + 255) / 256), dim3(256), 0, s, L.dir, L.set, L.nset);
  return hipGetLastError();
}

hipError_t launch_norm_b(const Types &ty, const LaunchSet &L, hipStream_t s) {
  if (L.nB == 0) return hipSuccess;
  PCG_DISPATCH_V(ty.vec, TV, {
    hipLaunchKernelGGL((k_norm_b<TV>), dim3(L.nB), dim3(kBlock), 0, s, L.dir, L.mapB);
  });
  hipLaunchKernelGGL(k_reduce_state, dim3(L.nset), dim3(kBlock), 0, s, L.dir, L.set, 0);
  return hipGetLastError();
}

hipError_t launch_zero_dirs(const Types &ty, const LaunchSet &L, bool zero_x, hipStream_t s) {
  if (L.nA == 0) return hipSuccess;
  PCG_DISPATCH_V(ty.vec, TV, {
    hipLaunchKernelGGL((k_zero_dirs<TV>), dim3(L.nA), dim3(kBlock), 0, s, L.dir, L.mapA, (int)zero_x);
  });
  return hipGetLastError();
}

hipError_t launch_outer(int vec_dtype, const LaunchSet &L64, int what, hipStream_t s) {
  if (L64.nA == 0) return hipSuccess;
  PCG_DISPATCH_V(vec_dtype, TV, {
    hipLaunchKernelGGL((k_outer<TV>), dim3(L64.nA), dim3(kBlock), 0, s, L64.dir, L64.mapA, what);
  });
  return hipGetLastError();
}

hipError_t launch_state_restart(const LaunchSet &L, hipStream_t s) {
  if (L.nset == 0) return hipSuccess;
  hipLaunchKernelGGL(k_state_restart, dim3((L.nset + 255) / 256), dim3(256), 0, s, L.dir, L.set, L.nset);
  return hipGetLastError();
}

hipError_t launch_spmv(const Types &ty, const DevCSR &M, const void *x, void *y, hipStream_t s) {
  PCG_DISPATCH_V(ty.vec, TV, PCG_DISPATCH_G(M.dtype, TM, {
    hipLaunchKernelGGL((k_spmv<TV, TM>), dim3(M.grid), dim3(kBlock), 0, s, M, (const TV *)x, (TV *)y);
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

hipError_t launch_fsai_rows(const int32_t *rp, const int32_t *ci, const double *v, const int32_t *dpos,
                            const int32_t *lrp, int32_t n, int32_t mmax, double *lv, int32_t *err, int grid,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (mmax < 1 || mmax > kFsaiMaxRow) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * ((size_t)mmax * mmax + mmax) + sizeof(int32_t) * mmax;
  hipLaunchKernelGGL(k_fsai_rows, dim3(grid), dim3(64), lds, s, rp, ci, v, dpos, lrp, n, mmax, lv, err);
  return hipGetLastError();
}

hipError_t launch_absmax(const double *x, int64_t m, double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_absmax, dim3(kAbsmaxGrid), dim3(kBlock), 0, s, x, m, part);
  return hipGetLastError();
}

hipError_t launch_fsai_place(const int32_t *rp, const int32_t *ci, const int32_t *dpos, const int32_t *lrp,
                             const double *lv, int32_t n, double scale, const DevCSR &GT, const DevCSR &G,
                             int32_t *err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fsai_place, dim3(ew_grid(n)), dim3(kBlock), 0, s, rp, ci, dpos, lrp, lv, n, scale, GT, G, err);
  return hipGetLastError();
}

hipError_t launch_spmm(const DevCSR &M, int32_t k, const double *X, double c, const double *Z, double d, double *Y,
                       hipStream_t s) {
  if (M.n <= 0 || k <= 0) return hipSuccess;
  const int lpr = k >= 64 ? 64 : k > 16 ? 32 : k > 8 ? 16 : 8;
  const int64_t rows_per_block = (int64_t)(kBlock / 64) * (64 / lpr);
  const int grid = (int)std::min<int64_t>(((int64_t)M.n + rows_per_block - 1) / rows_per_block, 65536);
#define PCG_SPMM(L)                                                                                          \
  PCG_DISPATCH_G(M.dtype, TM, {                                                                              \
    if (M.idx16)                                                                                             \
      hipLaunchKernelGGL((k_spmm<TM, L, int16_t>), dim3(grid), dim3(kBlock), 0, s, M, k, X, c, Z, d, Y);     \
    else                                                                                                     \
      hipLaunchKernelGGL((k_spmm<TM, L, int32_t>), dim3(grid), dim3(kBlock), 0, s, M, k, X, c, Z, d, Y);     \
  })
  switch (lpr) {
    case 64: PCG_SPMM(64); break;
    case 32: PCG_SPMM(32); break;
    case 16: PCG_SPMM(16); break;
    default: PCG_SPMM(8); break;
  }
#undef PCG_SPMM
  return hipGetLastError();
}

hipError_t launch_loss_partials(int32_t n, int32_t k, const double *W, const double *Y, double na, double *part,
                                hipStream_t s) {
  if (n <= 0 || k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_loss_partials, dim3(kLossGrid), dim3(kBlock), 0, s, n, k, W, Y, na, part);
  return hipGetLastError();
}

hipError_t launch_loss_final(int32_t k, const double *part, double *out, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_loss_final, dim3((k + kBlock - 1) / kBlock), dim3(kBlock), 0, s, k, part, out);
  return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, int64_t bytes, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kBlock), 0, s, (const u32x4 *)src, (u32x4 *)dst, bytes / 16);
  return hipGetLastError();
}

hipError_t launch_read(const void *src, int64_t bytes, uint32_t *sink, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_read, dim3(grid), dim3(kBlock), 0, s, (const u32x4 *)src, bytes / 16, sink);
  return hipGetLastError();
}

}  // namespace pcgk
