// Host side of the C ABI in include/pcg.h: contexts, per-system device
// storage, launch sets, the single-system driver (captured HIP graphs of whole
// iterations, device-resident scalars), FP64 iterative refinement, and the
// batching / serving scheduler (device memory pool, host preparation worker,
// iteration-level continuous batching).
#include "pcg.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <optional>
#include <string>
#include <thread>

#include <sched.h>
#include <sys/resource.h>
#include <sys/syscall.h>
#include <unistd.h>
#include <unordered_map>
#include <vector>

#include "host.h"
#include "kernels.h"

using pcgk::DevCSR;
using pcgk::LaunchSet;
using pcgk::State;
using pcgk::SysDev;
using pcgk::Types;

namespace {

constexpr size_t kAlign = 256;
constexpr int kDirCap = 4096;  // systems per context (directory and state slots)
// defaults of pcg_config.wg_max_n and wg_max_n_batch: rows of a system solved
// by one persistent workgroup, alone (measured crossover with the three-kernel
// iteration near 500 rows) and in a batch (many systems at once)
constexpr int kWgMaxN = 512;
// default pcg_config.grid_mult: workgroups per CU of the iteration kernels
// (128^3 FP64: 94 us per iteration at 4, 102 at 8, 139 at 16)
constexpr int kGridMult = 4;
constexpr int kWgMaxNBatch = 16384;
// page-locked host memory per context for the device images of systems
// waiting for admission (larger or further images go to ordinary memory)
constexpr size_t kStagingBytes = size_t(256) << 20;
constexpr int kSlotMain = 0, kSlot64 = 1, kSlotX = 2, kFirstBatchSlot = 3;

inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------ device allocations

// Device memory of a context: hipMalloc/hipFree, or the caller's allocator
// (pcg_config.alloc / free). Before memory goes back to the caller's
// allocator the context's stream is drained, so no queued kernel still uses it.
struct DevAlloc {
  void *(*alloc)(size_t, void *) = nullptr;
  void (*release)(void *, void *) = nullptr;
  void *user = nullptr;
  hipStream_t stream = nullptr;
  hipError_t get(void **p, size_t bytes) const {
    if (!alloc) return hipMalloc(p, bytes);
    *p = alloc(bytes, user);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  void put(void *p) const {
    if (!p) return;
    if (!release) {
      (void)hipFree(p);
      return;
    }
    if (stream) (void)hipStreamSynchronize(stream);
    release(p, user);
  }
};

// ------------------------------------------------------------- range allocator

// First-fit allocation of byte ranges (offsets) of one region; free ranges
// coalesce with their neighbours. The region's memory belongs to the user.
class FirstFit {
 public:
  void reset(size_t cap) {
    free_.clear();
    used_.clear();
    cap_ = cap;
    used_bytes_ = 0;
    if (cap) free_[0] = cap;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = align_up(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t o = it->first, sz = it->second;
      free_.erase(it);
      if (sz > bytes) free_[o + bytes] = sz - bytes;
      used_[o] = bytes;
      used_bytes_ += bytes;
      *off = o;
      return true;
    }
    return false;
  }
  void release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t start = off, sz = u->second;
    used_bytes_ -= sz;
    used_.erase(u);
    auto nx = free_.lower_bound(start);
    if (nx != free_.end() && nx->first == start + sz) {
      sz += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == start) {
        start = pv->first;
        sz += pv->second;
        free_.erase(pv);
      }
    }
    free_[start] = sz;
  }
  size_t capacity() const { return cap_; }
  size_t in_use() const { return used_bytes_; }

 private:
  size_t cap_ = 0, used_bytes_ = 0;
  std::map<size_t, size_t> free_, used_;
};

// ---------------------------------------------------------------- device pool

// First-fit sub-allocator over one device allocation (the admission budget
// of the batch/serving scheduler).
class DevPool {
 public:
  DevAlloc da;
  ~DevPool() { reset(); }
  int init(size_t cap) {
    reset();
    cap = align_up(cap);
    if (da.get(&base_, cap) != hipSuccess) {
      (void)hipGetLastError();
      base_ = nullptr;
      return PCG_ENOMEM;
    }
    ff_.reset(cap);
    return PCG_OK;
  }
  void reset() {
    if (base_) da.put(base_);
    base_ = nullptr;
    ff_.reset(0);
  }
  bool ready() const { return base_ != nullptr; }
  void *alloc(size_t bytes) {
    size_t off;
    return base_ && ff_.alloc(bytes, &off) ? (uint8_t *)base_ + off : nullptr;
  }
  void release(void *p) {
    if (p && base_) ff_.release((size_t)((uint8_t *)p - (uint8_t *)base_));
  }
  size_t capacity() const { return ff_.capacity(); }
  size_t in_use() const { return ff_.in_use(); }

 private:
  void *base_ = nullptr;
  FirstFit ff_;
};

// ------------------------------------------------------------- pinned staging

// Page-locked host memory in which the worker threads lay out each admitted
// system's device image (matrices and vectors at their offsets in the pool
// block), so that admission uploads a system with one DMA copy per block
// instead of one pageable copy per array. Thread-safe; when it is full the
// image goes to ordinary memory (still one copy per block).
class PinnedArena {
 public:
  ~PinnedArena() {
    if (base_) (void)hipHostFree(base_);
  }
  // allocate the region once (false: no pinned memory, images go to the heap)
  bool init(size_t cap) {
    std::lock_guard<std::mutex> lk(mu_);
    if (base_ || tried_) return base_ != nullptr;
    tried_ = true;
    if (hipHostMalloc(&base_, cap, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      base_ = nullptr;
      return false;
    }
    ff_.reset(cap);
    return true;
  }
  void *alloc(size_t bytes) {
    std::lock_guard<std::mutex> lk(mu_);
    size_t off;
    return base_ && ff_.alloc(bytes, &off) ? (uint8_t *)base_ + off : nullptr;
  }
  void release(void *p) {
    std::lock_guard<std::mutex> lk(mu_);
    if (p && base_) ff_.release((size_t)((uint8_t *)p - (uint8_t *)base_));
  }

 private:
  std::mutex mu_;
  void *base_ = nullptr;
  bool tried_ = false;
  FirstFit ff_;
};

// ------------------------------------------------------- host staging of a system

// One sparse matrix laid out for the device on the host (see DevCSR).
struct HostMat {
  int32_t fmt = pcgk::FMT_CSR;
  int dt = pcgk::F64;
  int32_t n = 0;
  int64_t nnz = 0;           // nonzeros of the matrix (padding excluded)
  std::vector<int32_t> rp;   // CSR row pointers (FMT_CSR only)
  std::vector<int32_t> ci;   // columns in storage order
  std::vector<uint8_t> val;  // values in dt, in storage order (empty: written on the device)
  std::vector<int32_t> blk;  // row-block pairs (FMT_CSR) or slice offsets (sliced layouts)
  std::vector<int16_t> ci16; // FMT_SELL with idx16: column - row of each stored entry (ci then empty)
  int64_t stored = 0;        // stored indices (padding included)
  int32_t idx16 = 0;
  int32_t nunits = 0, grid = 8;
  int vpi = 1;  // values per stored index (9 for 3x3 blocks)
  size_t val_bytes() const { return pcgk::dtype_size(dt) * (size_t)vpi * (size_t)std::max<int64_t>(stored, 1); }
  size_t idx_bytes() const {
    if (fmt == pcgk::FMT_SDIA) return 4 * std::max<size_t>(ci.size(), 1);
    return (idx16 ? 2 : 4) * (size_t)std::max<int64_t>(stored, 1);
  }
  size_t bytes() const {
    return align_up(4 * rp.size()) + align_up(idx_bytes()) + align_up(val_bytes()) + align_up(4 * blk.size());
  }
};

// Sliced columns as 16-bit differences from their rows, when every stored
// entry's difference fits (entry p of a slice belongs to row 64 c + p % 64).
bool narrow_columns(HostMat &M) {
  const int64_t m = (int64_t)M.ci.size();
  for (int32_t c = 0; c < M.nunits; ++c)
    for (int64_t p = (int64_t)M.blk[c] * pcgk::kSliceRows; p < (int64_t)M.blk[c + 1] * pcgk::kSliceRows; ++p) {
      const int64_t d = (int64_t)M.ci[p] - ((int64_t)c * pcgk::kSliceRows + p % pcgk::kSliceRows);
      if (d < INT16_MIN || d > INT16_MAX) return false;
    }
  M.ci16.resize(m);
  for (int32_t c = 0; c < M.nunits; ++c)
    for (int64_t p = (int64_t)M.blk[c] * pcgk::kSliceRows; p < (int64_t)M.blk[c + 1] * pcgk::kSliceRows; ++p)
      M.ci16[p] = (int16_t)(M.ci[p] - (c * pcgk::kSliceRows + (int32_t)(p % pcgk::kSliceRows)));
  std::vector<int32_t>().swap(M.ci);
  M.idx16 = 1;
  return true;
}

// Everything a system's A part needs on the device, prepared on the host.
struct APart {
  int32_t n = 0;
  int64_t nnz = 0;
  int adt = pcgk::F64, vdt = pcgk::F64;
  bool refine = false, staging = false;
  HostMat A;
  // refinement view: FP64 values of A on A's pattern (shared on the device),
  // with its own row blocks in the CSR layout
  std::vector<uint8_t> sliced64;  // sliced FP64 values (FMT_SELL)
  const double *val64 = nullptr;  // CSR-ordered FP64 values (FMT_CSR, borrowed)
  std::vector<int32_t> blk64;
  int32_t nunits64 = 0, grid64 = 8, gB = 8;
  size_t bytes = 0;
};

struct GPart {
  int32_t n = 0;
  int64_t nnz = 0;
  int gdt = pcgk::F64, vdt = pcgk::F64;
  HostMat G, GT;
  double scale = 1.0;
  size_t bytes = 0;
};

// Device storage of one system.
struct Sys {
  int32_t n = 0;
  int64_t nnz_a = 0, nnz_g = 0;
  double g_scale = 1.0;
  SysDev dev{};    // directory entry
  SysDev dev64{};  // FP64 view for refinement (single path)
  SysDev devx{};   // FP64 inner solves after an escalation (single path; FP64 view of A, G as stored)
  void *blkA = nullptr, *blkG = nullptr, *blkX = nullptr;
  bool pooled = false;
  void *tmp_in = nullptr, *tmp_out = nullptr;
  double *stage64 = nullptr;
};

int grid_for(int cus, int mult, int32_t units) {
  if (mult <= 0) mult = kGridMult;
  int64_t g = std::min<int64_t>(units, (int64_t)cus * mult);
  g = (g + 7) & ~int64_t(7);
  return (int)std::max<int64_t>(g, 8);
}

int norm_grid(int32_t n) {
  int64_t g = ((int64_t)n + pcgk::kBlock - 1) / pcgk::kBlock;
  g = std::min<int64_t>(std::max<int64_t>(g, 1), 1024);
  return (int)((g + 7) & ~int64_t(7));
}

void cast_values(const double *v, int64_t nnz, int dt, double scale, std::vector<uint8_t> &out) {
  out.resize(pcgk::dtype_size(dt) * (size_t)std::max<int64_t>(nnz, 1));
  for (int64_t k = 0; k < nnz; ++k) {
    const double x = v[k] * scale;
    switch (dt) {
      case pcgk::F64: ((double *)out.data())[k] = x; break;
      case pcgk::F32: ((float *)out.data())[k] = (float)x; break;
      case pcgk::BF16: ((uint16_t *)out.data())[k] = pcgh::to_bf16_bits(x); break;
      default: ((uint16_t *)out.data())[k] = pcgh::to_f16_bits(x); break;
    }
  }
}

// Layout choice (pcg_config.layout): the sliced layout when its padding stays
// small, the CSR row blocks otherwise.
bool use_sell(int layout, int32_t n, const int32_t *rp) {
  if (layout == PCG_LAYOUT_CSR || n <= 0) return false;
  if (layout == PCG_LAYOUT_BSR3) layout = PCG_LAYOUT_AUTO;  // a matrix without 3x3 blocks
  const int64_t nnz = rp[n], stored = pcgh::sell_entries(n, rp);
  if (stored >= ((int64_t)1 << 31)) return false;
  if (layout == PCG_LAYOUT_SELL) return stored <= 2 * nnz + pcgh::kSlice;
  return stored <= nnz + nnz / 8;
}

// The sliced diagonal layout when a slice's rows share their column offsets:
// its stored values (zeros included) within 1/8 of the nonzeros (2x when
// asked for explicitly).
bool sdia_fits(int layout, int64_t nnz, int64_t stored) {
  if (stored >= ((int64_t)1 << 31)) return false;
  return layout == PCG_LAYOUT_SDIA ? stored <= 2 * nnz + pcgh::kSlice : stored <= nnz + nnz / 8;
}

bool sdia_allowed(int layout) {
  return layout == PCG_LAYOUT_AUTO || layout == PCG_LAYOUT_SDIA || layout == PCG_LAYOUT_BSR3;
}

bool use_sdia(int layout, int32_t n, const int32_t *rp, const int32_t *ci) {
  if (n <= 0 || !sdia_allowed(layout)) return false;
  const int64_t nnz = rp[n];
  const int64_t cap = layout == PCG_LAYOUT_SDIA ? 2 * nnz + pcgh::kSlice : nnz + nnz / 8;
  return sdia_fits(layout, nnz, pcgh::sdia_entries(n, rp, ci, cap));
}

// The sliced 3x3-block layout for an exactly 3x3-blocked matrix whose block
// padding stays within 1/8 (at most 2x when asked for explicitly).
bool use_bsr3(int layout, int32_t n, const int32_t *rp, const int32_t *ci) {
  if (layout != PCG_LAYOUT_AUTO && layout != PCG_LAYOUT_BSR3) return false;
  int64_t nb = 0;
  if (!pcgh::is_block3(n, rp, ci, &nb) || nb == 0) return false;
  const int64_t stored = pcgh::bsell_blocks(n, rp);
  if (stored * 9 >= ((int64_t)1 << 31)) return false;
  return layout == PCG_LAYOUT_BSR3 ? stored <= 2 * nb : stored <= nb + nb / 8;
}

// The slice offsets and listed offsets of the sliced diagonal layout into M
// (blk, ci), when the layout is allowed and fits. Irregular patterns are
// turned down after their first slices (the stored count only grows).
bool sdia_layout(int layout, int32_t n, const int32_t *rp, const int32_t *ci, HostMat &M) {
  if (n <= 0 || !sdia_allowed(layout)) return false;
  const int64_t nnz = rp[n];
  const int64_t cap = layout == PCG_LAYOUT_SDIA ? 2 * nnz + pcgh::kSlice : nnz + nnz / 8;
  if (pcgh::sdia_entries(n, rp, ci, cap) > cap) return false;
  pcgh::sdia_pattern(n, rp, ci, M.blk, M.ci);
  return sdia_fits(layout, nnz, (int64_t)M.ci.size() * pcgh::kSlice);
}

// Lay out one matrix's pattern (no values); the row blocks (CSR) are sized for
// products in vector type vdt. `blocks`: the 3x3-block layout may be used.
// Preference: 3x3 blocks, sliced diagonals, sliced ELL, CSR row blocks.
void make_pattern(const pcg_config &cfg, int cus, int32_t n, const int32_t *rp, const int32_t *ci, int dt, int vdt,
                  HostMat &M, bool blocks = false) {
  M.n = n;
  M.nnz = rp[n];
  M.dt = dt;
  M.vpi = 1;
  M.idx16 = 0;
  M.ci16.clear();
  M.val.clear();
  if (blocks && use_bsr3(cfg.layout, n, rp, ci)) {
    M.fmt = pcgk::FMT_BSR3;
    M.rp.clear();
    pcgh::bsell_pattern(n, rp, ci, M.blk, M.ci);
    M.vpi = 9;
    M.nunits = (int32_t)M.blk.size() - 1;
    const int32_t rounds = (M.nunits + pcgk::kBlock / 64 - 1) / (pcgk::kBlock / 64);
    M.grid = grid_for(cus, cfg.grid_mult, rounds);
  } else if (sdia_layout(cfg.layout, n, rp, ci, M)) {
    M.fmt = pcgk::FMT_SDIA;
    M.rp.clear();
    M.nunits = (int32_t)M.blk.size() - 1;
    const int32_t rounds = (M.nunits + pcgk::kBlock / 64 - 1) / (pcgk::kBlock / 64);
    M.grid = grid_for(cus, cfg.grid_mult, rounds);
    M.stored = (int64_t)M.ci.size() * pcgh::kSlice;
    return;
  } else if (use_sell(cfg.layout, n, rp)) {
    M.fmt = pcgk::FMT_SELL;
    M.rp.clear();
    pcgh::sell_offsets(n, rp, M.blk);
    pcgh::sell_columns(n, rp, ci, M.blk, M.ci);
    M.nunits = (int32_t)M.blk.size() - 1;
    const int32_t rounds = (M.nunits + pcgk::kBlock / 64 - 1) / (pcgk::kBlock / 64);
    M.grid = grid_for(cus, cfg.grid_mult, rounds);
    M.stored = (int64_t)M.ci.size();
    if (!cfg.wide_index) (void)narrow_columns(M);
    return;
  } else {
    M.fmt = pcgk::FMT_CSR;
    M.rp.assign(rp, rp + n + 1);
    M.ci.assign(ci, ci + M.nnz);
    M.blk = pcgh::row_blocks(n, rp, pcgk::lds_cap(vdt));
    M.nunits = (int32_t)(M.blk.size() / 2 - 1);
    M.grid = grid_for(cus, cfg.grid_mult, M.nunits);
  }
  M.stored = (int64_t)M.ci.size();
}

// The 3x3-block cover of a scalar pattern (n a multiple of 3, rows sorted):
// each row lists the three columns of every block that any row of its block
// row touches, in column order; src[k] is the original position of entry k,
// or -1 for an explicit zero (which adds +0 to its row's sum; the order of the
// original products is unchanged).
int64_t block_cover_size(int32_t n, const int32_t *rp, const int32_t *ci) {
  int64_t x = 0;
  std::vector<int32_t> bc;
  for (int32_t R = 0; R < n / 3; ++R) {
    bc.clear();
    for (int s = 0; s < 3; ++s)
      for (int32_t k = rp[3 * R + s]; k < rp[3 * R + s + 1]; ++k) bc.push_back(ci[k] / 3);
    std::sort(bc.begin(), bc.end());
    x += 9 * (int64_t)(std::unique(bc.begin(), bc.end()) - bc.begin());
  }
  return x;
}

void block_cover(int32_t n, const int32_t *rp, const int32_t *ci, std::vector<int32_t> &xrp,
                 std::vector<int32_t> &xci, std::vector<int64_t> &src) {
  xrp.assign((size_t)n + 1, 0);
  xci.clear();
  src.clear();
  std::vector<int32_t> bc;
  for (int32_t R = 0; R < n / 3; ++R) {
    bc.clear();
    for (int s = 0; s < 3; ++s)
      for (int32_t k = rp[3 * R + s]; k < rp[3 * R + s + 1]; ++k) bc.push_back(ci[k] / 3);
    std::sort(bc.begin(), bc.end());
    bc.erase(std::unique(bc.begin(), bc.end()), bc.end());
    for (int s = 0; s < 3; ++s) {
      const int32_t r = 3 * R + s;
      int32_t k = rp[r];
      for (int32_t B : bc)
        for (int j = 0; j < 3; ++j) {
          const int32_t c = 3 * B + j;
          while (k < rp[r + 1] && ci[k] < c) ++k;
          const bool hit = k < rp[r + 1] && ci[k] == c;
          xci.push_back(c);
          src.push_back(hit ? k : -1);
        }
      xrp[r + 1] = (int32_t)xci.size();
    }
  }
}

// Lay out one matrix with values v (CSR order) times `scale` in dt. blocks:
// 0 scalar layouts only; 1 also exact 3x3 blocks; 2 also the 3x3-block cover
// of a pattern that is not exactly blocked (explicit zeros pad it), when the
// cover adds at most 1/8 of the nonzeros (2x with the block layout forced).
void make_mat(const pcg_config &cfg, int cus, int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
              int dt, double scale, int vdt, HostMat &M, int blocks = 0) {
  if (blocks == 2 && n > 0 && n % 3 == 0 && (cfg.layout == PCG_LAYOUT_AUTO || cfg.layout == PCG_LAYOUT_BSR3) &&
      !pcgh::is_block3(n, rp, ci, nullptr)) {
    const int64_t nnz = rp[n], x = block_cover_size(n, rp, ci);
    const bool ok = x < ((int64_t)1 << 31) / 9 && (cfg.layout == PCG_LAYOUT_BSR3 ? x <= 2 * nnz : x <= nnz + nnz / 8);
    if (ok) {
      std::vector<int32_t> xrp, xci;
      std::vector<int64_t> src;
      block_cover(n, rp, ci, xrp, xci, src);
      std::vector<double> xv(x);
      for (int64_t k = 0; k < x; ++k) xv[k] = src[k] >= 0 ? v[src[k]] : 0.0;
      make_mat(cfg, cus, n, xrp.data(), xci.data(), xv.data(), dt, scale, vdt, M, 1);
      if (M.fmt == pcgk::FMT_BSR3) {
        M.nnz = nnz;  // the matrix's own nonzeros (explicit zeros are padding)
        return;
      }
    }
  }
  make_pattern(cfg, cus, n, rp, ci, dt, vdt, M, blocks != 0);
  std::vector<uint8_t> csr_val;
  cast_values(v, M.nnz, dt, scale, csr_val);
  if (M.fmt == pcgk::FMT_BSR3)
    pcgh::bsell_bytes(n, rp, csr_val.data(), pcgk::dtype_size(dt), M.blk, M.val);
  else if (M.fmt == pcgk::FMT_SDIA)
    pcgh::sdia_bytes(n, rp, ci, csr_val.data(), pcgk::dtype_size(dt), M.blk, M.ci, M.val);
  else if (M.fmt == pcgk::FMT_SELL)
    pcgh::sell_bytes(n, rp, csr_val.data(), pcgk::dtype_size(dt), M.blk, M.val);
  else
    M.val.swap(csr_val);
}

void prep_a(const pcg_config &cfg, int cus, int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
            bool staging, APart &P) {
  P.n = n;
  P.nnz = rp[n];
  P.adt = cfg.a_dtype;
  P.vdt = cfg.vec_dtype;
  P.refine = cfg.refine != 0;
  P.staging = staging;
  make_mat(cfg, cus, n, rp, ci, v, P.adt, 1.0, P.vdt, P.A, 1);
  P.gB = norm_grid(n);
  size_t b64 = 0;
  if (P.refine) {
    if (P.A.fmt != pcgk::FMT_CSR) {
      if (P.A.fmt == pcgk::FMT_BSR3)
        pcgh::bsell_bytes(n, rp, (const uint8_t *)v, 8, P.A.blk, P.sliced64);
      else if (P.A.fmt == pcgk::FMT_SDIA)
        pcgh::sdia_bytes(n, rp, ci, (const uint8_t *)v, 8, P.A.blk, P.A.ci, P.sliced64);
      else
        pcgh::sell_bytes(n, rp, (const uint8_t *)v, 8, P.A.blk, P.sliced64);
      P.nunits64 = P.A.nunits;
      P.grid64 = P.A.grid;
      b64 = align_up(P.sliced64.size());
    } else {
      P.val64 = v;
      P.blk64 = pcgh::row_blocks(n, rp, pcgk::lds_cap(pcgk::F64));
      P.nunits64 = (int32_t)(P.blk64.size() / 2 - 1);
      P.grid64 = grid_for(cus, cfg.grid_mult, P.nunits64);
      b64 = align_up(8 * (size_t)std::max<int64_t>(P.nnz, 1)) + align_up(4 * P.blk64.size());
    }
  }
  const size_t vb = align_up(pcgk::dtype_size(P.vdt) * (size_t)n), db = align_up(8 * (size_t)n);
  size_t b = P.A.bytes() + 8 * vb;
  if (P.refine) b += b64 + 3 * db;
  if (P.staging) b += 2 * vb + db;
  const int gtr = std::max(P.A.grid, P.refine ? P.grid64 : 0);
  constexpr size_t W = 8 * pcgk::kAccWords;  // bytes per partial sum
  b += align_up(W * (size_t)P.A.grid) + align_up(W * (size_t)gtr) + align_up(W * (size_t)P.gB);
  P.bytes = b;
}

void prep_g(const pcg_config &cfg, int cus, int32_t n, std::vector<int32_t> &grp, std::vector<int32_t> &gci,
            std::vector<double> &gv, GPart &P) {
  P.n = n;
  P.nnz = (int64_t)gci.size();
  P.gdt = cfg.g_dtype;
  P.vdt = cfg.vec_dtype;
  std::vector<int32_t> trp, tci;
  std::vector<double> tv;
  pcgh::transpose_csr(n, grp, gci, gv, trp, tci, tv);
  // F16 has a narrow exponent range: store G times a power of two (PCG is
  // invariant to the scale of M^-1 when eps is scaled alike).
  P.scale = 1.0;
  if (P.gdt == pcgk::F16) {
    double mx = 0.0;
    for (double x : gv) mx = std::max(mx, std::fabs(x));
    if (mx > 0) {
      int e;
      std::frexp(mx, &e);
      P.scale = std::ldexp(1.0, 14 - e);  // max |G| scaled into [2^13, 2^14)
    }
  }
  make_mat(cfg, cus, n, grp.data(), gci.data(), gv.data(), P.gdt, P.scale, P.vdt, P.G, 2);
  make_mat(cfg, cus, n, trp.data(), tci.data(), tv.data(), P.gdt, P.scale, P.vdt, P.GT, 2);
  P.bytes = P.G.bytes() + P.GT.bytes() + align_up(16 * pcgk::kAccWords * (size_t)P.GT.grid);
}

struct Carver {
  uint8_t *base;
  size_t off = 0;
  void *take(size_t bytes) {
    void *p = base + off;
    off += align_up(std::max<size_t>(bytes, 1));
    return p;
  }
};

hipError_t h2d(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (!bytes) return hipSuccess;
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
}

// Where placement sends the host data of a system: straight to the device
// on a stream (Device); into a host image of the block, which the carver
// then walks in place of the device block (Image: the carved pointers are
// image addresses); or nowhere (Bind: the carved pointers are the device
// block's, whose contents arrive as one copy of the image).
struct Copier {
  enum Mode { Device, Image, Bind } mode = Device;
  hipStream_t s = nullptr;
  hipError_t put(void *dst, const void *src, size_t bytes) const {
    if (!bytes || mode == Bind) return hipSuccess;
    if (mode == Image) {
      std::memcpy(dst, src, bytes);
      return hipSuccess;
    }
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  }
};

// Carve one matrix out of `c` and upload it into M.
hipError_t put_mat(Carver &c, const HostMat &H, DevCSR &M, const Copier &cp) {
  hipError_t e = hipSuccess;
  auto chain = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  int32_t *drp = H.rp.empty() ? nullptr : (int32_t *)c.take(4 * H.rp.size());
  int32_t *dci = (int32_t *)c.take(H.idx_bytes());
  void *dval = c.take(H.val_bytes());
  int32_t *dblk = (int32_t *)c.take(4 * H.blk.size());
  if (drp) chain(cp.put(drp, H.rp.data(), 4 * H.rp.size()));
  if (H.idx16)
    chain(cp.put(dci, H.ci16.data(), 2 * H.ci16.size()));
  else
    chain(cp.put(dci, H.ci.data(), 4 * H.ci.size()));
  if (!H.val.empty()) chain(cp.put(dval, H.val.data(), H.val.size()));
  chain(cp.put(dblk, H.blk.data(), 4 * H.blk.size()));
  M.rp = drp;
  M.ci = dci;
  M.val = dval;
  M.blk = dblk;
  M.nblk = H.nunits;
  M.grid = H.grid;
  M.nnz = H.nnz;
  M.n = H.n;
  M.dtype = H.dt;
  M.fmt = H.fmt;
  M.idx16 = H.idx16;
  M.nidx = H.idx16 ? (int64_t)H.ci16.size() : (int64_t)H.ci.size();
  return e;
}

// Carve the A part into `block` and upload it (asynchronously: P must live
// until the stream has passed the copies).
hipError_t place_a(const APart &P, void *block, Sys &S, const Copier &cp) {
  Carver c{(uint8_t *)block};
  const int32_t n = P.n;
  const size_t vb = pcgk::dtype_size(P.vdt) * (size_t)n;
  DevCSR &A = S.dev.A;
  hipError_t e = put_mat(c, P.A, A, cp);
  auto chain = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  void **vecs[] = {&S.dev.x, &S.dev.r0, &S.dev.r1, &S.dev.d0, &S.dev.d1, &S.dev.q, &S.dev.t, &S.dev.b};
  for (void **v : vecs) *v = c.take(vb);
  S.dev.s = nullptr;  // s = G t + eps r is folded into d by the G-kernel
  S.dev.n = n;
  S.dev.gB = P.gB;
  S.n = n;
  S.nnz_a = P.nnz;
  constexpr size_t W = 8 * pcgk::kAccWords;  // bytes per partial sum
  S.dev.pg = (double *)c.take(W * (size_t)P.A.grid);
  S.dev.ptr = (double *)c.take(W * (size_t)std::max(P.A.grid, P.refine ? P.grid64 : 0));
  S.dev.pb = (double *)c.take(W * (size_t)P.gB);
  if (P.refine) {
    SysDev &D = S.dev64;
    D = SysDev{};
    D.A = A;
    D.A.dtype = pcgk::F64;
    if (P.A.fmt != pcgk::FMT_CSR) {  // same slices and columns, FP64 values
      void *v64 = c.take(P.sliced64.size());
      chain(cp.put(v64, P.sliced64.data(), P.sliced64.size()));
      D.A.val = v64;
    } else {  // same CSR pattern, FP64 values, row blocks for FP64 products
      void *v64 = c.take(8 * (size_t)std::max<int64_t>(P.nnz, 1));
      int32_t *b64k = (int32_t *)c.take(4 * P.blk64.size());
      chain(cp.put(v64, P.val64, 8 * (size_t)P.nnz));
      chain(cp.put(b64k, P.blk64.data(), 4 * P.blk64.size()));
      D.A.val = v64;
      D.A.blk = b64k;
    }
    D.A.nblk = P.nunits64;
    D.A.grid = P.grid64;
    D.x = c.take(8 * (size_t)n);
    D.b = c.take(8 * (size_t)n);
    D.r0 = D.r1 = D.d0 = D.d1 = c.take(8 * (size_t)n);
    D.ptr = S.dev.ptr;
    D.pb = S.dev.pb;
    D.pg = S.dev.pg;
    D.n = n;
    D.gB = P.gB;
  }
  if (P.staging) {
    S.tmp_in = c.take(vb);
    S.tmp_out = c.take(vb);
    S.stage64 = (double *)c.take(8 * (size_t)n);
  }
  return e;
}

hipError_t place_g(const GPart &P, void *block, Sys &S, const Copier &cp) {
  Carver c{(uint8_t *)block};
  hipError_t e = put_mat(c, P.G, S.dev.G, cp);
  hipError_t e2 = put_mat(c, P.GT, S.dev.GT, cp);
  if (e == hipSuccess) e = e2;
  S.dev.prt = (double *)c.take(16 * pcgk::kAccWords * (size_t)P.GT.grid);
  S.nnz_g = P.nnz;
  S.g_scale = P.scale;
  return e;
}

// ------------------------------------------------------------ launch sets

struct HostSet {
  std::vector<int> slots;
  void *dev = nullptr;  // maps + set
  size_t cap = 0;       // bytes allocated at dev (reused by the next build)
  LaunchSet L{};
};

// ----------------------------------------------------------------- requests

enum ReqState { RQ_PREP, RQ_READY, RQ_ACTIVE, RQ_DONE };

struct Req {
  uint64_t ticket = 0;
  int32_t n = 0;
  std::vector<int32_t> a_rp, a_ci, g_rp, g_ci;
  std::vector<double> a_val, g_val, b, x0;
  int g_kind = PCG_G_FSAI;
  uint64_t g_seed = 0;
  bool g_given = false;
  double tol = 1e-8;
  int maxit = 1000;
  double *x_out = nullptr;
  APart ap;
  GPart gp;
  // FSAI factored on the device at admission: A's diagonal positions and
  // G_L's row pointers (the patterns of G and G^T are laid out in gp)
  bool dev_fsai = false;
  std::vector<int32_t> fs_dpos, fs_lrp;
  int32_t fs_mmax = 0;
  // device images of the A and G blocks laid out on the host (pinned when the
  // context's arena has room, else in heap); admission copies each in one go
  uint8_t *img_a = nullptr, *img_g = nullptr;
  bool img_pinned = false;
  std::vector<uint8_t> img_heap;
  size_t bytes = 0;
  int prep_rc = PCG_OK;
  ReqState st = RQ_PREP;
  Sys sys;
  int slot = -1;
  int slot64 = -1;  // FP64 view under refinement
  int restarts = 0;
  int outer = 0, inner_total = 0;
  int iter_host = 0;  // the system's iteration count at the start of the next scheduler step
  bool wg = false;    // solved whole by the one-workgroup solver (small system)
  double prev_rn = INFINITY, relres64 = NAN, last_rec = NAN;
  double t_submit = 0, t_admit = 0, t_done = 0;
  pcg_result res{};
};

}  // namespace

// ----------------------------------------------------------------- context

struct pcg_ctx {
  pcg_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = true;  // created here (destroyed with the context)
  DevAlloc da;
  int cus = 256;
  int lds_per_block = 65536;  // the device's LDS bytes per workgroup
  std::string err;
  Types ty{};

  // directory of systems and their state slots (device), with a host mirror
  SysDev *d_dir = nullptr;
  void *loss_buf = nullptr;  // scratch of pcg_sai_loss, kept between calls
  size_t loss_bytes = 0;
  void *static_scratch = nullptr;  // this device's copy of the library's file-scope scratch
  State *d_states = nullptr;  // kDirCap * 2
  State *h_states = nullptr;  // pinned mirror
  State *h_init = nullptr;    // pinned upload staging (2 slots)
  std::vector<SysDev> dir;    // host copy of the directory
  std::vector<int> free_slots;

  // single-system path
  std::vector<int32_t> a_rp, a_ci;
  std::vector<double> a_val;
  double a_mean_abs = 1.0;  // mean |A_ij| over the nonzeros (the SAI loss's ||A||)
  bool have_a = false, have_g = false;
  // G as last set from the host (kept for re-layouts), or built on the device
  std::vector<int32_t> g_rp, g_ci;
  std::vector<double> g_val;
  bool g_from_device = false;
  // layouts and grid the autotuner chose for the current A and G
  struct Tune {
    bool on = false;
    int la = PCG_LAYOUT_AUTO, lg = PCG_LAYOUT_AUTO, gm = 8;
    int res = -1;  // matrices read with ordinary loads (bit 0 A, 1 G, 2 G^T); -1: the residency plan
    int gt_rows = 2;  // rows per lane of the G^T-kernel over sliced diagonals (1 or 2)
    int a_uw = 8;     // loads in flight per lane of the A-kernel's one-row sliced walks (4 or 8)
  } tune;
  Sys single;
  HostSet set_main, set_64;
  std::map<int, hipGraphExec_t> graphs;    // key: iters*2 + replace_first
  std::map<int, hipGraphExec_t> graphs_x;  // the same for the escalated FP64 inner solves
  HostSet set_x;
  hipEvent_t ev[2] = {nullptr, nullptr}, t0 = nullptr, t1 = nullptr;

  // batching / serving
  DevPool pool;
  PinnedArena staging;  // host images of admitted systems (see build_images)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Req>> prep_q;   // awaiting host preparation
  int preparing = 0;                         // taken from prep_q by a worker, not yet ready
  std::deque<std::shared_ptr<Req>> ready_q;  // prepared, awaiting admission
  std::vector<std::shared_ptr<Req>> active;  // admitted
  std::unordered_map<uint64_t, std::shared_ptr<Req>> by_ticket;
  uint64_t next_ticket = 1;
  std::vector<std::thread> workers;
  bool stop = false;
  HostSet set_active, set_done, set_tmp, set_tmp64;  // device buffers reused from step to step
  // small admitted systems solved whole by the one-workgroup solver, each
  // launch over a group of them on the side stream (own, default priority)
  struct WgGroup {
    std::vector<std::shared_ptr<Req>> reqs;
    HostSet set;
    hipEvent_t start = nullptr, done = nullptr;
  };
  // device-time accounting of the batching facility (pcg_batch_stats_get)
  hipEvent_t step_ev[2] = {nullptr, nullptr};
  pcg_batch_stats stats{};
  uint64_t completed = 0;  // tickets finished so far (under mu)
  std::vector<WgGroup> wg_groups;
  hipStream_t side = nullptr;
  int wg_inflight = 0;
  bool active_dirty = true;
  // the scheduler step (K iterations over the active set) as a HIP graph,
  // valid until the active set changes
  hipGraphExec_t step_graph = nullptr;
  int step_graph_iters = 0;
};

namespace {

#define HIPCHK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                  \
      return PCG_EDEVICE;                                                            \
    }                                                                                \
  } while (0)

void drop_graphs(pcg_ctx *ctx) {
  for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
  ctx->graphs.clear();
  for (auto &kv : ctx->graphs_x) (void)hipGraphExecDestroy(kv.second);
  ctx->graphs_x.clear();
}

void free_set(pcg_ctx *ctx, HostSet &hs) {
  if (hs.dev) ctx->da.put(hs.dev);
  hs = HostSet{};
}

// Maps for the systems in `slots` (directory indices).
// The maps (system, local workgroup) of the four launch shapes and the slot
// list, staged on the host and uploaded in one copy. The set's device buffer
// is reused when large enough (no graph may still reference the old maps:
// callers drop their graphs first, and no kernel of the set is in flight).
int build_set(pcg_ctx *ctx, HostSet &hs, const std::vector<int> &slots) {
  void *keep = hs.dev;
  const size_t kcap = hs.cap;
  hs = HostSet{};
  hs.slots = slots;
  size_t nA = 0, nGT = 0, nG = 0, nB = 0;
  for (int sl : slots) {
    const SysDev &D = ctx->dir[sl];
    nA += D.A.grid;
    nGT += D.GT.grid;
    nG += D.G.grid;
    nB += D.gB;
  }
  const size_t nmap = nA + nGT + nG + nB;
  std::vector<int2> h(nmap + (slots.size() + 1) / 2);
  size_t o = 0;
  for (int sl : slots)
    for (int l = 0; l < ctx->dir[sl].A.grid; ++l) h[o++] = make_int2(sl, l);
  for (int sl : slots)
    for (int l = 0; l < ctx->dir[sl].GT.grid; ++l) h[o++] = make_int2(sl, l);
  for (int sl : slots)
    for (int l = 0; l < ctx->dir[sl].G.grid; ++l) h[o++] = make_int2(sl, l);
  for (int sl : slots)
    for (int l = 0; l < ctx->dir[sl].gB; ++l) h[o++] = make_int2(sl, l);
  if (!slots.empty()) std::memcpy(h.data() + nmap, slots.data(), 4 * slots.size());
  const size_t used = 8 * h.size(), bytes = used + 64;
  if (keep && kcap >= bytes) {
    hs.dev = keep;
    hs.cap = kcap;
  } else {
    ctx->da.put(keep);
    HIPCHK(ctx->da.get(&hs.dev, bytes));
    hs.cap = bytes;
  }
  if (used) HIPCHK(hipMemcpy(hs.dev, h.data(), used, hipMemcpyHostToDevice));
  const int2 *p = (const int2 *)hs.dev;
  LaunchSet &L = hs.L;
  L.dir = ctx->d_dir;
  L.mapA = p;
  L.nA = (int32_t)nA;
  L.mapGT = p + nA;
  L.nGT = (int32_t)nGT;
  L.mapG = p + nA + nGT;
  L.nG = (int32_t)nG;
  L.mapB = p + nA + nGT + nG;
  L.nB = (int32_t)nB;
  L.set = (const int32_t *)(p + nmap);
  L.nset = (int32_t)slots.size();
  // LDS for the one-workgroup solver's vectors: a set of one system may take
  // what the device gives a workgroup beyond the kernel's static LDS; a set
  // of many keeps to a share that leaves room for several workgroups per CU
  const int64_t cap = slots.size() == 1
                          ? std::min<int64_t>(pcgk::kWgLdsVecBytesOne, ctx->lds_per_block - pcgk::kWgStaticLdsBytes)
                          : pcgk::kWgLdsVecBytes;
  for (int sl : slots) {
    const int32_t n = ctx->dir[sl].n;
    if (7 * 8 * (int64_t)n <= cap) L.wg_lds_rows8 = std::max(L.wg_lds_rows8, n);
    if (7 * 4 * (int64_t)n <= cap) L.wg_lds_rows4 = std::max(L.wg_lds_rows4, n);
  }
  return PCG_OK;
}

// Kernel knobs of the configuration (0: the defaults).
int cfg_rows_per_lane(const pcg_config &c) { return c.rows_per_lane == 1 ? 1 : 2; }
int cfg_loads_in_flight(const pcg_config &c) { return c.loads_in_flight == 4 ? 4 : 8; }

int upload_dir_entry(pcg_ctx *ctx, int slot) {
  HIPCHK(hipMemcpy(ctx->d_dir + slot, &ctx->dir[slot], sizeof(SysDev), hipMemcpyHostToDevice));
  return PCG_OK;
}

void free_sys(pcg_ctx *ctx, Sys &S) {
  if (S.pooled) {
    ctx->pool.release(S.blkA);
    ctx->pool.release(S.blkG);
  } else {
    ctx->da.put(S.blkA);
    ctx->da.put(S.blkG);
  }
  ctx->da.put(S.blkX);
  S = Sys{};
}

// Initial scalars of a solve. The inner solves of refinement run without
// residual replacement (inner = true): their recurrence residual must be free
// to fall below the true-residual floor of an FP32 iterate, because the FP64
// outer residual is what corrects x.
State init_state(const pcg_ctx *ctx, double tol, int maxit, double g_scale, bool inner = false) {
  State st{};
  st.tol = tol;
  st.maxit = maxit;
  st.eps = ctx->cfg.eps * g_scale * g_scale;
  st.rr_period = inner ? 0 : ctx->cfg.rr_period;
  return st;
}

// --------------------------------------------------------- single-system path

// The configuration one matrix of the single system is laid out with: the
// context's, with the tuned layout and grid when the autotuner has chosen.
pcg_config eff_cfg(const pcg_ctx *ctx, bool for_g) {
  pcg_config c = ctx->cfg;
  if (ctx->tune.on) {
    c.layout = for_g ? ctx->tune.lg : ctx->tune.la;
    c.grid_mult = ctx->tune.gm;
  }
  return c;
}

// Bytes a product with a placed matrix reads from it, as stored: values
// (padding included), column information and row or slice pointers.
// vsize: bytes per stored value.
double stored_matrix_bytes(const DevCSR &M, double vsize) {
  switch (M.fmt) {
    case pcgk::FMT_SELL:  // one value and one index per slot
      return (double)M.nidx * (vsize + (M.idx16 ? 2.0 : 4.0)) + 4.0 * (M.nblk + 1.0);
    case pcgk::FMT_SDIA:  // 64 values and one offset per slice entry
      return (double)M.nidx * (pcgk::kSliceRows * vsize + 4.0) + 4.0 * (M.nblk + 1.0);
    case pcgk::FMT_BSR3:  // nine values and one index per stored block
      return (double)M.nidx * (9.0 * vsize + 4.0) + 4.0 * (M.nblk + 1.0);
    default:  // CSR with row blocks
      return (double)M.nnz * (vsize + 4.0) + 4.0 * (M.n + 1.0) + 8.0 * (M.nblk + 1.0);
  }
}

// Bytes of one placed matrix as stored (padding included).
double placed_bytes(const pcgk::DevCSR &M) {
  return stored_matrix_bytes(M, (double)pcgk::dtype_size(M.dtype));
}

// Residency plan of the single system: which matrices are read with ordinary
// loads, so that they stay in the memory-side cache (cfg.cache_mb, default
// 256 MB) from one iteration to the next, and which stream past it. All three
// when the matrices and the 8 iteration vectors fit in 90% of the cache;
// else the first of A alone, G and G^T together, G alone that fits in 75%
// (the vectors and the other matrices stream around it); else none. The FP64
// view of A under refinement always streams.
int residency_plan(const pcg_ctx *ctx) {
  if (ctx->tune.on && ctx->tune.res >= 0) return ctx->tune.res;
  if (ctx->cfg.cache_mb < 0) return 0;
  const double cap = (ctx->cfg.cache_mb > 0 ? ctx->cfg.cache_mb : 256) * 1048576.0;
  const pcgk::SysDev &D = ctx->single.dev;
  const double a = placed_bytes(D.A), g = placed_bytes(D.G) + placed_bytes(D.GT);
  const double v = 8.0 * D.n * (double)pcgk::dtype_size(ctx->ty.vec);
  if (a + g + v <= 0.9 * cap) return 7;
  if (a <= 0.75 * cap) return 1;
  if (g <= 0.75 * cap) return 6;
  if (placed_bytes(D.G) <= 0.75 * cap) return 2;
  return 0;
}

int single_sets(pcg_ctx *ctx) {
  drop_graphs(ctx);
  // the FP64 record of escalated inner solves refers to the placed G: rebuilt
  // at the next escalation
  ctx->da.put(ctx->single.blkX);
  ctx->single.blkX = nullptr;
  {
    const int r = residency_plan(ctx);
    ctx->single.dev.A.temporal = r & 1;
    ctx->single.dev.G.temporal = (r >> 1) & 1;
    ctx->single.dev.GT.temporal = (r >> 2) & 1;
    ctx->single.dev64.A.temporal = 0;
    ctx->single.dev.GT.rpl = ctx->tune.on ? ctx->tune.gt_rows : cfg_rows_per_lane(ctx->cfg);
    ctx->single.dev.G.rpl = ctx->single.dev.GT.rpl;
  }
  ctx->single.dev.st = ctx->d_states + 2 * kSlotMain;
  ctx->dir[kSlotMain] = ctx->single.dev;
  int rc = upload_dir_entry(ctx, kSlotMain);
  if (rc) return rc;
  if (ctx->cfg.refine) {
    ctx->single.dev64.st = ctx->d_states + 2 * kSlot64;
    ctx->dir[kSlot64] = ctx->single.dev64;
    if ((rc = upload_dir_entry(ctx, kSlot64))) return rc;
    if ((rc = build_set(ctx, ctx->set_64, {kSlot64}))) return rc;
  }
  if ((rc = build_set(ctx, ctx->set_main, {kSlotMain}))) return rc;
  ctx->set_main.L.uw_a = ctx->tune.on ? ctx->tune.a_uw : cfg_loads_in_flight(ctx->cfg);
  return PCG_OK;
}

void enqueue_iteration(pcg_ctx *ctx, const Types &ty, const LaunchSet &L, bool replace, double eps, hipError_t &e) {
  auto chain = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  chain(pcgk::launch_iter_A(ty, L, ctx->stream));
  if (replace) chain(pcgk::launch_resid(ty, L, 1, true, false, true, ctx->stream));
  const int mode = replace ? 1 : 0;
  chain(pcgk::launch_iter_GT(ty, L, mode, ctx->stream));
  chain(pcgk::launch_iter_G(ty, L, eps != 0.0, mode, ctx->stream));
}

// What a single-system PCG runs on: the kernels' types, the launch set, the
// directory record (state slot, vectors) and the graph cache.
struct Core {
  Types ty;
  const LaunchSet *L;
  SysDev *dev;
  int slot;
  std::map<int, hipGraphExec_t> *graphs;
};

Core main_core(pcg_ctx *ctx) { return Core{ctx->ty, &ctx->set_main.L, &ctx->single.dev, kSlotMain, &ctx->graphs}; }

int get_graph(pcg_ctx *ctx, const Core &c, int iters, bool replace_first, double eps, hipGraphExec_t *out) {
  const int key = iters * 2 + (replace_first ? 1 : 0);
  auto it = c.graphs->find(key);
  if (it != c.graphs->end()) {
    *out = it->second;
    return PCG_OK;
  }
  HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int k = 0; k < iters; ++k) enqueue_iteration(ctx, c.ty, *c.L, replace_first && k == 0, eps, e);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(ctx->stream, &g);
  HIPCHK(e);
  HIPCHK(e2);
  hipGraphExec_t ex = nullptr;
  hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(e3);
  (*c.graphs)[key] = ex;
  *out = ex;
  return PCG_OK;
}

struct CoreOut {
  int status = PCG_OK;
  int iters = 0, restarts = 0;
  double rr = 0, true_rr = 0, bb = 0;
};

// Start sequence for the systems of L: ||b||, r = b - A x, t = G^T r,
// d = G t (+ eps r), delta (states already uploaded; x loaded).
int enqueue_start(pcg_ctx *ctx, const Types &ty, const LaunchSet &L, bool has_eps) {
  hipStream_t s = ctx->stream;
  HIPCHK(pcgk::launch_zero_dirs(ty, L, false, s));
  HIPCHK(pcgk::launch_norm_b(ty, L, s));
  HIPCHK(pcgk::launch_resid(ty, L, 0, false, false, true, s));
  HIPCHK(pcgk::launch_iter_GT(ty, L, 2, s));
  HIPCHK(pcgk::launch_iter_G(ty, L, has_eps, 2, s));
  return PCG_OK;
}

// PCG on the single system (b and x0 loaded). confirm: when the recurrence
// residual meets tol, check b - A x and restart from it if that fails (the
// inner solves of refinement skip this: the FP64 outer residual is the check,
// and an FP32 iterate's true residual has a floor near u32 ||A|| ||x||).
// The single system goes to the one-workgroup solver: small enough, and a
// storage-type combination it is built for.
bool use_solve_wg(const pcg_ctx *ctx, const Types &ty, int32_t n, bool batch = false) {
  const int cf = batch ? ctx->cfg.wg_max_n_batch : ctx->cfg.wg_max_n;
  const int lim = cf == 0 ? (batch ? kWgMaxNBatch : kWgMaxN) : cf;
  return lim > 0 && n <= lim && pcgk::solve_wg_supported(ty);
}

int solve_core(pcg_ctx *ctx, const Core &c, double tol, int maxit, CoreOut &out, bool confirm = true) {
  const Types &ty = c.ty;
  const LaunchSet &L = *c.L;
  SysDev &D = *c.dev;
  hipStream_t s = ctx->stream;
  State init = init_state(ctx, tol, maxit, ctx->single.g_scale, !confirm);
  const bool has_eps = init.eps != 0.0;
  init.confirm = confirm ? 1 : 0;
  ctx->h_init[0] = init;
  ctx->h_init[1] = init;
  HIPCHK(hipMemcpyAsync(D.st, ctx->h_init, 2 * sizeof(State), hipMemcpyHostToDevice, s));
  if (use_solve_wg(ctx, ty, D.n)) {  // the whole solve in one launch
    HIPCHK(pcgk::launch_solve_wg(ty, L, has_eps, s));
    State *hst = ctx->h_states + 2 * c.slot;
    HIPCHK(hipMemcpyAsync(hst, D.st, sizeof(State), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const State f = *hst;
    out = CoreOut{};
    if (f.status == pcgk::ST_ZERO_B) return PCG_OK;
    out.iters = f.iter;
    out.rr = f.rr;
    out.true_rr = f.true_rr;
    out.bb = f.bb;
    out.restarts = f.restarts;
    out.status = f.status == pcgk::ST_CONV_REC ? PCG_OK
                 : f.status == pcgk::ST_MAXIT  ? PCG_NOT_CONVERGED
                                               : PCG_EBREAKDOWN;
    return PCG_OK;
  }
  {
    int rc = enqueue_start(ctx, ty, L, has_eps);
    if (rc) return rc;
  }
  const int rr = init.rr_period;
  int K = ctx->cfg.graph_iters;
  if (K > 0 && rr > 0) {
    int a = K, b = rr;
    while (b) {
      int t = a % b;
      a = b;
      b = t;
    }
    K = a;  // K divides rr: replacement can only fall on a chunk's first iteration
  }
  State *hst = ctx->h_states + 2 * c.slot;  // two pinned readback buffers
  int base = 0;
  int restarts = 0;
  for (;;) {
    int inflight = 0, slot_next = 0, slot_wait = 0;
    bool done = false;
    while (!done) {
      while (inflight < 2) {
        const bool rep = rr > 0 && base > 0 && base % rr == 0;
        int len;
        if (K <= 0) {
          hipError_t e = hipSuccess;
          enqueue_iteration(ctx, ty, L, rep, init.eps, e);
          HIPCHK(e);
          len = 1;
        } else {
          len = (base % K == 0) ? K : 1;
          hipGraphExec_t g;
          int rc = get_graph(ctx, c, len, rep, init.eps, &g);
          if (rc) return rc;
          HIPCHK(hipGraphLaunch(g, s));
        }
        base += len;
        HIPCHK(hipMemcpyAsync(&hst[slot_next], D.st, sizeof(State), hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(ctx->ev[slot_next], s));
        slot_next ^= 1;
        ++inflight;
      }
      HIPCHK(hipEventSynchronize(ctx->ev[slot_wait]));
      const bool d = hst[slot_wait].done != 0;
      slot_wait ^= 1;
      --inflight;
      if (d) done = true;
    }
    HIPCHK(hipStreamSynchronize(s));
    State h;
    HIPCHK(hipMemcpy(&h, D.st, sizeof(State), hipMemcpyDeviceToHost));
    if (h.status == pcgk::ST_ZERO_B) {
      HIPCHK(pcgk::launch_fill(ty.vec, D.x, ctx->single.n, 0.0, s));
      HIPCHK(hipStreamSynchronize(s));
      out = CoreOut{};
      return PCG_OK;
    }
    HIPCHK(pcgk::launch_finalize(ty, L, s));
    HIPCHK(pcgk::launch_resid(ty, L, 0, false, true, false, s));
    HIPCHK(hipMemcpyAsync(&hst[0], D.st, sizeof(State), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const State f = hst[0];
    out.iters = f.iter;
    out.rr = f.rr;
    out.true_rr = f.true_rr;
    out.bb = f.bb;
    out.restarts = restarts;
    if (f.status == pcgk::ST_CONV_REC) {
      if (!confirm || std::sqrt(f.true_rr) <= f.tol_nb) {
        out.status = PCG_OK;
        return PCG_OK;
      }
      // restart from the true residual (now in the current r slot)
      ++restarts;
      HIPCHK(pcgk::launch_state_restart(L, s));
      HIPCHK(pcgk::launch_iter_GT(ty, L, 2, s));
      HIPCHK(pcgk::launch_iter_G(ty, L, has_eps, 2, s));
      base = f.iter;
      continue;
    }
    out.status = (f.status == pcgk::ST_MAXIT) ? PCG_NOT_CONVERGED : PCG_EBREAKDOWN;
    return PCG_OK;
  }
}

int load_vec(pcg_ctx *ctx, const double *src, int on_device, void *dst, int dtype, int32_t n) {
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (dtype == pcgk::F64) {
    HIPCHK(hipMemcpyAsync(dst, src, sizeof(double) * n, kind, ctx->stream));
    return PCG_OK;
  }
  const double *dsrc = src;
  if (!on_device) {  // stage host FP64 through the device FP64 buffer
    HIPCHK(hipMemcpyAsync(ctx->single.stage64, src, sizeof(double) * n, kind, ctx->stream));
    dsrc = ctx->single.stage64;
  }
  HIPCHK(pcgk::launch_convert(pcgk::F64, dsrc, dtype, dst, n, 1.0, ctx->stream));
  return PCG_OK;
}

int store_vec(pcg_ctx *ctx, const void *src, int dtype, double *dst, int on_device, int32_t n) {
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (dtype == pcgk::F64) {
    HIPCHK(hipMemcpyAsync(dst, src, sizeof(double) * n, kind, ctx->stream));
  } else if (on_device) {
    HIPCHK(pcgk::launch_convert(dtype, src, pcgk::F64, dst, n, 1.0, ctx->stream));
  } else {
    HIPCHK(pcgk::launch_convert(dtype, src, pcgk::F64, ctx->single.stage64, n, 1.0, ctx->stream));
    HIPCHK(hipMemcpyAsync(dst, ctx->single.stage64, sizeof(double) * n, kind, ctx->stream));
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return PCG_OK;
}

// Relative tolerance of inner solve number `step` (0 first). A solve runs to
// the configured tolerance, or to what brings ||r64|| from rn to a quarter of
// the target tol*nb when that is looser (the margin covers the gap between the
// inner solve's recurrence residual and the FP64 residual), never looser than
// 1/2. After the first step, whose result shows how deep the inner solve gets
// in its precision, the step that can finish also runs to that target when it
// is up to ten times tighter than the configured tolerance: one longer inner
// solve instead of one more outer step, which would restart the Krylov space.
double inner_tolerance(double cfg_inner_tol, double tol, double nb, double rn, int step) {
  const double base = cfg_inner_tol > 0 ? cfg_inner_tol : 1e-6;
  const double target = 0.25 * tol * nb / rn;
  if (target >= base || (step > 0 && target >= 0.1 * base)) return std::min(0.5, target);
  return base;
}

// Row blocks of a stored CSR matrix for products in FP64 vectors: the
// blocks a matrix was laid out with hold up to lds_cap(vec type) nonzeros,
// twice what an FP64 product's LDS window takes when the vectors are FP32.
// The row pointers are read back from the device.
int f64_row_blocks(pcg_ctx *ctx, const DevCSR &M, std::vector<int32_t> &blk) {
  std::vector<int32_t> rp((size_t)M.n + 1);
  HIPCHK(hipMemcpy(rp.data(), M.rp, 4 * rp.size(), hipMemcpyDeviceToHost));
  blk = pcgh::row_blocks(M.n, rp.data(), pcgk::lds_cap(pcgk::F64));
  return PCG_OK;
}

// The FP64 record of escalated inner solves: A's FP64 view, G and G^T as
// stored, FP64 vectors and partial sums of its own (allocated at the first
// escalation, kept until the system's storage is freed). G or G^T stored as
// CSR row blocks get blocks of their own, sized for FP64 products.
int prepare_escalation(pcg_ctx *ctx) {
  Sys &S = ctx->single;
  if (S.blkX) return PCG_OK;
  const int32_t n = S.n;
  std::vector<int32_t> bg, bgt;
  int rc0;
  if (S.dev.G.fmt == pcgk::FMT_CSR && (rc0 = f64_row_blocks(ctx, S.dev.G, bg))) return rc0;
  if (S.dev.GT.fmt == pcgk::FMT_CSR && (rc0 = f64_row_blocks(ctx, S.dev.GT, bgt))) return rc0;
  const pcg_config gcfg = eff_cfg(ctx, true);
  const int gm = gcfg.grid_mult;
  auto nunits = [](const std::vector<int32_t> &b) { return (int32_t)(b.size() / 2 - 1); };
  const int ga = S.dev64.A.grid, gb = S.dev.gB;
  const int gt = bgt.empty() ? S.dev.GT.grid : grid_for(ctx->cus, gm, nunits(bgt));
  const size_t vb = align_up(8 * (size_t)n);
  constexpr size_t W = 8 * pcgk::kAccWords;  // bytes per partial sum
  const size_t bytes = 8 * vb + align_up(W * (size_t)ga) * 2 + align_up(2 * W * (size_t)gt) + align_up(W * (size_t)gb) +
                       align_up(4 * bg.size()) + align_up(4 * bgt.size());
  void *blk = nullptr;
  if (ctx->da.get(&blk, bytes) != hipSuccess) {
    (void)hipGetLastError();
    ctx->err = "refinement: allocation for the FP64 inner solve failed";
    return PCG_ENOMEM;
  }
  S.blkX = blk;
  Carver c{(uint8_t *)blk};
  SysDev &D = S.devx;
  D = SysDev{};
  D.A = S.dev64.A;
  D.G = S.dev.G;
  D.GT = S.dev.GT;
  void **vecs[] = {&D.x, &D.r0, &D.r1, &D.d0, &D.d1, &D.q, &D.t, &D.b};
  for (void **v : vecs) *v = c.take(8 * (size_t)n);
  D.s = nullptr;
  D.pg = (double *)c.take(W * (size_t)ga);
  D.ptr = (double *)c.take(W * (size_t)ga);
  D.prt = (double *)c.take(2 * W * (size_t)gt);
  D.pb = (double *)c.take(W * (size_t)gb);
  auto put_blocks = [&](const std::vector<int32_t> &b, DevCSR &M) -> hipError_t {
    if (b.empty()) return hipSuccess;
    int32_t *d = (int32_t *)c.take(4 * b.size());
    M.blk = d;
    M.nblk = nunits(b);
    M.grid = grid_for(ctx->cus, gm, M.nblk);
    return hipMemcpy(d, b.data(), 4 * b.size(), hipMemcpyHostToDevice);
  };
  HIPCHK(put_blocks(bg, D.G));
  HIPCHK(put_blocks(bgt, D.GT));
  D.n = n;
  D.gB = gb;
  D.st = ctx->d_states + 2 * kSlotX;
  ctx->dir[kSlotX] = D;
  int rc = upload_dir_entry(ctx, kSlotX);
  if (!rc) rc = build_set(ctx, ctx->set_x, {kSlotX});
  return rc;
}

// FP64 iterative refinement: r64 = b - A64 x64 in FP64; inner PCG on
// A c = r64 / ||r64|| to the inner tolerance; x64 += ||r64|| c. An outer step
// that gains less than 2x (or an inner breakdown, the stored operator not
// being SPD in its precision) escalates: from then on the inner solves run in
// FP64 (FP64 view of A, FP64 vectors, G as stored); escalated steps that gain
// less than 10% end the solve (PCG_NOT_CONVERGED).
int refine_solve(pcg_ctx *ctx, double tol, int maxit, pcg_result *res) {
  Sys &S = ctx->single;
  const int32_t n = S.n;
  hipStream_t s = ctx->stream;
  const Types t64{pcgk::F64, pcgk::F64, pcgk::F64};
  const LaunchSet &L64 = ctx->set_64.L;
  State init{};
  init.tol = tol;
  ctx->h_init[0] = init;
  ctx->h_init[1] = init;
  HIPCHK(hipMemcpyAsync(S.dev64.st, ctx->h_init, 2 * sizeof(State), hipMemcpyHostToDevice, s));
  HIPCHK(pcgk::launch_norm_b(t64, L64, s));
  int total_iters = 0, outer = 0, restarts = 0, status = PCG_NOT_CONVERGED;
  bool escalated = false;
  double prev = INFINITY, relres = NAN, last_rec = NAN;
  const int max_outer = ctx->cfg.max_outer > 0 ? ctx->cfg.max_outer : 30;
  State *hst = ctx->h_states + 2 * kSlot64;
  bool redo = false;  // repeat the step escalated (its FP32 inner solve broke down)
  double rn = 0.0, nb = 0.0;
  for (;;) {
    if (!redo) {
      HIPCHK(pcgk::launch_resid(t64, L64, 0, false, true, false, s));
      HIPCHK(hipMemcpyAsync(hst, S.dev64.st, sizeof(State), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      const State h = *hst;
      if (h.bb == 0.0) {
        HIPCHK(pcgk::launch_fill(pcgk::F64, S.dev64.x, n, 0.0, s));
        status = PCG_OK;
        relres = 0.0;
        break;
      }
      rn = std::sqrt(h.true_rr);
      nb = std::sqrt(h.bb);
      relres = rn / nb;
      if (rn <= tol * nb) {
        status = PCG_OK;
        break;
      }
      if (!std::isfinite(rn)) {
        status = PCG_EBREAKDOWN;
        break;
      }
      if (outer >= max_outer || (escalated && rn > 0.9 * prev)) {
        status = PCG_NOT_CONVERGED;
        break;
      }
      if (!escalated && rn > 0.5 * prev) escalated = true;
      prev = rn;
    }
    redo = false;
    const double eta = inner_tolerance(ctx->cfg.inner_tol, tol, nb, rn, outer);
    CoreOut co;
    int rc;
    if (escalated) {
      if ((rc = prepare_escalation(ctx))) return rc;
      const Core cx{Types{pcgk::F64, pcgk::F64, ctx->ty.g}, &ctx->set_x.L, &S.devx, kSlotX, &ctx->graphs_x};
      HIPCHK(pcgk::launch_convert(pcgk::F64, S.dev64.r0, pcgk::F64, S.devx.b, n, 1.0 / rn, s));
      HIPCHK(pcgk::launch_fill(pcgk::F64, S.devx.x, n, 0.0, s));
      rc = solve_core(ctx, cx, eta, maxit, co, false);
    } else {
      // inner right-hand side: r64 / ||r64|| in the vector precision
      HIPCHK(pcgk::launch_convert(pcgk::F64, S.dev64.r0, ctx->ty.vec, S.dev.b, n, 1.0 / rn, s));
      HIPCHK(pcgk::launch_fill(ctx->ty.vec, S.dev.x, n, 0.0, s));
      rc = solve_core(ctx, main_core(ctx), eta, maxit, co, false);
    }
    if (rc) return rc;
    total_iters += co.iters;
    restarts += co.restarts;
    last_rec = co.bb > 0 ? std::sqrt(co.rr / co.bb) : 0.0;
    if (co.status == PCG_EBREAKDOWN) {
      if (!escalated) {
        escalated = redo = true;
        continue;
      }
      status = PCG_EBREAKDOWN;
      break;
    }
    if (escalated)
      HIPCHK(pcgk::launch_refine_update(n, (double *)S.dev64.x, S.devx.x, pcgk::F64, rn, s));
    else
      HIPCHK(pcgk::launch_refine_update(n, (double *)S.dev64.x, S.dev.x, ctx->ty.vec, rn, s));
    ++outer;
  }
  if (res) {
    res->status = status;
    res->iters = total_iters;
    res->outer_iters = outer;
    res->restarts = restarts;
    res->relres_true = relres;
    res->relres_rec = last_rec;
    res->escalated = escalated ? 1 : 0;
  }
  return status;
}

// ------------------------------------------------------- batching / serving

// Host part of a device FSAI for a batched system (integer work only): the
// diagonal positions, the patterns of G_L (tril) and G = G_L^T (triu), laid
// out for the device. False when the device builder does not apply (a row of
// tril(A) longer than it handles, a missing diagonal, or an unsymmetric
// pattern): the host builder is used then.
bool prep_fsai_pattern(const pcg_config &cfg, int cus, Req &R) {
  const int32_t n = R.n;
  const int32_t *rp = R.a_rp.data(), *ci = R.a_ci.data();
  std::vector<int32_t> dpos(n), lrp(n + 1, 0), grp(n + 1, 0);
  int32_t mmax = 0;
  for (int32_t i = 0; i < n; ++i) {
    int32_t d = -1;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] == i) d = k;
    if (d < 0) return false;
    dpos[i] = d;
    mmax = std::max(mmax, d - rp[i] + 1);
    lrp[i + 1] = lrp[i] + (d - rp[i] + 1);
    grp[i + 1] = grp[i] + (rp[i + 1] - d);
  }
  if (mmax > pcgk::kFsaiMaxRow || lrp[n] != grp[n]) return false;
  for (int32_t i = 0; i < n; ++i)  // structural symmetry: (j, i) stored for every (i, j), j < i
    for (int32_t k = rp[i]; k < dpos[i]; ++k) {
      const int32_t j = ci[k];
      if (!std::binary_search(ci + dpos[j], ci + rp[j + 1], i)) return false;
    }
  std::vector<int32_t> lci(lrp[n]), gci(grp[n]);
  for (int32_t i = 0; i < n; ++i) {
    std::copy(ci + rp[i], ci + dpos[i] + 1, lci.begin() + lrp[i]);
    std::copy(ci + dpos[i], ci + rp[i + 1], gci.begin() + grp[i]);
  }
  GPart &P = R.gp;
  P = GPart{};
  P.n = n;
  P.nnz = lrp[n];
  P.gdt = cfg.g_dtype;
  P.vdt = cfg.vec_dtype;
  make_pattern(cfg, cus, n, grp.data(), gci.data(), P.gdt, P.vdt, P.G);
  make_pattern(cfg, cus, n, lrp.data(), lci.data(), P.gdt, P.vdt, P.GT);
  P.bytes = P.G.bytes() + P.GT.bytes() + align_up(16 * pcgk::kAccWords * (size_t)P.GT.grid);
  R.fs_dpos.swap(dpos);
  R.fs_lrp.swap(lrp);
  R.fs_mmax = mmax;
  R.dev_fsai = true;
  return true;
}

void prep_parts(const pcg_config &cfg, int cus, Req &R);

// Lay out the device images of the request's two pool blocks on the host:
// matrices, and the right-hand side and starting guess in the vector type
// (FP32 by round-to-nearest, as the device conversion rounds), or their FP64
// view under refinement. The image holds what the placement would copy, at
// the same offsets; the rest of the block (work vectors, partial sums) is
// left as it comes.
void build_images(const pcg_config &cfg, PinnedArena *arena, Req &R) {
  const size_t na = align_up(R.ap.bytes), ng = align_up(R.gp.bytes);
  uint8_t *img = arena ? (uint8_t *)arena->alloc(na + ng) : nullptr;
  R.img_pinned = img != nullptr;
  if (!img) {
    R.img_heap.resize(na + ng);
    img = R.img_heap.data();
  }
  R.img_a = img;
  R.img_g = img + na;
  Sys tmp;
  (void)place_a(R.ap, R.img_a, tmp, Copier{Copier::Image});
  (void)place_g(R.gp, R.img_g, tmp, Copier{Copier::Image});
  const int32_t n = R.n;
  auto put_vec = [&](void *dst, const std::vector<double> &v, int dt) {
    if (dt == pcgk::F64) {
      if (v.empty())
        std::memset(dst, 0, 8 * (size_t)n);
      else
        std::memcpy(dst, v.data(), 8 * (size_t)n);
    } else {
      float *f = (float *)dst;
      for (int32_t i = 0; i < n; ++i) f[i] = v.empty() ? 0.0f : (float)v[i];
    }
  };
  if (cfg.refine) {
    put_vec(tmp.dev64.b, R.b, pcgk::F64);
    put_vec(tmp.dev64.x, R.x0, pcgk::F64);
  } else {
    put_vec(tmp.dev.b, R.b, cfg.vec_dtype);
    put_vec(tmp.dev.x, R.x0, cfg.vec_dtype);
  }
}

void release_images(PinnedArena *arena, Req &R) {
  if (R.img_pinned && arena) arena->release(R.img_a);
  std::vector<uint8_t>().swap(R.img_heap);
  R.img_a = R.img_g = nullptr;
  R.img_pinned = false;
}

void prep_request(const pcg_config &cfg, int cus, PinnedArena *arena, Req &R) {
  prep_parts(cfg, cus, R);
  if (R.prep_rc == PCG_OK) build_images(cfg, arena, R);
}

void prep_parts(const pcg_config &cfg, int cus, Req &R) {
  R.ap = APart{};
  prep_a(cfg, cus, R.n, R.a_rp.data(), R.a_ci.data(), R.a_val.data(), false, R.ap);
  if (!R.g_given && R.g_kind == PCG_G_FSAI && cfg.g_device && cfg.g_dtype != PCG_F16 &&
      prep_fsai_pattern(cfg, cus, R)) {
    R.bytes = R.ap.bytes + R.gp.bytes;
    R.prep_rc = PCG_OK;
    return;
  }
  std::vector<int32_t> grp, gci;
  std::vector<double> gv;
  if (R.g_given) {
    grp.swap(R.g_rp);
    gci.swap(R.g_ci);
    gv.swap(R.g_val);
  } else {
    // one thread: the workers already prepare several systems at once
    int rc = pcgh::build_g(R.g_kind, R.g_seed, R.n, R.a_rp.data(), R.a_ci.data(), R.a_val.data(), grp, gci, gv, 1);
    if (rc) {
      R.prep_rc = rc;
      return;
    }
  }
  R.gp = GPart{};
  prep_g(cfg, cus, R.n, grp, gci, gv, R.gp);
  R.bytes = R.ap.bytes + R.gp.bytes;
  R.prep_rc = PCG_OK;
}

void worker_main(pcg_ctx *ctx) {
  // below the scheduler thread: host preparation must not starve the thread
  // that keeps the GPU fed (lowering one's own priority needs no privilege)
  (void)setpriority(PRIO_PROCESS, (id_t)syscall(SYS_gettid), 10);
  for (;;) {
    std::shared_ptr<Req> R;
    {
      std::unique_lock<std::mutex> lk(ctx->mu);
      ctx->cv.wait(lk, [&] { return ctx->stop || !ctx->prep_q.empty(); });
      if (ctx->stop) return;
      R = ctx->prep_q.front();
      ctx->prep_q.pop_front();
      ++ctx->preparing;
    }
    const double t0 = now_ms();
    prep_request(ctx->cfg, ctx->cus, &ctx->staging, *R);
    const double t1 = now_ms();
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->stats.host_prep_ms += t1 - t0;
      R->st = RQ_READY;
      ctx->ready_q.push_back(R);
      --ctx->preparing;
    }
    ctx->cv.notify_all();
  }
}

int ensure_pool(pcg_ctx *ctx) {
  if (ctx->pool.ready()) return PCG_OK;
  size_t cap = ctx->cfg.mem_budget_mb > 0 ? (size_t)ctx->cfg.mem_budget_mb << 20 : 0;
  if (!cap) {
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    cap = fr / 2;
  }
  int rc = ctx->pool.init(cap);
  if (rc) ctx->err = "device pool allocation failed";
  return rc;
}

void start_workers(pcg_ctx *ctx) {
  if (!ctx->workers.empty()) return;
  // the CPUs this process may run on, less two (the scheduler and the
  // caller's thread), at most 32
  const unsigned ncpu = pcgh::available_cpus();
  const unsigned nt = std::max(1u, std::min(32u, ncpu > 2 ? ncpu - 2 : 1u));
  for (unsigned i = 0; i < nt; ++i) ctx->workers.emplace_back(worker_main, ctx);
}

// Bytes one iteration moves in the layouts in use: each matrix's values and
// column indices at their stored widths (3x3 blocks: one index per nine
// values; 16-bit column differences: two bytes), its row pointers, and the
// 11 vector streams.
double layout_bytes_per_iter(const SysDev &D, const pcg_config &cfg) {
  const double sa = (double)pcgk::dtype_size(cfg.a_dtype), sg = (double)pcgk::dtype_size(cfg.g_dtype),
               sv = (double)pcgk::dtype_size(cfg.vec_dtype);
  return stored_matrix_bytes(D.A, sa) + stored_matrix_bytes(D.G, sg) +
         stored_matrix_bytes(D.GT, sg) + 11.0 * D.n * sv;
}

void finish_request(pcg_ctx *ctx, Req &R, int status, const State &f, int restarts) {
  R.t_done = now_ms();
  R.res.status = status;
  R.res.iters = f.iter;
  R.res.outer_iters = 0;
  R.res.restarts = restarts;
  R.res.relres_true = f.bb > 0 ? std::sqrt(f.true_rr / f.bb) : 0.0;
  R.res.relres_rec = f.bb > 0 ? std::sqrt(f.rr / f.bb) : 0.0;
  R.res.t_solve_ms = R.t_done - R.t_admit;
  R.res.t_latency_ms = R.t_done - R.t_submit;
  R.res.t_queue_ms = R.t_admit - R.t_submit;
  R.st = RQ_DONE;
  ++ctx->completed;
}

int place_admitted(pcg_ctx *ctx, std::vector<std::shared_ptr<Req>> &cand, std::vector<void *> &temps);

// Admit ready requests (FIFO) while the pool has room; start their solves.
// On a device error none of this step's requests starts: each finishes with
// the error status and its storage returns to the pool.
int admit(pcg_ctx *ctx, std::vector<std::shared_ptr<Req>> &admitted) {
  std::vector<std::shared_ptr<Req>> cand;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    while (!ctx->ready_q.empty()) {
      auto R = ctx->ready_q.front();
      if (R->prep_rc != PCG_OK) {  // failed preparation completes at once
        ctx->ready_q.pop_front();
        State z{};
        R->t_admit = now_ms();
        finish_request(ctx, *R, R->prep_rc, z, 0);
        continue;
      }
      const size_t need_slots = ctx->cfg.refine ? 2 : 1;
      if (ctx->free_slots.size() < need_slots) break;
      void *bA = ctx->pool.alloc(R->ap.bytes);
      void *bG = bA ? ctx->pool.alloc(R->gp.bytes) : nullptr;
      if (!bA || !bG) {
        ctx->pool.release(bA);
        if (ctx->active.empty() && cand.empty() && ctx->pool.in_use() == 0) {
          ctx->ready_q.pop_front();  // larger than the whole pool: refuse
          release_images(&ctx->staging, *R);
          State z{};
          R->t_admit = now_ms();
          finish_request(ctx, *R, PCG_ENOMEM, z, 0);
          continue;
        }
        break;
      }
      ctx->ready_q.pop_front();
      R->sys.blkA = bA;
      R->sys.blkG = bG;
      R->sys.pooled = true;
      R->slot = ctx->free_slots.back();
      ctx->free_slots.pop_back();
      if (ctx->cfg.refine) {
        R->slot64 = ctx->free_slots.back();
        ctx->free_slots.pop_back();
      }
      cand.push_back(R);
    }
  }
  if (cand.empty()) return PCG_OK;
  std::vector<void *> temps;  // device FSAI scratch, freed once the stream has passed it
  const int rc = place_admitted(ctx, cand, temps);
  if (rc) (void)hipStreamSynchronize(ctx->stream);  // on success place_admitted has synchronized
  for (void *t : temps) ctx->da.put(t);
  for (auto &R : cand) release_images(&ctx->staging, *R);  // the stream has passed the copies
  if (rc) {  // none of them starts: give back their storage and finish their tickets with the error
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto &R : cand) {
      free_sys(ctx, R->sys);
      for (int *sl : {&R->slot, &R->slot64})
        if (*sl >= 0) {
          ctx->dir[*sl] = SysDev{};
          ctx->free_slots.push_back(*sl);
          *sl = -1;
        }
      State z{};
      R->t_admit = now_ms();
      finish_request(ctx, *R, rc, z, 0);
    }
    return rc;
  }
  const double t = now_ms();
  for (auto &R : cand) {
    R->t_admit = t;
    R->st = RQ_ACTIVE;
    R->ap = APart{};
    R->gp = GPart{};
    std::vector<int32_t>().swap(R->fs_dpos);
    std::vector<int32_t>().swap(R->fs_lrp);
    std::vector<int32_t>().swap(R->a_rp);
    std::vector<int32_t>().swap(R->a_ci);
    std::vector<double>().swap(R->a_val);
    std::vector<double>().swap(R->b);
    std::vector<double>().swap(R->x0);
    admitted.push_back(R);
  }
  return PCG_OK;
}

// Place the admitted requests' matrices and vectors in their pool blocks and
// start their solves; returns once the stream has passed every copy. Device
// FSAI scratch goes to `temps` (the caller frees it).
int place_admitted(pcg_ctx *ctx, std::vector<std::shared_ptr<Req>> &cand, std::vector<void *> &temps) {
  hipStream_t s = ctx->stream;
  std::vector<State> inits(2 * cand.size());
  std::vector<int> slots, wg_slots;
  auto fail_temps = [&](hipError_t e) {
    ctx->err = std::string("admission: ") + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      return PCG_ENOMEM;
    }
    return PCG_EDEVICE;
  };
  for (size_t i = 0; i < cand.size(); ++i) {
    Req &R = *cand[i];
    // the blocks' host images (matrices, b and x0, see build_images): the
    // pointers, then one copy per block
    HIPCHK(place_a(R.ap, R.sys.blkA, R.sys, Copier{Copier::Bind}));
    HIPCHK(place_g(R.gp, R.sys.blkG, R.sys, Copier{Copier::Bind}));
    HIPCHK(h2d(R.sys.blkA, R.img_a, R.ap.bytes, s));
    HIPCHK(h2d(R.sys.blkG, R.img_g, R.gp.bytes, s));
    if (R.dev_fsai) {  // G_L's rows on the device, written into both layouts
      const int32_t n = R.n;
      const int64_t nnz = (int64_t)R.a_ci.size(), nl = R.fs_lrp[n];
      const size_t tb = align_up(4 * (size_t)(n + 1)) + align_up(4 * (size_t)std::max<int64_t>(nnz, 1)) +
                        align_up(8 * (size_t)std::max<int64_t>(nnz, 1)) + align_up(4 * (size_t)n) +
                        align_up(4 * (size_t)(n + 1)) + align_up(8 * (size_t)std::max<int64_t>(nl, 1)) + align_up(8);
      void *tmp = nullptr;
      hipError_t e = ctx->da.get(&tmp, tb);
      if (e != hipSuccess) return fail_temps(e);
      temps.push_back(tmp);
      Carver c{(uint8_t *)tmp};
      int32_t *d_rp = (int32_t *)c.take(4 * (size_t)(n + 1));
      int32_t *d_ci = (int32_t *)c.take(4 * (size_t)std::max<int64_t>(nnz, 1));
      double *d_v = (double *)c.take(8 * (size_t)std::max<int64_t>(nnz, 1));
      int32_t *d_dpos = (int32_t *)c.take(4 * (size_t)n);
      int32_t *d_lrp = (int32_t *)c.take(4 * (size_t)(n + 1));
      double *d_lv = (double *)c.take(8 * (size_t)std::max<int64_t>(nl, 1));
      int32_t *d_err = (int32_t *)c.take(8);
      auto chain = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
      };
      chain(hipMemsetAsync((void *)R.sys.dev.G.val, 0, R.gp.G.val_bytes(), s));
      chain(hipMemsetAsync((void *)R.sys.dev.GT.val, 0, R.gp.GT.val_bytes(), s));
      chain(hipMemsetAsync(d_lv, 0, 8 * (size_t)std::max<int64_t>(nl, 1), s));
      chain(hipMemsetAsync(d_err, 0, 8, s));
      chain(h2d(d_rp, R.a_rp.data(), 4 * (size_t)(n + 1), s));
      chain(h2d(d_ci, R.a_ci.data(), 4 * (size_t)nnz, s));
      chain(h2d(d_v, R.a_val.data(), 8 * (size_t)nnz, s));
      chain(h2d(d_dpos, R.fs_dpos.data(), 4 * (size_t)n, s));
      chain(h2d(d_lrp, R.fs_lrp.data(), 4 * (size_t)(n + 1), s));
      const int grid = (int)std::min<int64_t>(n, (int64_t)ctx->cus * 16);
      chain(pcgk::launch_fsai_rows(d_rp, d_ci, d_v, d_dpos, d_lrp, n, R.fs_mmax, d_lv, d_err, grid, s));
      chain(pcgk::launch_fsai_place(d_rp, d_ci, d_dpos, d_lrp, d_lv, n, 1.0, R.sys.dev.GT, R.sys.dev.G, d_err, s));
      if (e != hipSuccess) return fail_temps(e);
      R.sys.g_scale = 1.0;
    }
    R.sys.dev.st = ctx->d_states + 2 * R.slot;
    ctx->dir[R.slot] = R.sys.dev;
    R.res.bytes_per_iter = layout_bytes_per_iter(R.sys.dev, ctx->cfg);
    inits[2 * i] = inits[2 * i + 1] = init_state(ctx, R.tol, R.maxit, R.sys.g_scale);
    R.iter_host = 0;
    if (ctx->cfg.refine) {
      // FP64 view: b64, x64 from the caller; s and t point at the inner x and b
      SysDev &V = R.sys.dev64;
      V.st = ctx->d_states + 2 * R.slot64;
      V.s = R.sys.dev.x;
      V.t = R.sys.dev.b;
      ctx->dir[R.slot64] = V;
      State o{};
      o.tol = R.tol;
      inits[2 * i] = inits[2 * i + 1] = o;
      slots.push_back(R.slot64);
      HIPCHK(h2d(ctx->d_dir + R.slot, &ctx->dir[R.slot], sizeof(SysDev), s));
      HIPCHK(h2d(ctx->d_dir + R.slot64, &ctx->dir[R.slot64], sizeof(SysDev), s));
      HIPCHK(h2d(ctx->d_states + 2 * R.slot64, &inits[2 * i], 2 * sizeof(State), s));
      continue;
    }
    R.wg = use_solve_wg(ctx, ctx->ty, R.n, true);
    if (R.wg) {
      inits[2 * i].confirm = inits[2 * i + 1].confirm = 1;
      wg_slots.push_back(R.slot);
    } else {
      slots.push_back(R.slot);
    }
    HIPCHK(h2d(ctx->d_dir + R.slot, &ctx->dir[R.slot], sizeof(SysDev), s));
    HIPCHK(h2d(ctx->d_states + 2 * R.slot, &inits[2 * i], 2 * sizeof(State), s));
  }
  HostSet &hs = ctx->set_tmp;
  int rc = build_set(ctx, hs, slots);
  if (rc) return rc;
  if (slots.empty()) {
    // only one-workgroup systems: they start in their own launch
  } else if (ctx->cfg.refine) {  // first FP64 residual of every new system
    const Types t64{pcgk::F64, pcgk::F64, pcgk::F64};
    HIPCHK(pcgk::launch_norm_b(t64, hs.L, s));
    HIPCHK(pcgk::launch_resid(t64, hs.L, 0, false, true, false, s));
  } else {
    rc = enqueue_start(ctx, ctx->ty, hs.L, ctx->cfg.eps != 0.0);
  }
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(s));  // copies done: host staging may go
  return PCG_OK;
}

void finish_refined(pcg_ctx *ctx, Req &R, int status);

// A stopped system waiting for its solution to reach the caller.
struct Retiring {
  std::shared_ptr<Req> R;
  int status;
  State f;       // its final state (single-level solves)
  bool refined;  // finish with the refinement totals
  int restarts;
};

// Copy the solutions of the stopped systems to their callers (host FP64):
// asynchronous copies into pinned staging, one wait for all of them, then
// on the host into the callers' arrays; free their storage and complete
// their tickets. Clears `list`.
int retire_all(pcg_ctx *ctx, std::vector<Retiring> &list) {
  if (list.empty()) return PCG_OK;
  hipStream_t s = ctx->stream;
  std::vector<void *> buf(list.size(), nullptr);
  std::vector<bool> pinned(list.size(), false);
  std::vector<std::vector<uint8_t>> heap(list.size());
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < list.size() && e == hipSuccess; ++i) {
    Req &R = *list[i].R;
    if (!R.x_out) continue;
    const bool f64 = R.slot64 >= 0 || ctx->ty.vec == pcgk::F64;
    const void *src = R.slot64 >= 0 ? R.sys.dev64.x : R.sys.dev.x;
    const size_t bytes = (f64 ? 8 : 4) * (size_t)R.n;
    buf[i] = ctx->staging.alloc(bytes);
    pinned[i] = buf[i] != nullptr;
    if (!buf[i]) {
      heap[i].resize(bytes);
      buf[i] = heap[i].data();
    }
    e = hipMemcpyAsync(buf[i], src, bytes, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  for (size_t i = 0; i < list.size(); ++i) {
    Req &R = *list[i].R;
    if (e == hipSuccess && R.x_out) {
      if (R.slot64 >= 0 || ctx->ty.vec == pcgk::F64) {
        std::memcpy(R.x_out, buf[i], 8 * (size_t)R.n);
      } else {
        const float *f = (const float *)buf[i];
        for (int32_t k = 0; k < R.n; ++k) R.x_out[k] = (double)f[k];
      }
    }
    if (pinned[i]) ctx->staging.release(buf[i]);
  }
  if (e != hipSuccess) {
    ctx->err = std::string("retire: ") + hipGetErrorString(e);
    list.clear();
    return PCG_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (auto &T : list) {
    Req &R = *T.R;
    free_sys(ctx, R.sys);
    ctx->dir[R.slot] = SysDev{};
    ctx->free_slots.push_back(R.slot);
    R.slot = -1;
    if (R.slot64 >= 0) {
      ctx->dir[R.slot64] = SysDev{};
      ctx->free_slots.push_back(R.slot64);
      R.slot64 = -1;
    }
    if (T.refined)
      finish_refined(ctx, R, T.status);
    else
      finish_request(ctx, R, T.status, T.f, T.restarts);
  }
  list.clear();
  return PCG_OK;
}

void finish_refined(pcg_ctx *ctx, Req &R, int status) {
  R.t_done = now_ms();
  R.res.status = status;
  R.res.iters = R.inner_total;
  R.res.outer_iters = R.outer;
  R.res.restarts = R.restarts;
  R.res.relres_true = R.relres64;
  R.res.relres_rec = R.last_rec;
  R.res.t_solve_ms = R.t_done - R.t_admit;
  R.res.t_latency_ms = R.t_done - R.t_submit;
  R.res.t_queue_ms = R.t_admit - R.t_submit;
  R.st = RQ_DONE;
  ++ctx->completed;
}

// Refinement decision after the FP64 residual of each system in `list` (its
// FP64 view's state already read back into h_states): finish, or start the
// next inner solve on r64 / ||r64||. Continuing systems go to `cont`.
int outer_decide(pcg_ctx *ctx, std::vector<std::shared_ptr<Req>> &list, std::vector<std::shared_ptr<Req>> &cont) {
  hipStream_t s = ctx->stream;
  const int max_outer = ctx->cfg.max_outer > 0 ? ctx->cfg.max_outer : 30;
  std::vector<int> slots, slots64;
  std::vector<std::shared_ptr<Req>> go;
  std::vector<double> itol;
  std::vector<Retiring> retiring;
  for (auto &R : list) {
    const State h = ctx->h_states[2 * R->slot64];
    int status = 1;  // continue
    double next_tol = 0.0;
    if (h.bb == 0.0) {
      HIPCHK(pcgk::launch_fill(pcgk::F64, R->sys.dev64.x, R->n, 0.0, s));
      R->relres64 = 0.0;
      status = PCG_OK;
    } else {
      const double rn = std::sqrt(h.true_rr), nb = std::sqrt(h.bb);
      R->relres64 = rn / nb;
      if (rn <= R->tol * nb)
        status = PCG_OK;
      else if (!std::isfinite(rn))
        status = PCG_EBREAKDOWN;
      else if (R->outer >= max_outer || rn > 0.9 * R->prev_rn)
        status = PCG_NOT_CONVERGED;
      else
        R->prev_rn = rn;
      next_tol = inner_tolerance(ctx->cfg.inner_tol, R->tol, nb, rn, R->outer);
    }
    if (status != 1) {
      retiring.push_back(Retiring{R, status, State{}, true, R->restarts});
      continue;
    }
    go.push_back(R);
    itol.push_back(next_tol);
    slots.push_back(R->slot);
    slots64.push_back(R->slot64);
  }
  int rc0 = retire_all(ctx, retiring);
  if (rc0) return rc0;
  if (go.empty()) return PCG_OK;
  HostSet &h64 = ctx->set_tmp64, &hin = ctx->set_tmp;
  int rc = build_set(ctx, h64, slots64);
  if (!rc) rc = build_set(ctx, hin, slots);
  if (rc) return rc;
  std::vector<State> inits(2 * go.size());
  HIPCHK(pcgk::launch_outer(ctx->ty.vec, h64.L, 1, s));  // inner b = r64 / ||r64||
  HIPCHK(pcgk::launch_zero_dirs(ctx->ty, hin.L, true, s));
  for (size_t i = 0; i < go.size(); ++i) {
    inits[2 * i] = inits[2 * i + 1] = init_state(ctx, itol[i], go[i]->maxit, go[i]->sys.g_scale, true);
    go[i]->iter_host = 0;
    HIPCHK(h2d(ctx->d_states + 2 * go[i]->slot, &inits[2 * i], 2 * sizeof(State), s));
  }
  rc = enqueue_start(ctx, ctx->ty, hin.L, ctx->cfg.eps != 0.0);
  HIPCHK(hipStreamSynchronize(s));
  if (rc) return rc;
  for (auto &R : go) cont.push_back(R);
  return PCG_OK;
}

void drop_step_graph(pcg_ctx *ctx) {
  if (ctx->step_graph) (void)hipGraphExecDestroy(ctx->step_graph);
  ctx->step_graph = nullptr;
  ctx->step_graph_iters = 0;
}

// Residency of the active set: when the matrices and iteration vectors of all
// active systems fit in 90% of the memory-side cache, their matrices are read
// with ordinary loads and stay cached from step to step; else they stream
// with nontemporal loads. Changed directory records are uploaded in stream
// order (the kernels read the flags from the directory at run time).
int batch_residency(pcg_ctx *ctx, hipStream_t s) {
  bool keep = false;
  if (ctx->cfg.cache_mb >= 0) {
    const double cap = (ctx->cfg.cache_mb > 0 ? ctx->cfg.cache_mb : 256) * 1048576.0;
    const double sv = (double)pcgk::dtype_size(ctx->ty.vec);
    double total = 0.0;
    for (auto &R : ctx->active) {
      const SysDev &D = ctx->dir[R->slot];
      total += placed_bytes(D.A) + placed_bytes(D.G) + placed_bytes(D.GT) + 8.0 * D.n * sv;
    }
    keep = total <= 0.9 * cap;
  }
  const int32_t t = keep ? 1 : 0;
  for (auto &R : ctx->active) {
    SysDev &D = ctx->dir[R->slot];
    if (D.A.temporal == t && D.G.temporal == t && D.GT.temporal == t) continue;
    D.A.temporal = D.G.temporal = D.GT.temporal = t;
    HIPCHK(h2d(ctx->d_dir + R->slot, &ctx->dir[R->slot], sizeof(SysDev), s));
  }
  return PCG_OK;
}

// Small admitted systems: one launch of the one-workgroup solver over all of
// them on the side stream (the uploads are complete: admission synchronised).
int launch_wg_group(pcg_ctx *ctx, std::vector<std::shared_ptr<Req>> &reqs) {
  if (!ctx->side) HIPCHK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
  pcg_ctx::WgGroup g;
  std::vector<int> slots;
  for (auto &R : reqs) slots.push_back(R->slot);
  int rc = build_set(ctx, g.set, slots);
  if (rc) return rc;
  g.reqs = reqs;
  HIPCHK(hipEventCreate(&g.start));
  HIPCHK(hipEventCreate(&g.done));
  HIPCHK(hipEventRecord(g.start, ctx->side));
  HIPCHK(pcgk::launch_solve_wg(ctx->ty, g.set.L, ctx->cfg.eps != 0.0, ctx->side));
  HIPCHK(hipEventRecord(g.done, ctx->side));
  ctx->wg_inflight += (int)reqs.size();
  ctx->wg_groups.push_back(std::move(g));
  return PCG_OK;
}

// Retire the systems of every finished one-workgroup launch.
int collect_wg_groups(pcg_ctx *ctx) {
  for (size_t k = 0; k < ctx->wg_groups.size();) {
    pcg_ctx::WgGroup &g = ctx->wg_groups[k];
    const hipError_t q = hipEventQuery(g.done);
    if (q == hipErrorNotReady) {
      ++k;
      continue;
    }
    HIPCHK(q);
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, g.start, g.done));
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->stats.wg_launches += 1;
      ctx->stats.wg_ms += ms;
    }
    std::vector<Retiring> retiring;
    for (auto &R : g.reqs) {
      State f;
      HIPCHK(hipMemcpy(&f, ctx->d_states + 2 * R->slot, sizeof(State), hipMemcpyDeviceToHost));
      {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->stats.wg_bytes += (double)f.iter * R->res.bytes_per_iter;
      }
      const int status = (f.status == pcgk::ST_CONV_REC || f.status == pcgk::ST_ZERO_B) ? PCG_OK
                         : f.status == pcgk::ST_MAXIT                                   ? PCG_NOT_CONVERGED
                                                                                        : PCG_EBREAKDOWN;
      retiring.push_back(Retiring{R, status, f, false, f.restarts});
    }
    int rc = retire_all(ctx, retiring);
    if (rc) return rc;
    ctx->wg_inflight -= (int)g.reqs.size();
    free_set(ctx, g.set);
    (void)hipEventDestroy(g.start);
    (void)hipEventDestroy(g.done);
    ctx->wg_groups.erase(ctx->wg_groups.begin() + (long)k);
  }
  return PCG_OK;
}

// One scheduler step: admit, `iters` iterations over the active set, retire.
// Adds the wall time since construction to one host-time counter of the
// batch statistics.
struct PhaseTimer {
  pcg_ctx *ctx;
  double pcg_batch_stats::*field;
  double t0;
  PhaseTimer(pcg_ctx *c, double pcg_batch_stats::*f) : ctx(c), field(f), t0(now_ms()) {}
  ~PhaseTimer() {
    const double t = now_ms() - t0;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stats.*field += t;
  }
};

int progress(pcg_ctx *ctx, int iters) {
  int rc;
  if ((rc = ensure_pool(ctx))) return rc;
  std::vector<std::shared_ptr<Req>> admitted;
  {
    PhaseTimer pt(ctx, &pcg_batch_stats::host_admit_ms);
    if ((rc = admit(ctx, admitted))) return rc;
    if (!admitted.empty() && ctx->cfg.refine) {  // the first refinement step of the new systems
      int mx = 0;
      for (auto &R : admitted) mx = std::max(mx, R->slot64);
      HIPCHK(hipMemcpy(ctx->h_states, ctx->d_states, 2 * sizeof(State) * (size_t)(mx + 1), hipMemcpyDeviceToHost));
      std::vector<std::shared_ptr<Req>> cont;
      if ((rc = outer_decide(ctx, admitted, cont))) return rc;
      admitted.swap(cont);
    }
  }
  if (!admitted.empty()) {
    std::vector<std::shared_ptr<Req>> wg;
    for (auto &R : admitted) {
      if (R->wg) {
        wg.push_back(R);
      } else {
        ctx->active.push_back(R);
        ctx->active_dirty = true;
      }
    }
    if (!wg.empty() && (rc = launch_wg_group(ctx, wg))) return rc;
  }
  if ((rc = collect_wg_groups(ctx))) return rc;
  if (ctx->active.empty()) return PCG_OK;
  std::optional<PhaseTimer> phase;
  phase.emplace(ctx, &pcg_batch_stats::host_step_ms);
  hipStream_t s = ctx->stream;
  const bool changed = ctx->active_dirty;
  if (ctx->active_dirty) {
    drop_step_graph(ctx);
    if ((rc = batch_residency(ctx, s))) return rc;
    std::vector<int> slots;
    for (auto &R : ctx->active) slots.push_back(R->slot);
    if ((rc = build_set(ctx, ctx->set_active, slots))) return rc;
    ctx->active_dirty = false;
  }
  const LaunchSet &L = ctx->set_active.L;
  const bool has_eps = ctx->cfg.eps != 0.0;
  // The residual kernel decides per system whether it is at a replacement
  // iteration; it is only launched when some running system may be (inner
  // solves of refinement never replace).
  const int rr = ctx->cfg.rr_period;
  auto any_replacement = [&](int k) {
    if (rr <= 0) return false;
    for (auto &R : ctx->active) {
      if (R->slot64 >= 0) continue;
      const int i = R->iter_host + k;
      if (i > 0 && i % rr == 0) return true;
    }
    return false;
  };
  if (!ctx->step_ev[0]) {
    HIPCHK(hipEventCreate(&ctx->step_ev[0]));
    HIPCHK(hipEventCreate(&ctx->step_ev[1]));
  }
  HIPCHK(hipEventRecord(ctx->step_ev[0], s));
  if (ctx->cfg.graph_iters > 0 && !changed) {
    // one graph per active set, captured once the set has stayed the same
    // for a step (a set that changes every step is cheaper to launch plainly
    // than to capture): the residual kernel runs every iteration and decides
    // per system, when some system replaces at all
    bool replaces = false;
    for (auto &R : ctx->active) replaces = replaces || (rr > 0 && R->slot64 < 0);
    if (!ctx->step_graph || ctx->step_graph_iters != iters) {
      drop_step_graph(ctx);
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipSuccess;
      auto chain = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
      };
      for (int k = 0; k < iters; ++k) {
        chain(pcgk::launch_iter_A(ctx->ty, L, s));
        if (replaces) chain(pcgk::launch_resid(ctx->ty, L, 2, true, false, true, s));
        chain(pcgk::launch_iter_GT(ctx->ty, L, 3, s));
        chain(pcgk::launch_iter_G(ctx->ty, L, has_eps, 3, s));
      }
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(s, &g);
      HIPCHK(e);
      HIPCHK(e2);
      const hipError_t e3 = hipGraphInstantiate(&ctx->step_graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCHK(e3);
      ctx->step_graph_iters = iters;
    }
    HIPCHK(hipGraphLaunch(ctx->step_graph, s));
  } else {
    for (int k = 0; k < iters; ++k) {
      HIPCHK(pcgk::launch_iter_A(ctx->ty, L, s));
      if (any_replacement(k)) HIPCHK(pcgk::launch_resid(ctx->ty, L, 2, true, false, true, s));
      HIPCHK(pcgk::launch_iter_GT(ctx->ty, L, 3, s));
      HIPCHK(pcgk::launch_iter_G(ctx->ty, L, has_eps, 3, s));
    }
  }
  HIPCHK(hipEventRecord(ctx->step_ev[1], s));
  int maxslot = 0;
  for (auto &R : ctx->active) maxslot = std::max(maxslot, R->slot);
  const size_t sb = 2 * sizeof(State) * (size_t)(maxslot + 1);
  HIPCHK(hipMemcpyAsync(ctx->h_states, ctx->d_states, sb, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->step_ev[0], ctx->step_ev[1]));
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stats.steps += 1;
    ctx->stats.step_ms += ms;
    for (auto &R : ctx->active) {  // iterations each system ran in this step (an inner solve restarts at 0)
      const int it0 = R->iter_host, it1 = ctx->h_states[2 * R->slot].iter;
      ctx->stats.step_bytes += (double)(it1 >= it0 ? it1 - it0 : it1) * R->res.bytes_per_iter;
    }
  }
  for (auto &R : ctx->active) R->iter_host = ctx->h_states[2 * R->slot].iter;
  std::vector<int> done_slots;
  for (auto &R : ctx->active)
    if (ctx->h_states[2 * R->slot].done) done_slots.push_back(R->slot);
  if (done_slots.empty()) return PCG_OK;
  phase.reset();
  phase.emplace(ctx, &pcg_batch_stats::host_retire_ms);
  // finish the stopped systems: any pending x update, true residual
  HostSet &hs = ctx->set_done;
  if ((rc = build_set(ctx, hs, done_slots))) return rc;
  HIPCHK(pcgk::launch_finalize(ctx->ty, hs.L, s));
  HIPCHK(pcgk::launch_resid(ctx->ty, hs.L, 0, false, true, false, s));
  HIPCHK(hipMemcpyAsync(ctx->h_states, ctx->d_states, sb, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<int> restart_slots;
  std::vector<std::shared_ptr<Req>> keep, outer_list;
  std::vector<Retiring> retiring;
  for (auto &R : ctx->active) {
    const State f = ctx->h_states[2 * R->slot];
    if (!f.done) {
      keep.push_back(R);
      continue;
    }
    int status;
    if (f.status == pcgk::ST_CONV_REC && R->slot64 < 0 && !(std::sqrt(f.true_rr) <= f.tol_nb)) {
      R->restarts++;
      restart_slots.push_back(R->slot);
      keep.push_back(R);
      continue;
    }
    if (R->slot64 >= 0) {  // an inner solve ended: refinement step next
      R->inner_total += f.iter;
      R->last_rec = f.bb > 0 ? std::sqrt(f.rr / f.bb) : 0.0;
      if (f.status == pcgk::ST_BREAK_GAMMA || f.status == pcgk::ST_BREAK_DELTA) {
        retiring.push_back(Retiring{R, PCG_EBREAKDOWN, f, true, R->restarts});
        continue;
      }
      outer_list.push_back(R);
      continue;
    }
    if (f.status == pcgk::ST_CONV_REC) {
      status = PCG_OK;
    } else if (f.status == pcgk::ST_ZERO_B) {
      HIPCHK(pcgk::launch_fill(ctx->ty.vec, R->sys.dev.x, R->n, 0.0, s));  // before its copy, in stream order
      status = PCG_OK;
    } else if (f.status == pcgk::ST_MAXIT) {
      status = PCG_NOT_CONVERGED;
    } else {
      status = PCG_EBREAKDOWN;
    }
    retiring.push_back(Retiring{R, status, f, false, R->restarts});
  }
  if ((rc = retire_all(ctx, retiring))) return rc;
  if (!restart_slots.empty()) {
    if ((rc = build_set(ctx, hs, restart_slots))) return rc;
    HIPCHK(pcgk::launch_state_restart(hs.L, s));
    HIPCHK(pcgk::launch_iter_GT(ctx->ty, hs.L, 2, s));
    HIPCHK(pcgk::launch_iter_G(ctx->ty, hs.L, has_eps, 2, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  if (!outer_list.empty()) {  // x64 += ||r|| c, then the FP64 residual
    const Types t64{pcgk::F64, pcgk::F64, pcgk::F64};
    std::vector<int> s64;
    int mx = 0;
    for (auto &R : outer_list) {
      s64.push_back(R->slot64);
      mx = std::max(mx, R->slot64);
    }
    if ((rc = build_set(ctx, hs, s64))) return rc;
    HIPCHK(pcgk::launch_outer(ctx->ty.vec, hs.L, 0, s));
    HIPCHK(pcgk::launch_resid(t64, hs.L, 0, false, true, false, s));
    HIPCHK(hipMemcpyAsync(ctx->h_states, ctx->d_states, 2 * sizeof(State) * (size_t)(mx + 1), hipMemcpyDeviceToHost,
                          s));
    HIPCHK(hipStreamSynchronize(s));
    for (auto &R : outer_list) R->outer++;
    std::vector<std::shared_ptr<Req>> cont;
    if ((rc = outer_decide(ctx, outer_list, cont))) return rc;
    for (auto &R : cont) keep.push_back(R);
  }
  if (keep.size() != ctx->active.size()) {
    ctx->active.swap(keep);
    ctx->active_dirty = true;
  }
  return PCG_OK;
}

int copy_request(const pcg_system &S, std::shared_ptr<Req> &out, std::string &err) {
  if (S.n <= 0 || !S.a_rowptr || !S.a_col || !S.a_val || !S.b || !(S.tol >= 0.0) || S.maxit < 0) {
    err = "pcg_submit_batch: bad system (n, arrays, tol or maxit)";
    return PCG_EINVAL;
  }
  if (S.a_rowptr[S.n] != S.nnz_a) {
    err = "pcg_submit_batch: a_rowptr[n] != nnz_a";
    return PCG_EINVAL;
  }
  int rc = pcgh::validate_csr(S.n, S.nnz_a, S.a_rowptr, S.a_col, 1, &err);
  if (rc) return rc;
  auto R = std::make_shared<Req>();
  R->n = S.n;
  R->a_rp.assign(S.a_rowptr, S.a_rowptr + S.n + 1);
  R->a_ci.assign(S.a_col, S.a_col + S.nnz_a);
  R->a_val.assign(S.a_val, S.a_val + S.nnz_a);
  R->b.assign(S.b, S.b + S.n);
  if (S.x) R->x0.assign(S.x, S.x + S.n);
  R->x_out = S.x;
  R->tol = S.tol;
  R->maxit = S.maxit;
  if (S.g_rowptr) {
    if (!S.g_col || !S.g_val || S.g_rowptr[S.n] != S.nnz_g) {
      err = "pcg_submit_batch: bad preconditioner arrays (g_col, g_val, or g_rowptr[n] != nnz_g)";
      return PCG_EINVAL;
    }
    rc = pcgh::validate_csr(S.n, S.nnz_g, S.g_rowptr, S.g_col, 0, &err);
    if (rc) return rc;
    R->g_given = true;
    R->g_rp.assign(S.g_rowptr, S.g_rowptr + S.n + 1);
    R->g_ci.assign(S.g_col, S.g_col + S.nnz_g);
    R->g_val.assign(S.g_val, S.g_val + S.nnz_g);
  } else {
    if (pcgh::g_nnz(S.g_kind, S.n, S.a_rowptr, S.a_col) < 0) {
      err = "pcg_submit_batch: unknown preconditioner kind";
      return PCG_EINVAL;
    }
    R->g_kind = S.g_kind;
    R->g_seed = S.g_seed;
  }
  out = R;
  return PCG_OK;
}

}  // namespace

// ================================================================ C ABI

extern "C" {

void pcg_config_default(pcg_config *cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->device = 0;
  cfg->stream = nullptr;
  cfg->vec_dtype = PCG_F64;
  cfg->a_dtype = PCG_F64;
  cfg->g_dtype = PCG_F64;
  cfg->rr_period = 50;
  cfg->eps = 0.0;
  cfg->refine = 0;
  cfg->inner_tol = 1e-6;
  cfg->max_outer = 30;
  cfg->graph_iters = 10;
  cfg->grid_mult = kGridMult;
  cfg->wg_max_n = kWgMaxN;
  cfg->wg_max_n_batch = kWgMaxNBatch;
  cfg->rows_per_lane = 2;
  cfg->loads_in_flight = 8;
}

int pcg_create(const pcg_config *cfg, pcg_ctx **out) {
  if (!out) return PCG_EINVAL;
  *out = nullptr;
  if (!cfg) return PCG_EINVAL;
  const int v = cfg->vec_dtype, a = cfg->a_dtype, g = cfg->g_dtype;
  const bool g_ok = g == PCG_F64 || g == PCG_F32 || g == PCG_BF16 || g == PCG_F16;
  const bool ok = (v == PCG_F64 && a == PCG_F64 && g_ok && !cfg->refine) ||
                  (v == PCG_F32 && a == PCG_F32 && g_ok && g != PCG_F64);
  const int rpl = cfg->rows_per_lane, uw = cfg->loads_in_flight;
  if (!ok || cfg->rr_period < 0 || cfg->graph_iters < 0 || !(cfg->eps >= 0.0) || cfg->mem_budget_mb < 0 ||
      (cfg->alloc == nullptr) != (cfg->free == nullptr) || rpl < 0 || rpl > 2 || (uw != 0 && uw != 4 && uw != 8))
    return PCG_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= cfg->device || cfg->device < 0) {
    (void)hipGetLastError();
    return PCG_EDEVICE;
  }
  pcg_ctx *ctx = new pcg_ctx();
  ctx->cfg = *cfg;
  ctx->ty = Types{v, a, g};
  auto fail = [&](int rc) {
    pcg_destroy(ctx);
    return rc;
  };
  if (hipSetDevice(cfg->device) != hipSuccess) return fail(PCG_EDEVICE);
  // the device address of the file-scope scratch (looked up once per device)
  if (pcgk::static_scratch(cfg->device, &ctx->static_scratch) != hipSuccess) {
    (void)hipGetLastError();
    ctx->static_scratch = nullptr;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, cfg->device) == hipSuccess && prop.multiProcessorCount > 0) {
    ctx->cus = prop.multiProcessorCount;
    ctx->lds_per_block = (int)prop.sharedMemPerBlock;
  }
  if (cfg->stream) {
    ctx->stream = (hipStream_t)cfg->stream;
    ctx->own_stream = false;
  } else if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
    return fail(PCG_EDEVICE);
  }
  ctx->da.alloc = cfg->alloc;
  ctx->da.release = cfg->free;
  ctx->da.user = cfg->alloc_user;
  ctx->da.stream = ctx->stream;
  ctx->pool.da = ctx->da;
  if (hipHostMalloc((void **)&ctx->h_states, sizeof(State) * 2 * kDirCap, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&ctx->h_init, sizeof(State) * 2, hipHostMallocDefault) != hipSuccess)
    return fail(PCG_EDEVICE);
  for (auto &e : ctx->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(PCG_EDEVICE);
  if (hipEventCreate(&ctx->t0) != hipSuccess || hipEventCreate(&ctx->t1) != hipSuccess) return fail(PCG_EDEVICE);
  if (ctx->da.get((void **)&ctx->d_dir, sizeof(SysDev) * kDirCap) != hipSuccess ||
      ctx->da.get((void **)&ctx->d_states, sizeof(State) * 2 * kDirCap) != hipSuccess)
    return fail(PCG_ENOMEM);
  if (hipMemset(ctx->d_dir, 0, sizeof(SysDev) * kDirCap) != hipSuccess ||
      hipMemset(ctx->d_states, 0, sizeof(State) * 2 * kDirCap) != hipSuccess)
    return fail(PCG_EDEVICE);
  ctx->dir.assign(kDirCap, SysDev{});
  for (int sl = kDirCap - 1; sl >= kFirstBatchSlot; --sl) ctx->free_slots.push_back(sl);
  *out = ctx;
  return PCG_OK;
}

void pcg_destroy(pcg_ctx *ctx) {
  if (!ctx) return;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stop = true;
  }
  ctx->cv.notify_all();
  for (auto &t : ctx->workers) t.join();
  ctx->workers.clear();
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->side) (void)hipStreamSynchronize(ctx->side);
  drop_graphs(ctx);
  drop_step_graph(ctx);
  for (auto &R : ctx->active) free_sys(ctx, R->sys);
  ctx->active.clear();
  for (auto &g : ctx->wg_groups) {
    for (auto &R : g.reqs) free_sys(ctx, R->sys);
    free_set(ctx, g.set);
    if (g.done) (void)hipEventDestroy(g.done);
  }
  ctx->wg_groups.clear();
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  free_set(ctx, ctx->set_main);
  free_set(ctx, ctx->set_64);
  free_set(ctx, ctx->set_x);
  free_set(ctx, ctx->set_active);
  free_set(ctx, ctx->set_done);
  free_set(ctx, ctx->set_tmp);
  free_set(ctx, ctx->set_tmp64);
  free_sys(ctx, ctx->single);
  ctx->pool.reset();
  for (auto &e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : ctx->step_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->t0) (void)hipEventDestroy(ctx->t0);
  if (ctx->t1) (void)hipEventDestroy(ctx->t1);
  if (ctx->h_states) (void)hipHostFree(ctx->h_states);
  if (ctx->h_init) (void)hipHostFree(ctx->h_init);
  ctx->da.put(ctx->d_dir);
  ctx->da.put(ctx->loss_buf);
  ctx->da.put(ctx->d_states);
  if (ctx->stream && ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

// Lay out and upload A (host copy in the context) for the single system.
static int place_single_a(pcg_ctx *ctx) {
  const int32_t n = (int32_t)ctx->a_rp.size() - 1;
  APart P;
  prep_a(eff_cfg(ctx, false), ctx->cus, n, ctx->a_rp.data(), ctx->a_ci.data(), ctx->a_val.data(), true, P);
  void *blk = nullptr;
  if (ctx->da.get(&blk, P.bytes) != hipSuccess) {
    (void)hipGetLastError();
    ctx->err = "pcg_set_matrix: device allocation failed";
    return PCG_ENOMEM;
  }
  ctx->single.blkA = blk;
  HIPCHK(place_a(P, blk, ctx->single, Copier{Copier::Device, ctx->stream}));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->have_a = true;
  return PCG_OK;
}

int pcg_set_matrix(pcg_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                   const double *val, int on_device) {
  if (!ctx) return PCG_EINVAL;
  if (n <= 0 || !rowptr || !col || !val) {
    ctx->err = "pcg_set_matrix: n must be positive and arrays non-null";
    return PCG_EINVAL;
  }
  HIPCHK(hipSetDevice(ctx->cfg.device));
  std::vector<int32_t> hrp(n + 1), hci;
  std::vector<double> hv;
  if (on_device) {
    HIPCHK(hipMemcpy(hrp.data(), rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
    if (hrp[n] != nnz || nnz < 0) {
      ctx->err = "pcg_set_matrix: rowptr[n] != nnz";
      return PCG_EINVAL;
    }
    hci.resize(nnz);
    hv.resize(nnz);
    if (nnz) {
      HIPCHK(hipMemcpy(hci.data(), col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(hv.data(), val, sizeof(double) * nnz, hipMemcpyDeviceToHost));
    }
  } else {
    hrp.assign(rowptr, rowptr + n + 1);
    if (hrp[n] != nnz) {
      ctx->err = "pcg_set_matrix: rowptr[n] != nnz";
      return PCG_EINVAL;
    }
    hci.assign(col, col + nnz);
    hv.assign(val, val + nnz);
  }
  int rc = pcgh::validate_csr(n, nnz, hrp.data(), hci.data(), 1, &ctx->err);
  if (rc) return rc;
  drop_graphs(ctx);
  free_set(ctx, ctx->set_main);
  free_set(ctx, ctx->set_64);
  free_set(ctx, ctx->set_x);
  free_sys(ctx, ctx->single);
  ctx->have_a = ctx->have_g = false;
  ctx->tune.on = false;  // a new matrix: automatic layouts until tuned again
  ctx->a_rp.swap(hrp);
  ctx->a_ci.swap(hci);
  ctx->a_val.swap(hv);
  {
    double sum = 0.0;
    int64_t cnt = 0;
    for (double x : ctx->a_val)
      if (x != 0.0) {
        sum += std::fabs(x);
        ++cnt;
      }
    ctx->a_mean_abs = cnt ? sum / (double)cnt : 1.0;
  }
  return place_single_a(ctx);
}

static int set_g_from_host(pcg_ctx *ctx, std::vector<int32_t> &grp, std::vector<int32_t> &gci,
                           std::vector<double> &gv) {
  drop_graphs(ctx);
  if (ctx->single.blkG) {
    ctx->da.put(ctx->single.blkG);
    ctx->single.blkG = nullptr;
  }
  ctx->have_g = false;
  ctx->g_rp = grp;
  ctx->g_ci = gci;
  ctx->g_val = gv;
  ctx->g_from_device = false;
  GPart P;
  prep_g(eff_cfg(ctx, true), ctx->cus, ctx->single.n, grp, gci, gv, P);
  void *blk = nullptr;
  if (ctx->da.get(&blk, P.bytes) != hipSuccess) {
    (void)hipGetLastError();
    ctx->err = "pcg_set_precond: device allocation failed";
    return PCG_ENOMEM;
  }
  ctx->single.blkG = blk;
  HIPCHK(place_g(P, blk, ctx->single, Copier{Copier::Device, ctx->stream}));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  int rc = single_sets(ctx);
  if (rc) return rc;
  ctx->have_g = true;
  return PCG_OK;
}

int pcg_set_precond(pcg_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                    const double *val, int on_device) {
  if (!ctx) return PCG_EINVAL;
  if (!ctx->have_a) {
    ctx->err = "pcg_set_precond: set the matrix first";
    return PCG_ESTATE;
  }
  if (n != ctx->single.n) {
    ctx->err = "pcg_set_precond: size differs from A";
    return PCG_ESTATE;
  }
  if (!rowptr || !col || !val) return PCG_EINVAL;
  HIPCHK(hipSetDevice(ctx->cfg.device));
  std::vector<int32_t> hrp(n + 1), hci;
  std::vector<double> hv;
  if (on_device) {
    HIPCHK(hipMemcpy(hrp.data(), rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
    if (hrp[n] != nnz || nnz < 0) return PCG_EINVAL;
    hci.resize(nnz);
    hv.resize(nnz);
    if (nnz) {
      HIPCHK(hipMemcpy(hci.data(), col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(hv.data(), val, sizeof(double) * nnz, hipMemcpyDeviceToHost));
    }
  } else {
    hrp.assign(rowptr, rowptr + n + 1);
    if (hrp[n] != nnz) {
      ctx->err = "pcg_set_precond: rowptr[n] != nnz";
      return PCG_EINVAL;
    }
    hci.assign(col, col + nnz);
    hv.assign(val, val + nnz);
  }
  int rc = pcgh::validate_csr(n, nnz, hrp.data(), hci.data(), 0, &ctx->err);
  if (rc) return rc;
  rc = set_g_from_host(ctx, hrp, hci, hv);
  if (!rc && ctx->cfg.autotune) rc = pcg_autotune(ctx, 20, nullptr);
  return rc;
}

// FSAI factored on the device: the host lays out the patterns of G = triu(A)
// and G^T = tril(A) (O(nnz) integer work), the device computes G_L's values
// row by row and writes them, cast, into both layouts. Returns 1 (nothing
// changed) when the host builder must be used instead.
static int build_fsai_device(pcg_ctx *ctx) {
  Sys &S = ctx->single;
  const int32_t n = S.n;
  const int32_t *rp = ctx->a_rp.data(), *ci = ctx->a_ci.data();
  const double *v = ctx->a_val.data();
  std::vector<int32_t> dpos(n), lrp(n + 1, 0), lci, grp(n + 1, 0), gci;
  int32_t mmax = 0;
  for (int32_t i = 0; i < n; ++i) {
    int32_t d = -1;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] == i) d = k;
    if (d < 0) {
      ctx->err = "pcg_build_precond: FSAI needs a stored diagonal in every row";
      return PCG_EINVAL;
    }
    dpos[i] = d;
    mmax = std::max(mmax, d - rp[i] + 1);
    lrp[i + 1] = lrp[i] + (d - rp[i] + 1);
    grp[i + 1] = grp[i] + (rp[i + 1] - d);
  }
  if (mmax > pcgk::kFsaiMaxRow || lrp[n] != grp[n]) return 1;  // long rows or unsymmetric counts
  lci.resize(lrp[n]);
  gci.resize(grp[n]);
  for (int32_t i = 0; i < n; ++i) {
    std::copy(ci + rp[i], ci + dpos[i] + 1, lci.begin() + lrp[i]);
    std::copy(ci + dpos[i], ci + rp[i + 1], gci.begin() + grp[i]);
  }
  drop_graphs(ctx);
  if (S.blkG) {
    ctx->da.put(S.blkG);
    S.blkG = nullptr;
  }
  ctx->have_g = false;
  GPart P;
  P.n = n;
  P.nnz = lrp[n];
  P.gdt = ctx->cfg.g_dtype;
  P.vdt = ctx->cfg.vec_dtype;
  const pcg_config gcfg = eff_cfg(ctx, true);
  make_pattern(gcfg, ctx->cus, n, grp.data(), gci.data(), P.gdt, P.vdt, P.G);
  make_pattern(gcfg, ctx->cus, n, lrp.data(), lci.data(), P.gdt, P.vdt, P.GT);
  P.bytes = P.G.bytes() + P.GT.bytes() + align_up(16 * pcgk::kAccWords * (size_t)P.GT.grid);
  // temporaries: A (CSR, FP64), dpos, lrp, G_L's values, flags, partial maxima
  const int64_t nnz = rp[n], nl = lrp[n];
  const size_t tb = align_up(4 * (size_t)(n + 1)) + align_up(4 * (size_t)std::max<int64_t>(nnz, 1)) +
                    align_up(8 * (size_t)std::max<int64_t>(nnz, 1)) + align_up(4 * (size_t)n) +
                    align_up(4 * (size_t)(n + 1)) + align_up(8 * (size_t)std::max<int64_t>(nl, 1)) + align_up(8) +
                    align_up(8 * (size_t)pcgk::kAbsmaxGrid);
  void *blk = nullptr, *tmp = nullptr;
  if (ctx->da.get(&blk, P.bytes) != hipSuccess || ctx->da.get(&tmp, tb) != hipSuccess) {
    (void)hipGetLastError();
    ctx->da.put(blk);
    ctx->err = "pcg_build_precond: device allocation failed";
    return PCG_ENOMEM;
  }
  S.blkG = blk;
  hipStream_t s = ctx->stream;
  Carver c{(uint8_t *)tmp};
  int32_t *d_rp = (int32_t *)c.take(4 * (size_t)(n + 1));
  int32_t *d_ci = (int32_t *)c.take(4 * (size_t)std::max<int64_t>(nnz, 1));
  double *d_v = (double *)c.take(8 * (size_t)std::max<int64_t>(nnz, 1));
  int32_t *d_dpos = (int32_t *)c.take(4 * (size_t)n);
  int32_t *d_lrp = (int32_t *)c.take(4 * (size_t)(n + 1));
  double *d_lv = (double *)c.take(8 * (size_t)std::max<int64_t>(nl, 1));
  int32_t *d_err = (int32_t *)c.take(8);
  double *d_part = (double *)c.take(8 * (size_t)pcgk::kAbsmaxGrid);
  int rc = PCG_OK;
  int32_t herr[2] = {0, 0};
  auto run = [&]() -> hipError_t {
    hipError_t e = hipSuccess;
    auto chain = [&](hipError_t x) {
      if (e == hipSuccess) e = x;
    };
    chain(place_g(P, blk, S, Copier{Copier::Device, s}));  // patterns (no values yet)
    // the sliced layout's padding must hold zeros (outside any graph capture)
    chain(hipMemsetAsync((void *)S.dev.G.val, 0, P.G.val_bytes(), s));
    chain(hipMemsetAsync((void *)S.dev.GT.val, 0, P.GT.val_bytes(), s));
    chain(h2d(d_rp, rp, 4 * (size_t)(n + 1), s));
    chain(h2d(d_ci, ci, 4 * (size_t)nnz, s));
    chain(h2d(d_v, v, 8 * (size_t)nnz, s));
    chain(h2d(d_dpos, dpos.data(), 4 * (size_t)n, s));
    chain(h2d(d_lrp, lrp.data(), 4 * (size_t)(n + 1), s));
    chain(h2d(d_err, herr, 8, s));
    const int grid = (int)std::min<int64_t>(n, (int64_t)ctx->cus * 16);
    chain(pcgk::launch_fsai_rows(d_rp, d_ci, d_v, d_dpos, d_lrp, n, mmax, d_lv, d_err, grid, s));
    double scale = 1.0;
    if (P.gdt == pcgk::F16) {  // same power-of-two scale as the host path
      std::vector<double> part(pcgk::kAbsmaxGrid);
      chain(pcgk::launch_absmax(d_lv, nl, d_part, s));
      chain(hipMemcpyAsync(part.data(), d_part, 8 * part.size(), hipMemcpyDeviceToHost, s));
      chain(hipStreamSynchronize(s));
      double mx = 0.0;
      for (double x : part) mx = std::max(mx, x);
      if (mx > 0) {
        int ex;
        std::frexp(mx, &ex);
        scale = std::ldexp(1.0, 14 - ex);
      }
    }
    chain(pcgk::launch_fsai_place(d_rp, d_ci, d_dpos, d_lrp, d_lv, n, scale, S.dev.GT, S.dev.G, d_err, s));
    chain(hipMemcpyAsync(herr, d_err, 8, hipMemcpyDeviceToHost, s));
    chain(hipStreamSynchronize(s));
    S.g_scale = scale;
    return e;
  };
  const hipError_t e = run();
  ctx->da.put(tmp);
  if (e != hipSuccess) {
    ctx->err = std::string("pcg_build_precond: ") + hipGetErrorString(e);
    return PCG_EDEVICE;
  }
  if (herr[0] == 2) return 1;  // pattern not symmetric: the host builder handles it
  if (herr[0] == 1) {
    ctx->err = "pcg_build_precond: FSAI pivot not positive (A not SPD)";
    return PCG_EBREAKDOWN;
  }
  if ((rc = single_sets(ctx))) return rc;
  std::vector<int32_t>().swap(ctx->g_rp);
  std::vector<int32_t>().swap(ctx->g_ci);
  std::vector<double>().swap(ctx->g_val);
  ctx->g_from_device = true;
  ctx->have_g = true;
  return PCG_OK;
}

int pcg_build_precond(pcg_ctx *ctx, int kind, uint64_t seed) {
  if (!ctx) return PCG_EINVAL;
  if (!ctx->have_a) {
    ctx->err = "pcg_build_precond: set the matrix first";
    return PCG_ESTATE;
  }
  int rc = 1;
  if (kind == PCG_G_FSAI && ctx->cfg.g_device) {
    HIPCHK(hipSetDevice(ctx->cfg.device));
    rc = build_fsai_device(ctx);  // 1: use the host builder
  }
  if (rc == 1) {
    std::vector<int32_t> grp, gci;
    std::vector<double> gv;
    rc = pcgh::build_g(kind, seed, ctx->single.n, ctx->a_rp.data(), ctx->a_ci.data(), ctx->a_val.data(), grp, gci,
                       gv);
    if (rc) {
      ctx->err = "pcg_build_precond: construction failed (kind or matrix not SPD)";
      return rc;
    }
    rc = set_g_from_host(ctx, grp, gci, gv);
  }
  if (!rc && ctx->cfg.autotune) rc = pcg_autotune(ctx, 20, nullptr);
  return rc;
}

// ------------------------------------------------------------------ autotuner

// Choices per matrix signature, shared by the contexts of the process and,
// when the environment names a file in PCG_TUNE_CACHE, kept there as lines
// "signature layout_a layout_g grid_mult load_policy".
static std::mutex g_tune_mu;
static std::map<std::string, pcg_ctx::Tune> g_tune_cache;
static bool g_tune_loaded = false;

static void tune_cache_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *path = std::getenv("PCG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  char line[768], key[512];
  while (std::fgets(line, sizeof line, f)) {
    int la, lg, gm, res, rows, uw;
    if (std::sscanf(line, "%511s %d %d %d %d %d %d", key, &la, &lg, &gm, &res, &rows, &uw) != 7) continue;
    pcg_ctx::Tune t;
    t.on = true;
    t.la = la;
    t.lg = lg;
    t.gm = gm;
    t.res = res;
    t.gt_rows = rows == 1 ? 1 : 2;
    t.a_uw = uw == 4 ? 4 : 8;
    g_tune_cache[key] = t;
  }
  std::fclose(f);
}

static void tune_cache_store(const std::string &key, const pcg_ctx::Tune &t) {
  g_tune_cache[key] = t;
  const char *path = std::getenv("PCG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d %d %d\n", key.c_str(), t.la, t.lg, t.gm, t.res, t.gt_rows, t.a_uw);
  std::fclose(f);
}

// What the layouts depend on: sizes, row-length structure, 3x3 blocking,
// storage types, the compute-unit count and the layout options.
static std::string tune_key(const pcg_ctx *ctx) {
  const int32_t n = (int32_t)ctx->a_rp.size() - 1;
  const int32_t *rp = ctx->a_rp.data();
  int32_t maxrow = 0;
  for (int32_t i = 0; i < n; ++i) maxrow = std::max(maxrow, rp[i + 1] - rp[i]);
  int64_t nb = 0;
  const bool b3 = pcgh::is_block3(n, rp, ctx->a_ci.data(), &nb);
  const pcg_config &c = ctx->cfg;
  char buf[384];
  std::snprintf(buf, sizeof buf, "n%d_a%lld_g%lld_r%d_s%lld_b%d_t%d.%d.%d_f%d.%d.%d.%d.%d_cu%d", n,
                (long long)rp[n], (long long)ctx->single.nnz_g, maxrow, (long long)pcgh::sell_entries(n, rp),
                (int)b3, c.vec_dtype, c.a_dtype, c.g_dtype, c.refine, c.layout, c.wide_index, c.grid_mult,
                c.cache_mb, ctx->cus);
  return buf;
}

// Lay A and G out again under ctx->tune (same values): G from the kept host
// copy, or factored on the device again.
static int relayout(pcg_ctx *ctx) {
  std::vector<int32_t> grp = ctx->g_rp, gci = ctx->g_ci;
  std::vector<double> gv = ctx->g_val;
  const bool dev_g = ctx->g_from_device;
  drop_graphs(ctx);
  free_set(ctx, ctx->set_main);
  free_set(ctx, ctx->set_64);
  free_set(ctx, ctx->set_x);
  free_sys(ctx, ctx->single);
  ctx->have_a = ctx->have_g = false;
  int rc = place_single_a(ctx);
  if (rc) return rc;
  if (dev_g) {
    rc = build_fsai_device(ctx);
    if (rc == 1) {  // cannot happen for a G the device built before; rebuild on the host
      rc = pcgh::build_g(PCG_G_FSAI, 0, ctx->single.n, ctx->a_rp.data(), ctx->a_ci.data(), ctx->a_val.data(), grp,
                         gci, gv);
      if (!rc) rc = set_g_from_host(ctx, grp, gci, gv);
    }
    return rc;
  }
  return set_g_from_host(ctx, grp, gci, gv);
}

// One CG iteration's time (three kernels) on the stored right-hand side b = 1:
// the smaller of two timings of `iters` iterations after as many for warm-up.
static int time_iteration(pcg_ctx *ctx, int iters, double *ms) {
  HIPCHK(pcgk::launch_fill(ctx->ty.vec, ctx->single.dev.b, ctx->single.n, 1.0, ctx->stream));
  double m[4];
  int rc = pcg_time_kernels(ctx, iters, m, nullptr);
  double best = INFINITY;
  for (int k = 0; k < 2 && !rc; ++k) {
    rc = pcg_time_kernels(ctx, iters, m, nullptr);
    best = std::min(best, m[3]);
  }
  if (!rc) *ms = best;
  return rc;
}

static int apply_tune(pcg_ctx *ctx, const pcg_ctx::Tune &t) {
  const bool same = ctx->tune.on == t.on && (!t.on || (ctx->tune.la == t.la && ctx->tune.lg == t.lg &&
                                                       ctx->tune.gm == t.gm));
  const bool same_rest = same && (!t.on || (ctx->tune.res == t.res && ctx->tune.gt_rows == t.gt_rows &&
                                             ctx->tune.a_uw == t.a_uw));
  ctx->tune = t;
  if (!same) return relayout(ctx);
  // load policy or kernel knobs only: new directory entries and launch sets
  return same_rest ? PCG_OK : single_sets(ctx);
}

int pcg_autotune(pcg_ctx *ctx, int iters, pcg_tune_result *res) {
  if (!ctx) return PCG_EINVAL;
  if (res) std::memset(res, 0, sizeof(*res));
  if (iters <= 0) iters = 20;
  if (iters > 1000) return PCG_EINVAL;
  if (!ctx->have_a || !ctx->have_g) {
    ctx->err = "pcg_autotune: matrix and preconditioner must be set";
    return PCG_ESTATE;
  }
  HIPCHK(hipSetDevice(ctx->cfg.device));
  const std::string key = tune_key(ctx);
  pcg_ctx::Tune best;
  bool cached = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      best = it->second;
      cached = true;
    }
  }
  int rc;
  double t_best = 0.0, t_auto = 0.0;
  int ncand = 0;
  if (cached) {
    if ((rc = apply_tune(ctx, best))) return rc;
    if ((rc = time_iteration(ctx, iters, &t_best))) return rc;
    t_auto = NAN;
  } else {
    // the automatic choice first (the default to beat)
    pcg_ctx::Tune a;
    a.gt_rows = cfg_rows_per_lane(ctx->cfg);
    a.a_uw = cfg_loads_in_flight(ctx->cfg);
    if ((rc = apply_tune(ctx, a))) return rc;
    if ((rc = time_iteration(ctx, iters, &t_auto))) return rc;
    ++ncand;
    const int32_t n = ctx->single.n;
    const int32_t *rp = ctx->a_rp.data(), *ci = ctx->a_ci.data();
    const int gm0 = ctx->cfg.grid_mult > 0 ? ctx->cfg.grid_mult : kGridMult;
    // layouts of A (distinct by the format they give) and of G
    std::vector<int> las, lgs;
    if (ctx->cfg.layout == PCG_LAYOUT_AUTO) {
      std::vector<int> fa;
      for (int l : {PCG_LAYOUT_CSR, PCG_LAYOUT_SELL, PCG_LAYOUT_SDIA, PCG_LAYOUT_BSR3}) {
        const int f = use_bsr3(l, n, rp, ci)   ? pcgk::FMT_BSR3
                      : use_sdia(l, n, rp, ci) ? pcgk::FMT_SDIA
                      : use_sell(l, n, rp)     ? pcgk::FMT_SELL
                                               : pcgk::FMT_CSR;
        if (std::find(fa.begin(), fa.end(), f) == fa.end()) {
          fa.push_back(f);
          las.push_back(l);
        }
      }
      lgs.push_back(PCG_LAYOUT_CSR);
      if (ctx->g_from_device || ctx->g_rp.empty() || use_sell(PCG_LAYOUT_SELL, n, ctx->g_rp.data()))
        lgs.push_back(PCG_LAYOUT_SELL);
      if (ctx->g_from_device || ctx->g_rp.empty() || use_sdia(PCG_LAYOUT_SDIA, n, ctx->g_rp.data(), ctx->g_ci.data()))
        lgs.push_back(PCG_LAYOUT_SDIA);
      if (!ctx->g_from_device && n % 3 == 0) lgs.push_back(PCG_LAYOUT_BSR3);  // the 3x3-block cover of G
    } else {
      las.push_back(ctx->cfg.layout);
      lgs.push_back(ctx->cfg.layout);
    }
    best = a;
    best.gm = gm0;
    t_best = t_auto;
    auto consider = [&](const pcg_ctx::Tune &t) -> int {
      int r = apply_tune(ctx, t);
      if (r) return r;
      double ms = 0.0;
      if ((r = time_iteration(ctx, iters, &ms))) return r;
      ++ncand;
      if (ms < 0.97 * t_best) {  // a change must gain 3% (timing noise)
        best = t;
        t_best = ms;
      }
      return PCG_OK;
    };
    for (int la : las)
      for (int lg : lgs) {
        pcg_ctx::Tune t = a;  // the configured kernel knobs
        t.on = true;
        t.la = la;
        t.lg = lg;
        t.gm = gm0;
        if ((rc = consider(t))) return rc;
      }
    pcg_ctx::Tune base = best;
    if (!base.on) {  // grids around the automatic layouts: pin them as the formats they gave
      base.on = true;
      base.la = ctx->cfg.layout;
      base.lg = ctx->cfg.layout;
    }
    for (int gm : {gm0 / 2, gm0 * 2}) {
      if (gm < 1) continue;
      pcg_ctx::Tune t = base;
      t.gm = gm;
      if ((rc = consider(t))) return rc;
    }
    // load policy for the best layouts and grid: every subset of {A, G, G^T}
    // read with ordinary loads (the residency plan's choice was timed above)
    base = best;
    if (!base.on) {
      base.on = true;
      base.la = ctx->cfg.layout;
      base.lg = ctx->cfg.layout;
      base.gm = gm0;
    }
    const int planned = residency_plan(ctx);
    for (int r = 0; r < 8; ++r) {
      if (r == planned) continue;
      pcg_ctx::Tune t = base;
      t.res = r;
      if ((rc = consider(t))) return rc;
    }
    // kernel knobs for the best of the above: rows per lane of the G^T-kernel
    // (vector width of its accesses over sliced diagonals), then loads in
    // flight per lane in the A-kernel
    base = best;
    if (!base.on) {
      base.on = true;
      base.la = ctx->cfg.layout;
      base.lg = ctx->cfg.layout;
      base.gm = gm0;
    }
    {
      pcg_ctx::Tune t = base;
      t.gt_rows = base.gt_rows == 2 ? 1 : 2;
      if ((rc = consider(t))) return rc;
    }
    base = best.on ? best : base;
    {
      pcg_ctx::Tune t = base;
      t.a_uw = base.a_uw == 8 ? 4 : 8;
      if ((rc = consider(t))) return rc;
    }
    if ((rc = apply_tune(ctx, best))) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_store(key, best);
  }
  if (res) {
    res->layout_a = best.on ? best.la : ctx->cfg.layout;
    res->layout_g = best.on ? best.lg : ctx->cfg.layout;
    res->grid_mult = best.on ? best.gm : (ctx->cfg.grid_mult > 0 ? ctx->cfg.grid_mult : kGridMult);
    res->candidates = ncand;
    res->ms_per_iter = t_best;
    res->ms_per_iter_auto = t_auto;
    res->fmt_a = ctx->single.dev.A.fmt;
    res->fmt_g = ctx->single.dev.G.fmt;
    res->fmt_gt = ctx->single.dev.GT.fmt;
    res->idx16 = (ctx->single.dev.A.idx16 ? 1 : 0) | (ctx->single.dev.G.idx16 ? 2 : 0) |
                 (ctx->single.dev.GT.idx16 ? 4 : 0);
    res->temporal = ctx->single.dev.A.temporal | (ctx->single.dev.G.temporal << 1) |
                    (ctx->single.dev.GT.temporal << 2);
    res->rows_per_lane_gt = ctx->single.dev.GT.rpl;
    res->loads_in_flight_a = ctx->set_main.L.uw_a;
  }
  return PCG_OK;
}

int pcg_solve(pcg_ctx *ctx, const double *b, double *x, double tol, int maxit, int on_device, pcg_result *res) {
  if (!ctx) return PCG_EINVAL;
  if (res) std::memset(res, 0, sizeof(*res));
  if (!b || !x || !(tol >= 0.0) || maxit < 0) {
    ctx->err = "pcg_solve: null vector, negative tol or maxit";
    return PCG_EINVAL;
  }
  if (!ctx->have_a || !ctx->have_g) {
    ctx->err = "pcg_solve: matrix and preconditioner must be set";
    return PCG_ESTATE;
  }
  Sys &S = ctx->single;
  const int32_t n = S.n;
  int rc;
  HIPCHK(hipSetDevice(ctx->cfg.device));
  if (on_device) HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipEventRecord(ctx->t0, ctx->stream));
  const double bpi = layout_bytes_per_iter(S.dev, ctx->cfg);
  if (ctx->cfg.refine) {
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(hipMemcpyAsync(S.dev64.b, b, sizeof(double) * n, kind, ctx->stream));
    HIPCHK(hipMemcpyAsync(S.dev64.x, x, sizeof(double) * n, kind, ctx->stream));
    pcg_result r{};
    rc = refine_solve(ctx, tol, maxit, &r);
    if (rc < PCG_EBREAKDOWN) return rc;  // device or memory error
    HIPCHK(hipEventRecord(ctx->t1, ctx->stream));
    HIPCHK(hipMemcpyAsync(x, S.dev64.x, sizeof(double) * n, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ctx->t0, ctx->t1));
    r.t_solve_ms = ms;
    r.bytes_per_iter = bpi;
    if (res) *res = r;
    if (r.status == PCG_EBREAKDOWN) ctx->err = "breakdown: A or M not SPD, or non-finite values";
    return r.status;
  }
  if ((rc = load_vec(ctx, b, on_device, S.dev.b, ctx->ty.vec, n))) return rc;
  if ((rc = load_vec(ctx, x, on_device, S.dev.x, ctx->ty.vec, n))) return rc;
  CoreOut co;
  if ((rc = solve_core(ctx, main_core(ctx), tol, maxit, co))) return rc;
  HIPCHK(hipEventRecord(ctx->t1, ctx->stream));
  if ((rc = store_vec(ctx, S.dev.x, ctx->ty.vec, x, on_device, n))) return rc;
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, ctx->t0, ctx->t1));
  if (res) {
    res->status = co.status;
    res->iters = co.iters;
    res->outer_iters = 0;
    res->restarts = co.restarts;
    res->relres_true = co.bb > 0 ? std::sqrt(co.true_rr / co.bb) : 0.0;
    res->relres_rec = co.bb > 0 ? std::sqrt(co.rr / co.bb) : 0.0;
    res->t_solve_ms = ms;
    res->bytes_per_iter = bpi;
  }
  if (co.status == PCG_EBREAKDOWN) ctx->err = "breakdown: A or M not SPD, or non-finite values";
  return co.status;
}

int pcg_matvec(pcg_ctx *ctx, int op, const double *x, double *y, int on_device) {
  if (!ctx) return PCG_EINVAL;
  if (!x || !y || op < PCG_OP_A || op > PCG_OP_MINV) return PCG_EINVAL;
  if (!ctx->have_a || (op != PCG_OP_A && !ctx->have_g)) {
    ctx->err = "pcg_matvec: operator not set";
    return PCG_ESTATE;
  }
  Sys &S = ctx->single;
  const int32_t n = S.n;
  const int vdt = ctx->ty.vec;
  int rc;
  HIPCHK(hipSetDevice(ctx->cfg.device));
  if (on_device) HIPCHK(hipDeviceSynchronize());
  if ((rc = load_vec(ctx, x, on_device, S.tmp_in, vdt, n))) return rc;
  hipStream_t s = ctx->stream;
  const double inv_scale2 = 1.0 / (S.g_scale * S.g_scale);
  switch (op) {
    case PCG_OP_A: HIPCHK(pcgk::launch_spmv(ctx->ty, S.dev.A, S.tmp_in, S.tmp_out, s)); break;
    case PCG_OP_GT:
      HIPCHK(pcgk::launch_spmv(ctx->ty, S.dev.GT, S.tmp_in, S.tmp_out, s));
      if (S.g_scale != 1.0) HIPCHK(pcgk::launch_axpby(vdt, n, 1.0 / S.g_scale, S.tmp_out, 0.0, S.tmp_in, s));
      break;
    case PCG_OP_G:
      HIPCHK(pcgk::launch_spmv(ctx->ty, S.dev.G, S.tmp_in, S.tmp_out, s));
      if (S.g_scale != 1.0) HIPCHK(pcgk::launch_axpby(vdt, n, 1.0 / S.g_scale, S.tmp_out, 0.0, S.tmp_in, s));
      break;
    default:
      HIPCHK(pcgk::launch_spmv(ctx->ty, S.dev.GT, S.tmp_in, S.dev.t, s));
      HIPCHK(pcgk::launch_spmv(ctx->ty, S.dev.G, S.dev.t, S.tmp_out, s));
      HIPCHK(pcgk::launch_axpby(vdt, n, inv_scale2, S.tmp_out, ctx->cfg.eps, S.tmp_in, s));
      break;
  }
  return store_vec(ctx, S.tmp_out, vdt, y, on_device, n);
}

int pcg_sai_loss(pcg_ctx *ctx, int32_t k, const double *W, int on_device, double *sai, double *l2, double *cs) {
  if (!ctx) return PCG_EINVAL;
  if (k < 1 || !W) {
    ctx->err = "pcg_sai_loss: need k >= 1 probes and W";
    return PCG_EINVAL;
  }
  if (!ctx->have_a || !ctx->have_g) {
    ctx->err = "pcg_sai_loss: matrix and preconditioner must be set";
    return PCG_ESTATE;
  }
  HIPCHK(hipSetDevice(ctx->cfg.device));
  Sys &S = ctx->single;
  const int32_t n = S.n;
  const double na = ctx->a_mean_abs;  // ||A|| = mean |A_ij| over the nonzeros
  const size_t nk = (size_t)n * (size_t)k;
  const size_t pb = sizeof(double) * (size_t)pcgk::kLossGrid * 5 * (size_t)k;
  const size_t need = 3 * align_up(8 * nk) + align_up(pb);
  if (need > ctx->loss_bytes) {
    ctx->da.put(ctx->loss_buf);
    ctx->loss_buf = nullptr;
    ctx->loss_bytes = 0;
    if (ctx->da.get(&ctx->loss_buf, need) != hipSuccess) {
      (void)hipGetLastError();
      ctx->loss_buf = nullptr;
      ctx->err = "pcg_sai_loss: device allocation failed";
      return PCG_ENOMEM;
    }
    ctx->loss_bytes = need;
  }
  Carver c{(uint8_t *)ctx->loss_buf};
  double *Wd = (double *)c.take(8 * nk), *T = (double *)c.take(8 * nk), *U = (double *)c.take(8 * nk);
  double *part = (double *)c.take(pb);
  std::vector<double> hp((size_t)pcgk::kLossGrid * 5 * (size_t)k);
  hipStream_t s = ctx->stream;
  hipError_t e = hipSuccess;
  auto chain = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  if (on_device) chain(hipDeviceSynchronize());
  chain(hipMemcpyAsync(Wd, W, 8 * nk, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  const double eps = ctx->cfg.eps;
  chain(pcgk::launch_spmm(S.dev.GT, k, Wd, 1.0, nullptr, 0.0, T, s));  // T = G^T W
  chain(pcgk::launch_spmm(S.dev.G, k, T, 1.0 / (S.g_scale * S.g_scale), eps != 0.0 ? Wd : nullptr, eps, U, s));
  chain(pcgk::launch_spmm(S.dev.A, k, U, 1.0, nullptr, 0.0, T, s));  // Y = A M^-1 W
  chain(pcgk::launch_loss_partials(n, k, Wd, T, na, part, s));
  chain(hipMemcpyAsync(hp.data(), part, pb, hipMemcpyDeviceToHost, s));
  chain(hipStreamSynchronize(s));
  if (e != hipSuccess) {
    ctx->err = std::string("pcg_sai_loss: ") + hipGetErrorString(e);
    return PCG_EDEVICE;
  }
  for (int32_t p = 0; p < k; ++p) {
    double q[5] = {0, 0, 0, 0, 0};
    for (int b = 0; b < pcgk::kLossGrid; ++b)
      for (int j = 0; j < 5; ++j) q[j] += hp[((size_t)b * 5 + j) * k + p];
    if (sai) sai[p] = q[0];
    if (l2) l2[p] = q[1];
    if (cs) cs[p] = q[2] / (std::sqrt(q[4]) * std::sqrt(q[3]));
  }
  return PCG_OK;
}

int pcg_sai_loss_noalloc(pcg_ctx *ctx, int32_t k, const double *W, double *sai, double *l2, double *cs) {
  if (!ctx) return PCG_EINVAL;
  if (k < 1 || !W) {
    ctx->err = "pcg_sai_loss_noalloc: need k >= 1 probes and W";
    return PCG_EINVAL;
  }
  if (!ctx->have_a || !ctx->have_g) {
    ctx->err = "pcg_sai_loss_noalloc: matrix and preconditioner must be set";
    return PCG_ESTATE;
  }
  if (!ctx->static_scratch) {
    ctx->err = "pcg_sai_loss_noalloc: the device address of the static scratch is unknown";
    return PCG_EDEVICE;
  }
  Sys &S = ctx->single;
  const int32_t n = S.n;
  const size_t nk = (size_t)n * (size_t)k;
  const size_t pb = sizeof(double) * (size_t)pcgk::kLossGrid * 5 * (size_t)k;
  const size_t need = 2 * align_up(8 * nk) + align_up(pb) + align_up(8 * 3 * (size_t)k);
  if (need > pcgk::kStaticScratchBytes) {
    char m[200];
    std::snprintf(m, sizeof m,
                  "pcg_sai_loss_noalloc: n = %d with k = %d probes needs %zu bytes of scratch, above the %zu of "
                  "the static scratch",
                  n, k, need, pcgk::kStaticScratchBytes);
    ctx->err = m;
    return PCG_EINVAL;
  }
  HIPCHK(hipSetDevice(ctx->cfg.device));
  Carver c{(uint8_t *)ctx->static_scratch};
  double *T = (double *)c.take(8 * nk), *U = (double *)c.take(8 * nk);
  double *part = (double *)c.take(pb), *out = (double *)c.take(8 * 3 * (size_t)k);
  hipStream_t s = ctx->stream;
  hipError_t e = hipSuccess;
  auto chain = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  chain(hipDeviceSynchronize());  // W may come from work queued on another stream
  const double eps = ctx->cfg.eps;
  chain(pcgk::launch_spmm(S.dev.GT, k, W, 1.0, nullptr, 0.0, T, s));  // T = G^T W
  chain(pcgk::launch_spmm(S.dev.G, k, T, 1.0 / (S.g_scale * S.g_scale), eps != 0.0 ? W : nullptr, eps, U, s));
  chain(pcgk::launch_spmm(S.dev.A, k, U, 1.0, nullptr, 0.0, T, s));  // Y = A M^-1 W
  chain(pcgk::launch_loss_partials(n, k, W, T, ctx->a_mean_abs, part, s));
  chain(pcgk::launch_loss_final(k, part, out, s));
  double *dst[3] = {sai, l2, cs};
  for (int j = 0; j < 3; ++j)
    if (dst[j]) chain(hipMemcpyAsync(dst[j], out + (size_t)j * k, 8 * (size_t)k, hipMemcpyDeviceToHost, s));
  chain(hipStreamSynchronize(s));
  if (e != hipSuccess) {
    ctx->err = std::string("pcg_sai_loss_noalloc: ") + hipGetErrorString(e);
    return PCG_EDEVICE;
  }
  return PCG_OK;
}

int pcg_time_kernels(pcg_ctx *ctx, int iters, double *ms, double *bytes) {
  if (!ctx) return PCG_EINVAL;
  if (!ms || iters < 1 || iters > 100000) return PCG_EINVAL;
  if (!ctx->have_a || !ctx->have_g) {
    ctx->err = "pcg_time_kernels: matrix and preconditioner must be set";
    return PCG_ESTATE;
  }
  Sys &S = ctx->single;
  const int32_t n = S.n;
  const Types ty = ctx->ty;
  const LaunchSet &L = ctx->set_main.L;
  hipStream_t s = ctx->stream;
  HIPCHK(hipSetDevice(ctx->cfg.device));
  // a fresh solve of the stored right-hand side from x0 = 0 that never stops
  State init = init_state(ctx, -1.0, INT32_MAX, S.g_scale);
  init.rr_period = 0;
  const bool has_eps = init.eps != 0.0;
  ctx->h_init[0] = init;
  ctx->h_init[1] = init;
  HIPCHK(hipMemcpyAsync(S.dev.st, ctx->h_init, 2 * sizeof(State), hipMemcpyHostToDevice, s));
  HIPCHK(pcgk::launch_fill(ty.vec, S.dev.x, n, 0.0, s));
  {
    int rc0 = enqueue_start(ctx, ty, L, has_eps);
    if (rc0) return rc0;
  }
  HIPCHK(hipStreamSynchronize(s));
  State h;
  HIPCHK(hipMemcpy(&h, S.dev.st, sizeof(State), hipMemcpyDeviceToHost));
  if (h.done) {
    ctx->err = "pcg_time_kernels: solve a nonzero right-hand side first";
    return PCG_ESTATE;
  }
  // events attached to each dispatch: the kernels' own execution intervals
  std::vector<hipEvent_t> ev(6 * (size_t)iters, nullptr);
  int rc = PCG_OK;
  for (auto &e : ev)
    if (hipEventCreate(&e) != hipSuccess) rc = PCG_EDEVICE;
  double acc[4] = {0, 0, 0, 0};
  if (rc == PCG_OK) {
    hipError_t e = hipSuccess;
    auto chain = [&](hipError_t x) {
      if (e == hipSuccess) e = x;
    };
    for (int it = 0; it < iters; ++it) {
      hipEvent_t *E = &ev[6 * (size_t)it];
      chain(pcgk::launch_iter_A(ty, L, s, E[0], E[1]));
      chain(pcgk::launch_iter_GT(ty, L, 0, s, E[2], E[3]));
      chain(pcgk::launch_iter_G(ty, L, has_eps, 0, s, E[4], E[5]));
    }
    chain(hipStreamSynchronize(s));
    for (int it = 0; it < iters && e == hipSuccess; ++it) {
      const hipEvent_t *E = &ev[6 * (size_t)it];
      float t;
      for (int k = 0; k < 3; ++k) {
        chain(hipEventElapsedTime(&t, E[2 * k], E[2 * k + 1]));
        acc[k] += t;
      }
      chain(hipEventElapsedTime(&t, E[0], E[5]));
      acc[3] += t;
    }
    if (e != hipSuccess) {
      ctx->err = std::string("pcg_time_kernels: ") + hipGetErrorString(e);
      rc = PCG_EDEVICE;
    }
  }
  for (auto &e : ev)
    if (e) (void)hipEventDestroy(e);
  if (rc) return rc;
  HIPCHK(hipMemcpy(&h, S.dev.st, sizeof(State), hipMemcpyDeviceToHost));
  if (h.done) {
    ctx->err = "pcg_time_kernels: the iteration stopped (breakdown) while timing";
    return PCG_EBREAKDOWN;
  }
  for (int k = 0; k < 4; ++k) ms[k] = acc[k] / iters;
  if (bytes) {
    const double sa = (double)pcgk::dtype_size(ctx->cfg.a_dtype), sg = (double)pcgk::dtype_size(ctx->cfg.g_dtype),
                 sv = (double)pcgk::dtype_size(ctx->cfg.vec_dtype);
    bytes[0] = stored_matrix_bytes(S.dev.A, sa) + 2.0 * n * sv;
    bytes[1] = stored_matrix_bytes(S.dev.GT, sg) + 4.0 * n * sv;
    bytes[2] = stored_matrix_bytes(S.dev.G, sg) + (has_eps ? 6.0 : 5.0) * n * sv;
    bytes[3] = bytes[0] + bytes[1] + bytes[2];
  }
  return PCG_OK;
}

// Copy (kind 0: read and write `bytes`) or read-only (kind 1) stream over
// freshly allocated buffers, `reps` timed launches after two warm-up ones.
static int stream_bandwidth(int device, int kind, int64_t bytes, int reps, double *gbps, double *ms_per_launch) {
  if (bytes < 16 || reps < 1 || !gbps) return PCG_EINVAL;
  bytes &= ~int64_t(15);
  if (hipSetDevice(device) != hipSuccess) return PCG_EDEVICE;
  void *src = nullptr, *dst = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = PCG_OK;
  hipDeviceProp_t prop;
  int cus = 256;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0) cus = prop.multiProcessorCount;
  const int grid = cus * 8;  // one full-occupancy round of 256-thread workgroups
  const size_t dbytes = kind == 0 ? (size_t)bytes : sizeof(uint32_t) * (size_t)grid;
  if (hipMalloc(&src, bytes) != hipSuccess || hipMalloc(&dst, dbytes) != hipSuccess) rc = PCG_ENOMEM;
  if (!rc && (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
              hipEventCreate(&e1) != hipSuccess))
    rc = PCG_EDEVICE;
  if (!rc && hipMemsetAsync(src, 0, bytes, s) != hipSuccess) rc = PCG_EDEVICE;
  float ms = 0.0f;
  if (!rc) {
    auto launch = [&]() {
      return kind == 0 ? pcgk::launch_copy(src, dst, bytes, grid, s)
                       : pcgk::launch_read(src, bytes, (uint32_t *)dst, grid, s);
    };
    hipError_t e = hipSuccess;
    for (int w = 0; w < 2 && e == hipSuccess; ++w) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) rc = PCG_EDEVICE;
  }
  if (!rc) {
    *gbps = (kind == 0 ? 2.0 : 1.0) * (double)bytes * reps / (ms * 1e-3) / 1e9;
    if (ms_per_launch) *ms_per_launch = ms / reps;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (src) (void)hipFree(src);
  if (dst) (void)hipFree(dst);
  (void)hipGetLastError();
  return rc;
}

int pcg_copy_bandwidth(int device, int64_t bytes, int reps, double *gbps, double *ms_per_copy) {
  return stream_bandwidth(device, 0, bytes, reps, gbps, ms_per_copy);
}

int pcg_read_bandwidth(int device, int64_t bytes, int reps, double *gbps, double *ms_per_read) {
  return stream_bandwidth(device, 1, bytes, reps, gbps, ms_per_read);
}

// ------------------------------------------------------------ batching / serving

int pcg_submit_batch(pcg_ctx *ctx, int count, const pcg_system *sys, uint64_t *tickets) {
  if (!ctx) return PCG_EINVAL;
  if (count < 0 || (count > 0 && (!sys || !tickets))) return PCG_EINVAL;
  // validate and copy the systems, on several threads for a large batch
  std::vector<std::shared_ptr<Req>> reqs(count);
  std::vector<int> rcs(count, PCG_OK);
  std::vector<std::string> errs(count);
  const unsigned nt = count < 8 ? 1u : std::min(16u, std::min(pcgh::available_cpus(), (unsigned)count));
  if (nt <= 1) {
    for (int i = 0; i < count; ++i) rcs[i] = copy_request(sys[i], reqs[i], errs[i]);
  } else {
    std::atomic<int> next{0};
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nt; ++w)
      th.emplace_back([&] {
        for (int i; (i = next.fetch_add(1)) < count;) rcs[i] = copy_request(sys[i], reqs[i], errs[i]);
      });
    for (auto &t : th) t.join();
  }
  for (int i = 0; i < count; ++i)
    if (rcs[i]) {  // nothing queued on error
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->err = errs[i];
      return rcs[i];
    }
  if (count > 0) {  // pinned staging for the device images (once; without it images use the heap)
    (void)hipSetDevice(ctx->cfg.device);
    (void)ctx->staging.init(kStagingBytes);
  }
  const double t = now_ms();
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (int i = 0; i < count; ++i) {
      reqs[i]->ticket = ctx->next_ticket++;
      reqs[i]->t_submit = t;
      tickets[i] = reqs[i]->ticket;
      ctx->by_ticket[reqs[i]->ticket] = reqs[i];
      ctx->prep_q.push_back(reqs[i]);
    }
    start_workers(ctx);
  }
  ctx->cv.notify_all();
  return PCG_OK;
}

int pcg_progress(pcg_ctx *ctx, int iters, int *active, int *queued) {
  if (!ctx) return PCG_EINVAL;
  if (iters < 0) return PCG_EINVAL;
  HIPCHK(hipSetDevice(ctx->cfg.device));
  int rc;
  {
    PhaseTimer pt(ctx, &pcg_batch_stats::host_progress_ms);
    rc = progress(ctx, iters);
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (active) *active = (int)ctx->active.size() + ctx->wg_inflight;
  if (queued) *queued = (int)(ctx->prep_q.size() + ctx->ready_q.size()) + ctx->preparing;
  return rc;
}

int pcg_poll(pcg_ctx *ctx, uint64_t ticket, pcg_result *res) {
  if (!ctx) return PCG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->by_ticket.find(ticket);
  if (it == ctx->by_ticket.end()) return PCG_EINVAL;
  if (it->second->st != RQ_DONE) return PCG_PENDING;
  if (res) *res = it->second->res;
  const int st = it->second->res.status;
  ctx->by_ticket.erase(it);
  return st;
}

// Drives the scheduler until every ticket is done (or the time limit).
static int wait_tickets(pcg_ctx *ctx, int count, const uint64_t *tickets, pcg_result *results, double timeout_s,
                        int iters_per_step) {
  const int step = iters_per_step > 0 ? iters_per_step : 20;
  const double t_end = now_ms() + (timeout_s < 0 ? 1e300 : timeout_s * 1e3);
  uint64_t seen = UINT64_MAX;  // completions counted at the last look at the tickets
  for (;;) {
    bool all = true;
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      // the tickets are looked at again only after some ticket has finished
      if (ctx->completed == seen) all = false;
      seen = ctx->completed;
      for (int i = 0; i < count && all; ++i) {
        auto it = ctx->by_ticket.find(tickets[i]);
        if (it == ctx->by_ticket.end()) {
          ctx->err = "pcg_wait: unknown or already collected ticket";
          return PCG_EINVAL;
        }
        all = it->second->st == RQ_DONE;
      }
    }
    if (all) break;
    if (now_ms() >= t_end) return PCG_PENDING;
    int act = 0, q = 0;
    const int rc = pcg_progress(ctx, step, &act, &q);
    if (rc) return rc;
    if (act == 0) {
      PhaseTimer pt(ctx, &pcg_batch_stats::host_idle_ms);
      std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
  }
  // collect every result before any ticket is dropped, so that a ticket
  // listed twice gets its result twice
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (int i = 0; i < count; ++i) {
    auto it = ctx->by_ticket.find(tickets[i]);
    if (it == ctx->by_ticket.end()) {  // collected by another thread meanwhile
      ctx->err = "pcg_wait: ticket collected by another caller";
      return PCG_EINVAL;
    }
    if (results) results[i] = it->second->res;
  }
  for (int i = 0; i < count; ++i) ctx->by_ticket.erase(tickets[i]);
  return PCG_OK;
}

int pcg_wait(pcg_ctx *ctx, int count, const uint64_t *tickets, pcg_result *results, double timeout_s) {
  if (!ctx || count < 0 || (count > 0 && !tickets)) return PCG_EINVAL;
  HIPCHK(hipSetDevice(ctx->cfg.device));
  return wait_tickets(ctx, count, tickets, results, timeout_s, ctx->cfg.graph_iters);
}

int pcg_solve_batch(pcg_ctx *ctx, int count, const pcg_system *sys, pcg_result *results, int iters_per_step) {
  if (!ctx || count < 0 || (count > 0 && (!sys || !results))) return PCG_EINVAL;
  std::vector<uint64_t> t(count);
  int rc = pcg_submit_batch(ctx, count, sys, t.data());
  if (rc) return rc;
  return wait_tickets(ctx, count, t.data(), results, -1.0, iters_per_step);
}

int pcg_batch_stats_get(pcg_ctx *ctx, pcg_batch_stats *out, int reset) {
  if (!ctx || !out) return PCG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  *out = ctx->stats;
  if (reset) ctx->stats = pcg_batch_stats{};
  return PCG_OK;
}

int pcg_pool_info(pcg_ctx *ctx, size_t *capacity, size_t *in_use) {
  if (!ctx) return PCG_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (capacity) *capacity = ctx->pool.capacity();
  if (in_use) *in_use = ctx->pool.in_use();
  return PCG_OK;
}

const char *pcg_last_error(const pcg_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

}  // extern "C"
