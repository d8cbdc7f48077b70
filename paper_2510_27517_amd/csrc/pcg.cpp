// Host side of the C ABI in include/pcg.h: context, validation, device
// storage, preconditioner construction, and the solve driver that replays
// captured HIP graphs of whole CG iterations with device-resident scalars.
#include "pcg.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "kernels.h"

using pcgk::DevCSR;
using pcgk::State;
using pcgk::Types;
using pcgk::Vecs;

namespace {

// ------------------------------------------------------------ host helpers

int validate_csr(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, int require_diag, std::string *why) {
  auto fail = [&](const char *m, int64_t i) {
    if (why) {
      char buf[160];
      snprintf(buf, sizeof buf, "%s (at %lld)", m, (long long)i);
      *why = buf;
    }
    return PCG_EINVAL;
  };
  if (n < 0 || nnz < 0 || nnz > INT32_MAX) return fail("bad n or nnz", nnz);
  if (n > 0 && (!rp || (nnz > 0 && !ci))) return fail("null CSR array", 0);
  if (n == 0) return nnz == 0 ? PCG_OK : fail("nnz > 0 with n = 0", nnz);
  if (rp[0] != 0) return fail("rowptr[0] != 0", 0);
  for (int32_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return fail("rowptr decreases", i);
    bool diag = false;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      if (k >= nnz) return fail("rowptr exceeds nnz", i);
      if (ci[k] < 0 || ci[k] >= n) return fail("column out of range", k);
      if (k > rp[i] && ci[k] <= ci[k - 1]) return fail("columns not strictly ascending", k);
      if (ci[k] == i) diag = true;
    }
    if (require_diag && !diag) return fail("missing diagonal entry", i);
  }
  if (rp[n] != nnz) return fail("rowptr[n] != nnz", n);
  return PCG_OK;
}

void transpose_csr(int32_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                   const std::vector<double> &v, std::vector<int32_t> &trp, std::vector<int32_t> &tci,
                   std::vector<double> &tv) {
  const int64_t nnz = rp[n];
  trp.assign(n + 1, 0);
  tci.resize(nnz);
  tv.resize(nnz);
  for (int64_t k = 0; k < nnz; ++k) trp[ci[k] + 1]++;
  for (int32_t j = 0; j < n; ++j) trp[j + 1] += trp[j];
  std::vector<int32_t> pos(trp.begin(), trp.end() - 1);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int32_t p = pos[ci[k]]++;
      tci[p] = i;
      tv[p] = v[k];
    }
}

// Round to nearest, ties to even, onto a binary format with `sig` significant
// bits, minimum normal exponent emin and largest finite value vmax.
double round_to_format(double v, int sig, int emin, double vmax) {
  if (v == 0.0 || !std::isfinite(v)) return v;
  int e;
  std::frexp(std::fabs(v), &e);  // |v| in [2^(e-1), 2^e)
  int q = e - sig;
  if (e - 1 < emin) q = emin - (sig - 1);  // subnormal quantum
  double r = std::ldexp(std::nearbyint(std::ldexp(std::fabs(v), -q)), q);
  if (r > vmax) r = INFINITY;
  return std::copysign(r, v);
}

uint16_t to_bf16_bits(double v) {
  const float f = (float)round_to_format(v, 8, -126, 3.3895313892515355e38);
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (uint16_t)(u >> 16);
}

uint16_t to_f16_bits(double v) {
  const double r = round_to_format(v, 11, -14, 65504.0);
  if (std::isinf(r)) return r > 0 ? 0x7C00 : 0xFC00;
  if (std::isnan(r)) return 0x7E00;
  uint16_t sign = std::signbit(r) ? 0x8000 : 0;
  double a = std::fabs(r);
  if (a == 0.0) return sign;
  int e;
  double m = std::frexp(a, &e);  // a = m 2^e, m in [0.5, 1)
  if (e - 1 >= -14) {
    const uint16_t exp = (uint16_t)(e - 1 + 15);
    const uint16_t frac = (uint16_t)std::lround((m * 2.0 - 1.0) * 1024.0);
    return sign | (uint16_t)(exp << 10) | frac;
  }
  return sign | (uint16_t)std::lround(a * 16777216.0);  // subnormal: multiples of 2^-24
}

// ---------------------------------------------- preconditioner builders (host)

int64_t g_nnz(int kind, int32_t n, const int32_t *rp, const int32_t *ci) {
  if (kind == PCG_G_JACOBI || kind == PCG_G_IDENTITY) return n;
  if (kind != PCG_G_FSAI && kind != PCG_G_FIXED) return -1;
  int64_t c = 0;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) c += (ci[k] <= i);
  return c;
}

// FSAI rows [r0, r1) of the lower factor G_L on tril(A): with A[J,J] = L L^T
// (J = lower pattern of row i, i last), the FSAI row is L^-T e_last, i.e. the
// last column of L^-T, found by one back substitution L^T g = e_last.
int fsai_rows(int32_t r0, int32_t r1, const int32_t *rp, const int32_t *ci, const double *v, const int32_t *lrp,
              int32_t *lci, double *lv, int32_t n) {
  std::vector<int32_t> where(n, -1);
  std::vector<int32_t> J;
  std::vector<double> S, g;
  for (int32_t i = r0; i < r1; ++i) {
    J.clear();
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] <= i) J.push_back(ci[k]);
    const int m = (int)J.size();
    if (m == 0 || J.back() != i) return PCG_EINVAL;
    for (int a = 0; a < m; ++a) where[J[a]] = a;
    S.assign((size_t)m * m, 0.0);
    for (int a = 0; a < m; ++a) {
      const int32_t row = J[a];
      for (int32_t k = rp[row]; k < rp[row + 1]; ++k) {
        const int32_t c = ci[k];
        if (c > i) break;
        const int b = where[c];
        if (b >= 0) S[(size_t)a * m + b] = v[k];
      }
    }
    for (int a = 0; a < m; ++a) where[J[a]] = -1;
    // Cholesky (lower) in place
    for (int c = 0; c < m; ++c) {
      double dsum = S[(size_t)c * m + c];
      for (int k = 0; k < c; ++k) dsum -= S[(size_t)c * m + k] * S[(size_t)c * m + k];
      if (!(dsum > 0.0)) return PCG_EBREAKDOWN;
      const double l = std::sqrt(dsum);
      S[(size_t)c * m + c] = l;
      for (int a = c + 1; a < m; ++a) {
        double e = S[(size_t)a * m + c];
        for (int k = 0; k < c; ++k) e -= S[(size_t)a * m + k] * S[(size_t)c * m + k];
        S[(size_t)a * m + c] = e / l;
      }
    }
    // back substitution L^T g = e_last
    g.assign(m, 0.0);
    for (int a = m - 1; a >= 0; --a) {
      double e = (a == m - 1) ? 1.0 : 0.0;
      for (int k = a + 1; k < m; ++k) e -= S[(size_t)k * m + a] * g[k];
      g[a] = e / S[(size_t)a * m + a];
    }
    for (int a = 0; a < m; ++a) {
      lci[lrp[i] + a] = J[a];
      lv[lrp[i] + a] = g[a];
    }
  }
  return PCG_OK;
}

// Builds G (CSR) for `kind`; for the lower kinds also returns G^T directly.
int build_g(int kind, int32_t n, const int32_t *rp, const int32_t *ci, const double *v, std::vector<int32_t> &grp,
            std::vector<int32_t> &gci, std::vector<double> &gv) {
  if (kind == PCG_G_JACOBI || kind == PCG_G_IDENTITY) {
    grp.resize(n + 1);
    gci.resize(n);
    gv.resize(n);
    for (int32_t i = 0; i <= n; ++i) grp[i] = i;
    for (int32_t i = 0; i < n; ++i) {
      gci[i] = i;
      if (kind == PCG_G_IDENTITY) {
        gv[i] = 1.0;
        continue;
      }
      double d = 0.0;
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] == i) d = v[k];
      if (!(d > 0.0)) return PCG_EINVAL;
      gv[i] = 1.0 / std::sqrt(d);
    }
    return PCG_OK;
  }
  const int64_t m = g_nnz(kind, n, rp, ci);
  if (m < 0) return PCG_EINVAL;
  std::vector<int32_t> lrp(n + 1, 0), lci(m);
  std::vector<double> lv(m);
  for (int32_t i = 0; i < n; ++i) {
    int32_t c = 0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) c += (ci[k] <= i);
    lrp[i + 1] = lrp[i] + c;
  }
  if (kind == PCG_G_FIXED) {
    std::vector<double> dg(n, 0.0);
    for (int32_t i = 0; i < n; ++i)
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
        if (ci[k] == i) dg[i] = v[k];
    for (int32_t i = 0; i < n; ++i) {
      if (!(dg[i] > 0.0)) return PCG_EINVAL;
      int32_t p = lrp[i];
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        const int32_t j = ci[k];
        if (j > i) break;
        lci[p] = j;
        lv[p] = (j == i) ? 1.0 / std::sqrt(dg[i]) : -0.25 * v[k] / std::sqrt(dg[i] * dg[j]);
        ++p;
      }
    }
    grp.swap(lrp);
    gci.swap(lci);
    gv.swap(lv);
    return PCG_OK;  // this G is lower-triangular itself
  }
  // FSAI: G_L rows in parallel, then G = G_L^T
  unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (n < 20000) nt = 1;
  std::vector<int> rcs(nt, PCG_OK);
  std::vector<std::thread> th;
  for (unsigned w = 0; w < nt; ++w) {
    const int32_t a = (int32_t)((int64_t)n * w / nt), b = (int32_t)((int64_t)n * (w + 1) / nt);
    th.emplace_back([&, a, b, w] { rcs[w] = fsai_rows(a, b, rp, ci, v, lrp.data(), lci.data(), lv.data(), n); });
  }
  for (auto &t : th) t.join();
  for (int rc : rcs)
    if (rc != PCG_OK) return rc;
  transpose_csr(n, lrp, lci, lv, grp, gci, gv);
  return PCG_OK;
}

// Row-block partition for the CSR-stream kernels: consecutive rows, at most
// kBlock rows and `cap` nonzeros per block; a longer row is a block alone.
// Returned as (row start, nonzero start) pairs, nblk + 1 of them.
std::vector<int32_t> row_blocks(int32_t n, const int32_t *rp, int cap) {
  std::vector<int32_t> blk;
  blk.push_back(0);
  blk.push_back(rp[0]);
  int32_t start = 0;
  while (start < n) {
    int32_t end = start + 1;
    if (rp[start + 1] - rp[start] <= cap) {
      while (end < n && end - start < pcgk::kBlock && rp[end + 1] - rp[start] <= cap) ++end;
    }
    blk.push_back(end);
    blk.push_back(rp[end]);
    start = end;
  }
  return blk;
}

double bytes_per_iter(int32_t n, int64_t a, int64_t g, int adt, int gdt, int vdt) {
  const double sa = (double)pcgk::dtype_size(adt), sg = (double)pcgk::dtype_size(gdt),
               sv = (double)pcgk::dtype_size(vdt);
  return (double)a * (sa + 4) + 2.0 * (double)g * (sg + 4) + 3.0 * 4.0 * (n + 1.0) + 12.0 * n * sv;
}

}  // namespace

// ----------------------------------------------------------------- context

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

struct pcg_ctx {
  pcg_config cfg{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int cus = 256;
  std::string err;

  // host copies used by pcg_build_precond / G^T construction
  int32_t n = 0;
  std::vector<int32_t> a_rp, a_ci;
  std::vector<double> a_val;
  bool have_a = false, have_g = false;
  int64_t g_nnz = 0;
  double g_scale = 1.0;  // G is stored times this (power of two, half formats)

  std::vector<DevBuf> bufs;  // everything allocated, freed at destroy
  DevCSR A, A64, G, GT;      // A64 shares A's pattern (refinement residual)
  Types ty{};
  Vecs v{};                  // vectors in vec_dtype
  double *x64 = nullptr, *b64 = nullptr, *r64 = nullptr;
  void *tmp_in = nullptr, *tmp_out = nullptr;  // matvec staging (vec dtype)
  double *stage64 = nullptr;                   // FP64 staging of boundary vectors
  State *st = nullptr, *st64 = nullptr;  // two slots each (see State)
  pcgk::Partials parts{};
  double *partials = nullptr;  // backing store of parts: 5 * partial_cap doubles
  int64_t partial_cap = 0;
  State *hst = nullptr;  // pinned: [0..1] status readback, [2] upload
  hipEvent_t ev[2] = {nullptr, nullptr}, t0 = nullptr, t1 = nullptr;
  std::map<int, hipGraphExec_t> graphs;  // key: iters*2 + replace_first
  int32_t vec_n = 0;                     // size the vectors were allocated for
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

int dev_alloc(pcg_ctx *ctx, size_t bytes, void **out) {
  *out = nullptr;
  if (bytes == 0) bytes = 64;
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ctx->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed";
    *out = nullptr;
    return PCG_ENOMEM;
  }
  ctx->bufs.push_back(DevBuf{*out, bytes});
  return PCG_OK;
}

void dev_free(pcg_ctx *ctx, void *p) {
  if (!p) return;
  for (size_t i = 0; i < ctx->bufs.size(); ++i)
    if (ctx->bufs[i].p == p) {
      (void)hipFree(p);
      ctx->bufs.erase(ctx->bufs.begin() + i);
      return;
    }
}

void free_csr(pcg_ctx *ctx, DevCSR &m, bool pattern_too) {
  if (pattern_too) {
    dev_free(ctx, m.rp);
    dev_free(ctx, m.ci);
    dev_free(ctx, m.blk);
  }
  dev_free(ctx, m.val);
  m = DevCSR{};
}

void drop_graphs(pcg_ctx *ctx) {
  for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
  ctx->graphs.clear();
}

int grid_for(pcg_ctx *ctx, int32_t nblk) {
  const int mult = ctx->cfg.grid_mult > 0 ? ctx->cfg.grid_mult : 8;
  int64_t g = std::min<int64_t>(nblk, (int64_t)ctx->cus * mult);
  g = (g + 7) & ~int64_t(7);
  return (int)std::max<int64_t>(g, 8);
}

// Upload a host CSR with values cast to dtype (times `scale`).
int upload_csr(pcg_ctx *ctx, int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int dtype,
               double scale, DevCSR &m) {
  m.n = n;
  m.nnz = rp[n];
  m.dtype = dtype;
  int rc;
  if ((rc = dev_alloc(ctx, sizeof(int32_t) * (n + 1), (void **)&m.rp))) return rc;
  if ((rc = dev_alloc(ctx, sizeof(int32_t) * m.nnz, (void **)&m.ci))) return rc;
  if ((rc = dev_alloc(ctx, pcgk::dtype_size(dtype) * m.nnz, &m.val))) return rc;
  HIPCHK(hipMemcpy(m.rp, rp, sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(m.ci, ci, sizeof(int32_t) * m.nnz, hipMemcpyHostToDevice));
  if (dtype == pcgk::F64 && scale == 1.0) {
    HIPCHK(hipMemcpy(m.val, v, sizeof(double) * m.nnz, hipMemcpyHostToDevice));
  } else {
    std::vector<uint8_t> h(pcgk::dtype_size(dtype) * m.nnz);
    for (int64_t k = 0; k < m.nnz; ++k) {
      const double x = v[k] * scale;
      switch (dtype) {
        case pcgk::F64: ((double *)h.data())[k] = x; break;
        case pcgk::F32: ((float *)h.data())[k] = (float)x; break;
        case pcgk::BF16: ((uint16_t *)h.data())[k] = to_bf16_bits(x); break;
        default: ((uint16_t *)h.data())[k] = to_f16_bits(x); break;
      }
    }
    HIPCHK(hipMemcpy(m.val, h.data(), h.size(), hipMemcpyHostToDevice));
  }
  const int vdt = ctx->cfg.vec_dtype;
  std::vector<int32_t> blk = row_blocks(n, rp, pcgk::lds_cap(vdt));
  m.nblk = (int32_t)blk.size() / 2 - 1;
  if ((rc = dev_alloc(ctx, sizeof(int32_t) * blk.size(), (void **)&m.blk))) return rc;
  HIPCHK(hipMemcpy(m.blk, blk.data(), sizeof(int32_t) * blk.size(), hipMemcpyHostToDevice));
  m.grid = grid_for(ctx, m.nblk);
  return PCG_OK;
}

int ensure_partials(pcg_ctx *ctx) {
  int64_t need = 1024;
  for (const DevCSR *m : {&ctx->A, &ctx->G, &ctx->GT, &ctx->A64})
    if (m->grid > need) need = m->grid;
  if (need <= ctx->partial_cap) return PCG_OK;
  dev_free(ctx, ctx->partials);
  ctx->partial_cap = 0;
  int rc = dev_alloc(ctx, sizeof(double) * 5 * need, (void **)&ctx->partials);
  if (rc) return rc;
  ctx->partial_cap = need;
  ctx->parts.g = ctx->partials;
  ctx->parts.rt = ctx->partials + need;
  ctx->parts.b = ctx->partials + 3 * need;
  ctx->parts.tr = ctx->partials + 4 * need;
  return PCG_OK;
}

int ensure_vectors(pcg_ctx *ctx, int32_t n) {
  if (ctx->vec_n == n && ctx->v.x) return PCG_OK;
  drop_graphs(ctx);
  for (void *p : {ctx->v.x, ctx->v.r0, ctx->v.r1, ctx->v.d0, ctx->v.d1, ctx->v.q, ctx->v.t, ctx->v.s, ctx->v.b,
                  ctx->tmp_in, ctx->tmp_out, (void *)ctx->x64, (void *)ctx->b64, (void *)ctx->r64,
                  (void *)ctx->stage64})
    dev_free(ctx, p);
  ctx->v = Vecs{};
  ctx->x64 = ctx->b64 = ctx->r64 = ctx->stage64 = nullptr;
  const size_t vb = pcgk::dtype_size(ctx->cfg.vec_dtype) * (size_t)std::max(n, 1);
  int rc;
  void **slots[] = {&ctx->v.x, &ctx->v.r0, &ctx->v.r1, &ctx->v.d0, &ctx->v.d1, &ctx->v.q,
                    &ctx->v.t, &ctx->v.s,  &ctx->v.b,  &ctx->tmp_in, &ctx->tmp_out};
  for (void **p : slots)
    if ((rc = dev_alloc(ctx, vb, p))) return rc;
  const size_t db = sizeof(double) * (size_t)std::max(n, 1);
  if ((rc = dev_alloc(ctx, db, (void **)&ctx->stage64))) return rc;
  if (ctx->cfg.refine) {
    if ((rc = dev_alloc(ctx, db, (void **)&ctx->x64))) return rc;
    if ((rc = dev_alloc(ctx, db, (void **)&ctx->b64))) return rc;
    if ((rc = dev_alloc(ctx, db, (void **)&ctx->r64))) return rc;
  }
  ctx->vec_n = n;
  return PCG_OK;
}

// Fetch a CSR given by device pointers to the host (setup only).
int fetch_csr(pcg_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v,
              std::vector<int32_t> &hrp, std::vector<int32_t> &hci, std::vector<double> &hv) {
  hrp.resize(n + 1);
  hci.resize(nnz);
  hv.resize(nnz);
  HIPCHK(hipMemcpy(hrp.data(), rp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
  if (nnz) {
    HIPCHK(hipMemcpy(hci.data(), ci, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hv.data(), v, sizeof(double) * nnz, hipMemcpyDeviceToHost));
  }
  return PCG_OK;
}

int set_g_host(pcg_ctx *ctx, std::vector<int32_t> &grp, std::vector<int32_t> &gci, std::vector<double> &gv) {
  const int32_t n = ctx->n;
  std::vector<int32_t> trp, tci;
  std::vector<double> tv;
  transpose_csr(n, grp, gci, gv, trp, tci, tv);
  drop_graphs(ctx);
  free_csr(ctx, ctx->G, true);
  free_csr(ctx, ctx->GT, true);
  // F16 has a narrow exponent range: store G times a power of two (PCG is
  // invariant to the scale of M^-1 when eps is scaled alike).
  ctx->g_scale = 1.0;
  if (ctx->cfg.g_dtype == pcgk::F16) {
    double mx = 0.0;
    for (double x : gv) mx = std::max(mx, std::fabs(x));
    if (mx > 0) {
      int e;
      std::frexp(mx, &e);
      ctx->g_scale = std::ldexp(1.0, 14 - e);  // max |G| scaled into [2^13, 2^14)
    }
  }
  int rc = upload_csr(ctx, n, grp.data(), gci.data(), gv.data(), ctx->cfg.g_dtype, ctx->g_scale, ctx->G);
  if (rc) return rc;
  rc = upload_csr(ctx, n, trp.data(), tci.data(), tv.data(), ctx->cfg.g_dtype, ctx->g_scale, ctx->GT);
  if (rc) return rc;
  ctx->g_nnz = (int64_t)gci.size();
  ctx->have_g = true;
  return ensure_partials(ctx);
}

// --------------------------------------------------------------- solve core

void enqueue_iteration(pcg_ctx *ctx, const Types &ty, bool replace, hipError_t &e) {
  const double eps = ctx->cfg.eps * ctx->g_scale * ctx->g_scale;
  auto chain = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  const pcgk::Partials &p = ctx->parts;
  chain(pcgk::launch_iter_A(ty, ctx->A, ctx->v, ctx->st, p, ctx->stream));
  if (replace) chain(pcgk::launch_resid(ty, ctx->A, ctx->v, ctx->st, p, 1, true, false, true, ctx->stream));
  const int mode = replace ? 1 : 0;
  chain(pcgk::launch_iter_GT(ty, ctx->GT, ctx->v, ctx->st, p, ctx->A.grid, mode, ctx->stream));
  chain(pcgk::launch_iter_G(ty, ctx->G, ctx->v, ctx->st, p, ctx->GT.grid, eps != 0.0, mode, ctx->stream));
}

// Start (or restart) sequence: t = G^T r, s = G t, delta, beta = 0, tests.
int enqueue_start(pcg_ctx *ctx, const Types &ty, double eps) {
  const pcgk::Partials &p = ctx->parts;
  HIPCHK(pcgk::launch_iter_GT(ty, ctx->GT, ctx->v, ctx->st, p, ctx->A.grid, 2, ctx->stream));
  HIPCHK(pcgk::launch_iter_G(ty, ctx->G, ctx->v, ctx->st, p, ctx->GT.grid, eps != 0.0, 2, ctx->stream));
  return PCG_OK;
}

int get_graph(pcg_ctx *ctx, const Types &ty, int iters, bool replace_first, hipGraphExec_t *out) {
  const int key = iters * 2 + (replace_first ? 1 : 0);
  auto it = ctx->graphs.find(key);
  if (it != ctx->graphs.end()) {
    *out = it->second;
    return PCG_OK;
  }
  HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int k = 0; k < iters; ++k) enqueue_iteration(ctx, ty, replace_first && k == 0, e);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(ctx->stream, &g);
  HIPCHK(e);
  HIPCHK(e2);
  hipGraphExec_t ex = nullptr;
  hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(e3);
  ctx->graphs[key] = ex;
  *out = ex;
  return PCG_OK;
}

struct CoreOut {
  int status = PCG_OK;
  int iters = 0, restarts = 0;
  double rr = 0, true_rr = 0, bb = 0;
};

// Runs PCG on the vectors in ctx->v (b and x0 loaded) with ctx->st.
int solve_core(pcg_ctx *ctx, const Types &ty, double tol, int maxit, CoreOut &out) {
  const int32_t n = ctx->n;
  hipStream_t s = ctx->stream;
  State init{};
  init.maxit = maxit;
  init.tol = tol;
  init.eps = ctx->cfg.eps * ctx->g_scale * ctx->g_scale;
  init.rr_period = ctx->cfg.rr_period;
  ctx->hst[2] = init;
  ctx->hst[3] = init;
  HIPCHK(hipMemcpyAsync(ctx->st, &ctx->hst[2], 2 * sizeof(State), hipMemcpyHostToDevice, s));
  HIPCHK(pcgk::launch_fill(ty.vec, ctx->v.d0, n, 0.0, s));
  HIPCHK(pcgk::launch_fill(ty.vec, ctx->v.d1, n, 0.0, s));
  HIPCHK(pcgk::launch_norm_b(ty, n, ctx->v, ctx->st, ctx->parts, s));
  HIPCHK(pcgk::launch_resid(ty, ctx->A, ctx->v, ctx->st, ctx->parts, 0, false, false, true, s));
  {
    int rc = enqueue_start(ctx, ty, init.eps);
    if (rc) return rc;
  }

  const int rr = ctx->cfg.rr_period;
  int K = ctx->cfg.graph_iters;
  if (K > 0 && rr > 0) {
    int a = K, b = rr;
    while (b) { int t = a % b; a = b; b = t; }
    K = a;  // K divides rr: replacement can only fall on a chunk's first iteration
  }
  int base = 0;  // iterations enqueued so far (exact while not done)
  int restarts = 0;
  for (;;) {
    // chunks in flight: launch up to two ahead, read the status of the oldest
    int inflight = 0, slot_next = 0, slot_wait = 0;
    bool done = false;
    while (!done) {
      while (inflight < 2) {
        const bool rep = rr > 0 && base > 0 && base % rr == 0;
        int len;
        if (K <= 0) {
          hipError_t e = hipSuccess;
          enqueue_iteration(ctx, ty, rep, e);
          HIPCHK(e);
          len = 1;
        } else {
          len = (base % K == 0) ? K : 1;
          hipGraphExec_t g;
          int rc = get_graph(ctx, ty, len, rep, &g);
          if (rc) return rc;
          HIPCHK(hipGraphLaunch(g, s));
        }
        base += len;
        HIPCHK(hipMemcpyAsync(&ctx->hst[slot_next], ctx->st, sizeof(State), hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(ctx->ev[slot_next], s));
        slot_next ^= 1;
        ++inflight;
      }
      HIPCHK(hipEventSynchronize(ctx->ev[slot_wait]));
      const State &h = ctx->hst[slot_wait];
      slot_wait ^= 1;
      --inflight;
      if (h.done) done = true;
    }
    HIPCHK(hipStreamSynchronize(s));
    State h;
    HIPCHK(hipMemcpy(&h, ctx->st, sizeof(State), hipMemcpyDeviceToHost));
    if (h.status == pcgk::ST_ZERO_B) {
      HIPCHK(pcgk::launch_fill(ty.vec, ctx->v.x, n, 0.0, s));
      HIPCHK(hipStreamSynchronize(s));
      out = CoreOut{};
      out.status = PCG_OK;
      return PCG_OK;
    }
    HIPCHK(pcgk::launch_finalize(ty, n, ctx->v, ctx->st, s));
    HIPCHK(pcgk::launch_resid(ty, ctx->A, ctx->v, ctx->st, ctx->parts, 0, false, true, false, s));
    State f;
    HIPCHK(hipMemcpyAsync(&ctx->hst[0], ctx->st, sizeof(State), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    f = ctx->hst[0];
    out.iters = f.iter;
    out.rr = f.rr;
    out.true_rr = f.true_rr;
    out.bb = f.bb;
    out.restarts = restarts;
    if (f.status == pcgk::ST_CONV_REC) {
      if (std::sqrt(f.true_rr) <= f.tol_nb) {
        out.status = PCG_OK;
        return PCG_OK;
      }
      // restart from the true residual (now in the current r slot)
      ++restarts;
      HIPCHK(pcgk::launch_state_restart(ctx->st, s));
      {
        int rc = enqueue_start(ctx, ty, init.eps);
        if (rc) return rc;
      }
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
    HIPCHK(hipMemcpyAsync(ctx->stage64, src, sizeof(double) * n, kind, ctx->stream));
    dsrc = ctx->stage64;
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
    HIPCHK(pcgk::launch_convert(dtype, src, pcgk::F64, ctx->stage64, n, 1.0, ctx->stream));
    HIPCHK(hipMemcpyAsync(dst, ctx->stage64, sizeof(double) * n, kind, ctx->stream));
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return PCG_OK;
}

int refine_solve(pcg_ctx *ctx, double tol, int maxit, pcg_result *res) {
  // FP64 iterative refinement: r64 = b - A64 x64 in FP64; inner FP32 PCG on
  // A c = r64 / ||r64|| to inner_tol; x64 += ||r64|| c.
  const int32_t n = ctx->n;
  hipStream_t s = ctx->stream;
  Types t64{pcgk::F64, pcgk::F64, pcgk::F64};
  Vecs v64{};
  v64.x = ctx->x64;
  v64.b = ctx->b64;
  v64.r0 = ctx->r64;
  v64.r1 = ctx->r64;
  v64.d0 = ctx->r64;
  v64.d1 = ctx->r64;
  State init{};
  init.tol = tol;
  ctx->hst[2] = init;
  ctx->hst[3] = init;
  HIPCHK(hipMemcpyAsync(ctx->st64, &ctx->hst[2], 2 * sizeof(State), hipMemcpyHostToDevice, s));
  HIPCHK(pcgk::launch_norm_b(t64, n, v64, ctx->st64, ctx->parts, s));
  int total_iters = 0, outer = 0, restarts = 0, status = PCG_NOT_CONVERGED;
  double prev = INFINITY, relres = NAN, last_rec = NAN;
  const double inner_tol = ctx->cfg.inner_tol > 0 ? ctx->cfg.inner_tol : 1e-4;
  const int max_outer = ctx->cfg.max_outer > 0 ? ctx->cfg.max_outer : 30;
  for (;;) {
    HIPCHK(pcgk::launch_resid(t64, ctx->A64, v64, ctx->st64, ctx->parts, 0, false, true, false, s));
    HIPCHK(hipMemcpyAsync(&ctx->hst[0], ctx->st64, sizeof(State), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const State h = ctx->hst[0];
    if (h.bb == 0.0) {
      HIPCHK(pcgk::launch_fill(pcgk::F64, ctx->x64, n, 0.0, s));
      status = PCG_OK;
      relres = 0.0;
      break;
    }
    const double rn = std::sqrt(h.true_rr), nb = std::sqrt(h.bb);
    relres = rn / nb;
    if (rn <= tol * nb) {
      status = PCG_OK;
      break;
    }
    if (!std::isfinite(rn)) {
      status = PCG_EBREAKDOWN;
      break;
    }
    if (outer >= max_outer || rn > 0.9 * prev) {
      status = PCG_NOT_CONVERGED;
      break;
    }
    prev = rn;
    // inner right-hand side: r64 / ||r64|| in the vector precision
    HIPCHK(pcgk::launch_convert(pcgk::F64, ctx->r64, ctx->ty.vec, ctx->v.b, n, 1.0 / rn, s));
    HIPCHK(pcgk::launch_fill(ctx->ty.vec, ctx->v.x, n, 0.0, s));
    CoreOut co;
    int rc = solve_core(ctx, ctx->ty, inner_tol, maxit, co);
    if (rc) return rc;
    total_iters += co.iters;
    restarts += co.restarts;
    last_rec = co.bb > 0 ? std::sqrt(co.rr / co.bb) : 0.0;
    if (co.status == PCG_EBREAKDOWN) {
      status = PCG_EBREAKDOWN;
      break;
    }
    HIPCHK(pcgk::launch_refine_update(n, ctx->x64, ctx->v.x, ctx->ty.vec, rn, s));
    ++outer;
  }
  if (res) {
    res->status = status;
    res->iters = total_iters;
    res->outer_iters = outer;
    res->restarts = restarts;
    res->relres_true = relres;
    res->relres_rec = last_rec;
  }
  return status;
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
  cfg->inner_tol = 1e-4;
  cfg->max_outer = 30;
  cfg->graph_iters = 10;
  cfg->grid_mult = 8;
}

int pcg_create(const pcg_config *cfg, pcg_ctx **out) {
  if (!out) return PCG_EINVAL;
  *out = nullptr;
  if (!cfg) return PCG_EINVAL;
  const int v = cfg->vec_dtype, a = cfg->a_dtype, g = cfg->g_dtype;
  const bool ok = (v == PCG_F64 && a == PCG_F64 && g == PCG_F64 && !cfg->refine) ||
                  (v == PCG_F32 && a == PCG_F32 && (g == PCG_F32 || g == PCG_BF16 || g == PCG_F16));
  if (!ok || cfg->rr_period < 0 || cfg->graph_iters < 0 || !(cfg->eps >= 0.0)) return PCG_EINVAL;
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
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, cfg->device) == hipSuccess && prop.multiProcessorCount > 0)
    ctx->cus = prop.multiProcessorCount;
  if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) return fail(PCG_EDEVICE);
  ctx->own_stream = true;
  if (hipHostMalloc((void **)&ctx->hst, sizeof(State) * 4, hipHostMallocDefault) != hipSuccess)
    return fail(PCG_EDEVICE);
  for (auto &e : ctx->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(PCG_EDEVICE);
  if (hipEventCreate(&ctx->t0) != hipSuccess || hipEventCreate(&ctx->t1) != hipSuccess) return fail(PCG_EDEVICE);
  if (dev_alloc(ctx, 2 * sizeof(State), (void **)&ctx->st) || dev_alloc(ctx, 2 * sizeof(State), (void **)&ctx->st64))
    return fail(PCG_ENOMEM);
  if (hipMemset(ctx->st, 0, 2 * sizeof(State)) != hipSuccess || hipMemset(ctx->st64, 0, 2 * sizeof(State)) != hipSuccess)
    return fail(PCG_EDEVICE);
  *out = ctx;
  return PCG_OK;
}

void pcg_destroy(pcg_ctx *ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  drop_graphs(ctx);
  for (auto &b : ctx->bufs) (void)hipFree(b.p);
  ctx->bufs.clear();
  for (auto &e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->t0) (void)hipEventDestroy(ctx->t0);
  if (ctx->t1) (void)hipEventDestroy(ctx->t1);
  if (ctx->hst) (void)hipHostFree(ctx->hst);
  if (ctx->stream && ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

int pcg_set_matrix(pcg_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                   const double *val, int on_device) {
  if (!ctx) return PCG_EINVAL;
  if (n <= 0 || !rowptr || !col || !val) {
    ctx->err = "pcg_set_matrix: n must be positive and arrays non-null";
    return PCG_EINVAL;
  }
  std::vector<int32_t> hrp, hci;
  std::vector<double> hv;
  if (on_device) {
    int rc = fetch_csr(ctx, n, nnz, rowptr, col, val, hrp, hci, hv);
    if (rc) return rc;
  } else {
    hrp.assign(rowptr, rowptr + n + 1);
    if (hrp[n] != nnz) {
      ctx->err = "pcg_set_matrix: rowptr[n] != nnz";
      return PCG_EINVAL;
    }
    hci.assign(col, col + nnz);
    hv.assign(val, val + nnz);
  }
  int rc = validate_csr(n, nnz, hrp.data(), hci.data(), 1, &ctx->err);
  if (rc) return rc;
  drop_graphs(ctx);
  dev_free(ctx, ctx->A64.val);  // A64 shares A's rp/ci but owns its values and row blocks
  dev_free(ctx, ctx->A64.blk);
  ctx->A64 = DevCSR{};
  free_csr(ctx, ctx->A, true);
  if (ctx->have_g && ctx->n != n) {
    free_csr(ctx, ctx->G, true);
    free_csr(ctx, ctx->GT, true);
    ctx->have_g = false;
  }
  ctx->n = n;
  ctx->a_rp.swap(hrp);
  ctx->a_ci.swap(hci);
  ctx->a_val.swap(hv);
  rc = upload_csr(ctx, n, ctx->a_rp.data(), ctx->a_ci.data(), ctx->a_val.data(), ctx->cfg.a_dtype, 1.0, ctx->A);
  if (rc) return rc;
  if (ctx->cfg.refine) {
    // FP64 values on A's pattern for the refinement residual
    ctx->A64 = ctx->A;
    ctx->A64.dtype = pcgk::F64;
    ctx->A64.val = nullptr;
    if ((rc = dev_alloc(ctx, sizeof(double) * std::max<int64_t>(nnz, 1), &ctx->A64.val))) return rc;
    HIPCHK(hipMemcpy(ctx->A64.val, ctx->a_val.data(), sizeof(double) * nnz, hipMemcpyHostToDevice));
    // the FP64 kernels stage FP64 products: their row blocks differ
    std::vector<int32_t> blk = row_blocks(n, ctx->a_rp.data(), pcgk::lds_cap(pcgk::F64));
    ctx->A64.nblk = (int32_t)blk.size() / 2 - 1;
    ctx->A64.blk = nullptr;
    if ((rc = dev_alloc(ctx, sizeof(int32_t) * blk.size(), (void **)&ctx->A64.blk))) return rc;
    HIPCHK(hipMemcpy(ctx->A64.blk, blk.data(), sizeof(int32_t) * blk.size(), hipMemcpyHostToDevice));
    ctx->A64.grid = grid_for(ctx, ctx->A64.nblk);
  }
  ctx->have_a = true;
  if ((rc = ensure_partials(ctx))) return rc;
  return ensure_vectors(ctx, n);
}

int pcg_set_precond(pcg_ctx *ctx, int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                    const double *val, int on_device) {
  if (!ctx) return PCG_EINVAL;
  if (!ctx->have_a) {
    ctx->err = "pcg_set_precond: set the matrix first";
    return PCG_ESTATE;
  }
  if (n != ctx->n) {
    ctx->err = "pcg_set_precond: size differs from A";
    return PCG_ESTATE;
  }
  if (!rowptr || !col || !val) return PCG_EINVAL;
  std::vector<int32_t> hrp, hci;
  std::vector<double> hv;
  if (on_device) {
    int rc = fetch_csr(ctx, n, nnz, rowptr, col, val, hrp, hci, hv);
    if (rc) return rc;
  } else {
    hrp.assign(rowptr, rowptr + n + 1);
    if (hrp[n] != nnz) {
      ctx->err = "pcg_set_precond: rowptr[n] != nnz";
      return PCG_EINVAL;
    }
    hci.assign(col, col + nnz);
    hv.assign(val, val + nnz);
  }
  int rc = validate_csr(n, nnz, hrp.data(), hci.data(), 0, &ctx->err);
  if (rc) return rc;
  return set_g_host(ctx, hrp, hci, hv);
}

int pcg_build_precond(pcg_ctx *ctx, int kind) {
  if (!ctx) return PCG_EINVAL;
  if (!ctx->have_a) {
    ctx->err = "pcg_build_precond: set the matrix first";
    return PCG_ESTATE;
  }
  std::vector<int32_t> grp, gci;
  std::vector<double> gv;
  int rc = build_g(kind, ctx->n, ctx->a_rp.data(), ctx->a_ci.data(), ctx->a_val.data(), grp, gci, gv);
  if (rc) {
    ctx->err = "pcg_build_precond: construction failed (kind or matrix not SPD)";
    return rc;
  }
  return set_g_host(ctx, grp, gci, gv);
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
  const int32_t n = ctx->n;
  int rc;
  HIPCHK(hipSetDevice(ctx->cfg.device));
  if (on_device) HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipEventRecord(ctx->t0, ctx->stream));
  if (ctx->cfg.refine) {
    HIPCHK(hipMemcpyAsync(ctx->b64, b, sizeof(double) * n, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->x64, x, sizeof(double) * n, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          ctx->stream));
    pcg_result r{};
    rc = refine_solve(ctx, tol, maxit, &r);
    if (rc < PCG_EBREAKDOWN) return rc;  // device or memory error
    HIPCHK(hipEventRecord(ctx->t1, ctx->stream));
    HIPCHK(hipMemcpyAsync(x, ctx->x64, sizeof(double) * n, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ctx->t0, ctx->t1));
    r.t_solve_ms = ms;
    r.bytes_per_iter = bytes_per_iter(n, ctx->A.nnz, ctx->g_nnz, ctx->cfg.a_dtype, ctx->cfg.g_dtype, ctx->cfg.vec_dtype);
    if (res) *res = r;
    if (r.status == PCG_EBREAKDOWN) ctx->err = "breakdown: A or M not SPD, or non-finite values";
    return r.status;
  }
  if ((rc = load_vec(ctx, b, on_device, ctx->v.b, ctx->ty.vec, n))) return rc;
  if ((rc = load_vec(ctx, x, on_device, ctx->v.x, ctx->ty.vec, n))) return rc;
  CoreOut co;
  if ((rc = solve_core(ctx, ctx->ty, tol, maxit, co))) return rc;
  HIPCHK(hipEventRecord(ctx->t1, ctx->stream));
  if ((rc = store_vec(ctx, ctx->v.x, ctx->ty.vec, x, on_device, n))) return rc;
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
    res->bytes_per_iter =
        bytes_per_iter(n, ctx->A.nnz, ctx->g_nnz, ctx->cfg.a_dtype, ctx->cfg.g_dtype, ctx->cfg.vec_dtype);
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
  const int32_t n = ctx->n;
  const int vdt = ctx->ty.vec;
  int rc;
  HIPCHK(hipSetDevice(ctx->cfg.device));
  if (on_device) HIPCHK(hipDeviceSynchronize());
  if ((rc = load_vec(ctx, x, on_device, ctx->tmp_in, vdt, n))) return rc;
  hipStream_t s = ctx->stream;
  const double inv_scale2 = 1.0 / (ctx->g_scale * ctx->g_scale);
  switch (op) {
    case PCG_OP_A: HIPCHK(pcgk::launch_spmv(ctx->ty, ctx->A, ctx->A.dtype, ctx->tmp_in, ctx->tmp_out, s)); break;
    case PCG_OP_GT:
      HIPCHK(pcgk::launch_spmv(ctx->ty, ctx->GT, ctx->GT.dtype, ctx->tmp_in, ctx->tmp_out, s));
      if (ctx->g_scale != 1.0) HIPCHK(pcgk::launch_axpby(vdt, n, 1.0 / ctx->g_scale, ctx->tmp_out, 0.0, ctx->tmp_in, s));
      break;
    case PCG_OP_G:
      HIPCHK(pcgk::launch_spmv(ctx->ty, ctx->G, ctx->G.dtype, ctx->tmp_in, ctx->tmp_out, s));
      if (ctx->g_scale != 1.0) HIPCHK(pcgk::launch_axpby(vdt, n, 1.0 / ctx->g_scale, ctx->tmp_out, 0.0, ctx->tmp_in, s));
      break;
    default:
      HIPCHK(pcgk::launch_spmv(ctx->ty, ctx->GT, ctx->GT.dtype, ctx->tmp_in, ctx->v.t, s));
      HIPCHK(pcgk::launch_spmv(ctx->ty, ctx->G, ctx->G.dtype, ctx->v.t, ctx->tmp_out, s));
      HIPCHK(pcgk::launch_axpby(vdt, n, inv_scale2, ctx->tmp_out, ctx->cfg.eps, ctx->tmp_in, s));
      break;
  }
  return store_vec(ctx, ctx->tmp_out, vdt, y, on_device, n);
}

int pcg_time_kernels(pcg_ctx *ctx, int iters, double *ms, double *bytes) {
  if (!ctx) return PCG_EINVAL;
  if (!ms || iters < 1 || iters > 100000) return PCG_EINVAL;
  if (!ctx->have_a || !ctx->have_g) {
    ctx->err = "pcg_time_kernels: matrix and preconditioner must be set";
    return PCG_ESTATE;
  }
  const int32_t n = ctx->n;
  const Types ty = ctx->ty;
  hipStream_t s = ctx->stream;
  HIPCHK(hipSetDevice(ctx->cfg.device));
  // a fresh solve of the stored right-hand side from x0 = 0 that never stops
  State init{};
  init.maxit = INT32_MAX;
  init.tol = -1.0;
  init.eps = ctx->cfg.eps * ctx->g_scale * ctx->g_scale;
  ctx->hst[2] = init;
  ctx->hst[3] = init;
  HIPCHK(hipMemcpyAsync(ctx->st, &ctx->hst[2], 2 * sizeof(State), hipMemcpyHostToDevice, s));
  HIPCHK(pcgk::launch_fill(ty.vec, ctx->v.x, n, 0.0, s));
  HIPCHK(pcgk::launch_fill(ty.vec, ctx->v.d0, n, 0.0, s));
  HIPCHK(pcgk::launch_fill(ty.vec, ctx->v.d1, n, 0.0, s));
  HIPCHK(pcgk::launch_norm_b(ty, n, ctx->v, ctx->st, ctx->parts, s));
  HIPCHK(pcgk::launch_resid(ty, ctx->A, ctx->v, ctx->st, ctx->parts, 0, false, false, true, s));
  {
    int rc0 = enqueue_start(ctx, ty, init.eps);
    if (rc0) return rc0;
  }
  HIPCHK(hipStreamSynchronize(s));
  State h;
  HIPCHK(hipMemcpy(&h, ctx->st, sizeof(State), hipMemcpyDeviceToHost));
  if (h.done) {
    ctx->err = "pcg_time_kernels: solve a nonzero right-hand side first";
    return PCG_ESTATE;
  }
  std::vector<hipEvent_t> ev(4 * (size_t)iters, nullptr);
  int rc = PCG_OK;
  for (auto &e : ev)
    if (hipEventCreate(&e) != hipSuccess) rc = PCG_EDEVICE;
  double acc[4] = {0, 0, 0, 0};
  if (rc == PCG_OK) {
    hipError_t e = hipSuccess;
    auto chain = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    for (int it = 0; it < iters; ++it) {
      chain(hipEventRecord(ev[4 * it], s));
      chain(pcgk::launch_iter_A(ty, ctx->A, ctx->v, ctx->st, ctx->parts, s));
      chain(hipEventRecord(ev[4 * it + 1], s));
      chain(pcgk::launch_iter_GT(ty, ctx->GT, ctx->v, ctx->st, ctx->parts, ctx->A.grid, 0, s));
      chain(hipEventRecord(ev[4 * it + 2], s));
      chain(pcgk::launch_iter_G(ty, ctx->G, ctx->v, ctx->st, ctx->parts, ctx->GT.grid, init.eps != 0.0, 0, s));
      chain(hipEventRecord(ev[4 * it + 3], s));
    }
    chain(hipStreamSynchronize(s));
    for (int it = 0; it < iters && e == hipSuccess; ++it) {
      float t;
      for (int k = 0; k < 3; ++k) {
        chain(hipEventElapsedTime(&t, ev[4 * it + k], ev[4 * it + k + 1]));
        acc[k] += t;
      }
      chain(hipEventElapsedTime(&t, ev[4 * it], ev[4 * it + 3]));
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
  HIPCHK(hipMemcpy(&h, ctx->st, sizeof(State), hipMemcpyDeviceToHost));
  if (h.done) {
    ctx->err = "pcg_time_kernels: the iteration stopped (breakdown) while timing";
    return PCG_EBREAKDOWN;
  }
  for (int k = 0; k < 4; ++k) ms[k] = acc[k] / iters;
  if (bytes) {
    const double sa = (double)pcgk::dtype_size(ctx->cfg.a_dtype), sg = (double)pcgk::dtype_size(ctx->cfg.g_dtype),
                 sv = (double)pcgk::dtype_size(ctx->cfg.vec_dtype);
    const double rp = 4.0 * (n + 1.0);
    bytes[0] = (double)ctx->A.nnz * (sa + 4) + rp + 6.0 * n * sv;
    bytes[1] = (double)ctx->GT.nnz * (sg + 4) + rp + 4.0 * n * sv;
    bytes[2] = (double)ctx->G.nnz * (sg + 4) + rp + (init.eps != 0.0 ? 3.0 : 2.0) * n * sv;
    bytes[3] = bytes[0] + bytes[1] + bytes[2];
  }
  return PCG_OK;
}

int pcg_copy_bandwidth(int device, int64_t bytes, int reps, double *gbps, double *ms_per_copy) {
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
  if (hipMalloc(&src, bytes) != hipSuccess || hipMalloc(&dst, bytes) != hipSuccess) rc = PCG_ENOMEM;
  if (!rc && (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
              hipEventCreate(&e1) != hipSuccess))
    rc = PCG_EDEVICE;
  if (!rc && hipMemsetAsync(src, 0, bytes, s) != hipSuccess) rc = PCG_EDEVICE;
  float ms = 0.0f;
  if (!rc) {
    const int grid = cus * 16;
    hipError_t e = hipSuccess;
    for (int w = 0; w < 2 && e == hipSuccess; ++w) e = pcgk::launch_copy(src, dst, bytes, grid, s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = pcgk::launch_copy(src, dst, bytes, grid, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) rc = PCG_EDEVICE;
  }
  if (!rc) {
    *gbps = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    if (ms_per_copy) *ms_per_copy = ms / reps;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (src) (void)hipFree(src);
  if (dst) (void)hipFree(dst);
  (void)hipGetLastError();
  return rc;
}

int pcg_validate_csr(int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col, int require_diag) {
  return validate_csr(n, nnz, rowptr, col, require_diag, nullptr);
}

int64_t pcg_g_nnz(int kind, int32_t n, const int32_t *rowptr, const int32_t *col) {
  if (n <= 0 || !rowptr || !col) return -1;
  return g_nnz(kind, n, rowptr, col);
}

int pcg_build_g_host(int kind, int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                     int32_t *g_rowptr, int32_t *g_col, double *g_val) {
  if (n <= 0 || !rowptr || !col || !val || !g_rowptr || !g_col || !g_val) return PCG_EINVAL;
  int rc = validate_csr(n, rowptr[n], rowptr, col, 1, nullptr);
  if (rc) return rc;
  std::vector<int32_t> grp, gci;
  std::vector<double> gv;
  rc = build_g(kind, n, rowptr, col, val, grp, gci, gv);
  if (rc) return rc;
  std::memcpy(g_rowptr, grp.data(), sizeof(int32_t) * grp.size());
  std::memcpy(g_col, gci.data(), sizeof(int32_t) * gci.size());
  std::memcpy(g_val, gv.data(), sizeof(double) * gv.size());
  return PCG_OK;
}

double pcg_bytes_per_iter(int32_t n, int64_t nnz_a, int64_t nnz_g, int a_dtype, int g_dtype, int vec_dtype) {
  return bytes_per_iter(n, nnz_a, nnz_g, a_dtype, g_dtype, vec_dtype);
}

const char *pcg_last_error(const pcg_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

const char *pcg_strerror(int status) {
  switch (status) {
    case PCG_OK: return "ok";
    case PCG_PENDING: return "pending";
    case PCG_NOT_CONVERGED: return "not converged (maxit reached)";
    case PCG_EINVAL: return "invalid argument";
    case PCG_ESTATE: return "invalid state";
    case PCG_ENOMEM: return "out of device memory";
    case PCG_EBREAKDOWN: return "breakdown (matrix or preconditioner not SPD, or non-finite values)";
    case PCG_EDEVICE: return "device error";
    default: return "unknown status";
  }
}

}  // extern "C"
