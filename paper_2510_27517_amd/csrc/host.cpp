// Host-side building blocks (see host.h) and the host-only C ABI entry points.
#include "host.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <thread>

#include <sched.h>

#include "kernels.h"
#include "pcg.h"

namespace pcgh {

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

// 3x3 blocks of block row I on or left of the diagonal block (from row 3I,
// whose columns come in complete triples in an exactly 3x3-blocked matrix).
static int32_t tril_blocks(int32_t I, const int32_t *rp, const int32_t *ci) {
  int32_t m = 0;
  for (int32_t k = rp[3 * I]; k < rp[3 * I + 1] && ci[k] <= 3 * I + 2; k += 3) ++m;
  return m;
}

int64_t g_nnz(int kind, int32_t n, const int32_t *rp, const int32_t *ci) {
  if (kind == PCG_G_JACOBI || kind == PCG_G_IDENTITY) return n;
  if (kind == PCG_G_SEEDED) return rp[n];
  if (kind == PCG_G_BFSAI) {
    if (!is_block3(n, rp, ci, nullptr)) return -1;
    int64_t c = 0;
    for (int32_t I = 0; I < n / 3; ++I) c += 9 * (int64_t)tril_blocks(I, rp, ci);
    return c;
  }
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

// Block FSAI rows of the lower factor G_L for block rows [I0, I1) of an
// exactly 3x3-blocked A: with J the tril blocks of block row I (I last),
// A[J,J] = L L^T (3|J| x 3|J|), block row I of G_L is the last three rows of
// L^-1 (three back substitutions L^T w = e), so that its diagonal block is
// the inverse of L's trailing 3x3 block and each diagonal block of
// G_L A G_L^T is the identity. Every 3x3 block is stored whole (zeros above
// the diagonal of the diagonal block included).
int bfsai_rows(int32_t I0, int32_t I1, const int32_t *rp, const int32_t *ci, const double *v, const int32_t *lrp,
               int32_t *lci, double *lv, int32_t n) {
  std::vector<int32_t> where(n / 3, -1), J;
  std::vector<double> S, w;
  for (int32_t I = I0; I < I1; ++I) {
    J.clear();
    for (int32_t k = rp[3 * I]; k < rp[3 * I + 1] && ci[k] <= 3 * I + 2; k += 3) J.push_back(ci[k] / 3);
    const int m = (int)J.size(), M = 3 * m;
    if (m == 0 || J.back() != I) return PCG_EINVAL;
    for (int a = 0; a < m; ++a) where[J[a]] = a;
    S.assign((size_t)M * M, 0.0);
    for (int a = 0; a < m; ++a)
      for (int s = 0; s < 3; ++s) {
        const int32_t row = 3 * J[a] + s;
        for (int32_t k = rp[row]; k < rp[row + 1]; ++k) {
          const int32_t c = ci[k];
          if (c > 3 * I + 2) break;
          const int b = where[c / 3];
          if (b >= 0) S[(size_t)(3 * a + s) * M + 3 * b + c % 3] = v[k];
        }
      }
    for (int a = 0; a < m; ++a) where[J[a]] = -1;
    for (int c = 0; c < M; ++c) {  // Cholesky (lower) in place
      double dsum = S[(size_t)c * M + c];
      for (int k = 0; k < c; ++k) dsum -= S[(size_t)c * M + k] * S[(size_t)c * M + k];
      if (!(dsum > 0.0)) return PCG_EBREAKDOWN;
      const double l = std::sqrt(dsum);
      S[(size_t)c * M + c] = l;
      for (int a = c + 1; a < M; ++a) {
        double e = S[(size_t)a * M + c];
        for (int k = 0; k < c; ++k) e -= S[(size_t)a * M + k] * S[(size_t)c * M + k];
        S[(size_t)a * M + c] = e / l;
      }
    }
    for (int p = 0; p < 3; ++p) {  // row p of the block row: L^T w = e_(M-3+p)
      w.assign(M, 0.0);
      for (int a = M - 1; a >= 0; --a) {
        double e = (a == M - 3 + p) ? 1.0 : 0.0;
        for (int k = a + 1; k < M; ++k) e -= S[(size_t)k * M + a] * w[k];
        w[a] = e / S[(size_t)a * M + a];
      }
      const int32_t r = 3 * I + p;
      for (int a = 0; a < M; ++a) {
        lci[lrp[r] + a] = 3 * J[a / 3] + a % 3;
        lv[lrp[r] + a] = w[a];
      }
    }
  }
  return PCG_OK;
}

// SplitMix64 (Steele, Lea and Flood 2014) used as a counter generator: draw
// k of stream `stream` under `seed` is mix(key + (k + 1) GAMMA) with
// key = mix(mix(seed + GAMMA) + (stream + 1) GAMMA); U(0,1] from its top 53 bits.
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t kStreamG = 3;  // stream of the seeded preconditioner's draws

inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

inline double sm_u01(uint64_t key, uint64_t k) {
  return (double)((sm_mix(key + (k + 1) * kGamma) >> 11) + 1) * 0x1.0p-53;
}

// Seeded G on A's full pattern (stand-in for a learned G of that shape).
int build_seeded(uint64_t seed, int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                 std::vector<int32_t> &grp, std::vector<int32_t> &gci, std::vector<double> &gv) {
  std::vector<double> dg(n, 0.0);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] == i) dg[i] = v[k];
  for (int32_t i = 0; i < n; ++i)
    if (!(dg[i] > 0.0)) return PCG_EINVAL;
  const uint64_t key = sm_mix(sm_mix(seed + kGamma) + (kStreamG + 1) * kGamma);
  grp.assign(rp, rp + n + 1);
  gci.assign(ci, ci + rp[n]);
  gv.resize(rp[n]);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int32_t j = ci[k];
      if (j == i) {
        gv[k] = 1.0 / std::sqrt(dg[i]);
      } else {
        const double u = 2.0 * sm_u01(key, (uint64_t)i * (uint64_t)n + (uint64_t)j) - 1.0;
        gv[k] = 0.25 * u * std::fabs(v[k]) / std::sqrt(dg[i] * dg[j]);
      }
    }
  return PCG_OK;
}

// Builds G (CSR) for `kind`; for the lower kinds also returns G^T directly.
unsigned available_cpus() {
  cpu_set_t cs;
  if (sched_getaffinity(0, sizeof cs, &cs) == 0) return (unsigned)std::max(1, CPU_COUNT(&cs));
  return std::max(1u, std::thread::hardware_concurrency());
}

int build_g(int kind, uint64_t seed, int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
            std::vector<int32_t> &grp, std::vector<int32_t> &gci, std::vector<double> &gv, int threads) {
  const unsigned nthreads = std::min(32u, threads > 0 ? (unsigned)threads : available_cpus());
  if (kind == PCG_G_SEEDED) return build_seeded(seed, n, rp, ci, v, grp, gci, gv);
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
  if (kind == PCG_G_BFSAI) {
    for (int32_t I = 0; I < n / 3; ++I)
      for (int p = 0; p < 3; ++p) lrp[3 * I + p + 1] = lrp[3 * I + p] + 3 * tril_blocks(I, rp, ci);
    const int32_t nb = n / 3;
    const unsigned nt = nb < 2000 ? 1u : nthreads;
    std::vector<int> rcs(nt, PCG_OK);
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nt; ++w) {
      const int32_t a = (int32_t)((int64_t)nb * w / nt), b = (int32_t)((int64_t)nb * (w + 1) / nt);
      th.emplace_back([&, a, b, w] { rcs[w] = bfsai_rows(a, b, rp, ci, v, lrp.data(), lci.data(), lv.data(), n); });
    }
    for (auto &t : th) t.join();
    for (int rc : rcs)
      if (rc != PCG_OK) return rc;
    transpose_csr(n, lrp, lci, lv, grp, gci, gv);
    return PCG_OK;
  }
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
  const unsigned nt = n < 20000 ? 1u : nthreads;
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

int64_t sell_entries(int32_t n, const int32_t *rp) {
  int64_t tot = 0;
  for (int32_t r0 = 0; r0 < n; r0 += kSlice) {
    int32_t w = 0;
    for (int32_t r = r0; r < std::min(n, r0 + kSlice); ++r) w = std::max(w, rp[r + 1] - rp[r]);
    tot += (int64_t)w * kSlice;
  }
  return tot;
}

void sell_offsets(int32_t n, const int32_t *rp, std::vector<int32_t> &so) {
  const int32_t ns = (n + kSlice - 1) / kSlice;
  so.assign(ns + 1, 0);
  for (int32_t c = 0; c < ns; ++c) {
    int32_t w = 0;
    for (int32_t r = c * kSlice; r < std::min(n, (c + 1) * kSlice); ++r) w = std::max(w, rp[r + 1] - rp[r]);
    so[c + 1] = so[c] + w;
  }
}

void sell_columns(int32_t n, const int32_t *rp, const int32_t *ci, const std::vector<int32_t> &so,
                  std::vector<int32_t> &out) {
  const int32_t ns = (int32_t)so.size() - 1;
  out.resize((size_t)so[ns] * kSlice);
  for (int32_t c = 0; c < ns; ++c)
    for (int32_t l = 0; l < kSlice; ++l) {
      const int32_t r = c * kSlice + l;
      const int32_t len = r < n ? rp[r + 1] - rp[r] : 0;
      for (int32_t k = 0; k < so[c + 1] - so[c]; ++k)
        out[((size_t)so[c] + k) * kSlice + l] = k < len ? ci[rp[r] + k] : (r < n ? r : 0);
    }
}

void sell_bytes(int32_t n, const int32_t *rp, const uint8_t *in, size_t esz, const std::vector<int32_t> &so,
                std::vector<uint8_t> &out) {
  const int32_t ns = (int32_t)so.size() - 1;
  out.assign((size_t)so[ns] * kSlice * esz, 0);
  for (int32_t r = 0; r < n; ++r) {
    const int32_t c = r / kSlice, l = r % kSlice;
    for (int32_t k = 0; k < rp[r + 1] - rp[r]; ++k)
      std::memcpy(&out[(((size_t)so[c] + k) * kSlice + l) * esz], in + (size_t)(rp[r] + k) * esz, esz);
  }
}

// The distinct offsets of slice c's entries, ascending.
static void slice_offsets(int32_t n, const int32_t *rp, const int32_t *ci, int32_t c, std::vector<int32_t> &d) {
  d.clear();
  for (int32_t r = c * kSlice; r < std::min(n, (c + 1) * kSlice); ++r)
    for (int32_t k = rp[r]; k < rp[r + 1]; ++k) d.push_back(ci[k] - r);
  std::sort(d.begin(), d.end());
  d.erase(std::unique(d.begin(), d.end()), d.end());
}

int64_t sdia_entries(int32_t n, const int32_t *rp, const int32_t *ci, int64_t stop) {
  const int32_t ns = (n + kSlice - 1) / kSlice;
  std::vector<int32_t> d;
  int64_t tot = 0;
  for (int32_t c = 0; c < ns && tot <= stop; ++c) {
    slice_offsets(n, rp, ci, c, d);
    tot += (int64_t)d.size() * kSlice;
  }
  return tot;
}

void sdia_pattern(int32_t n, const int32_t *rp, const int32_t *ci, std::vector<int32_t> &so,
                  std::vector<int32_t> &offs) {
  const int32_t ns = (n + kSlice - 1) / kSlice;
  so.assign(ns + 1, 0);
  offs.clear();
  std::vector<int32_t> d;
  for (int32_t c = 0; c < ns; ++c) {
    slice_offsets(n, rp, ci, c, d);
    offs.insert(offs.end(), d.begin(), d.end());
    so[c + 1] = (int32_t)offs.size();
  }
}

void sdia_bytes(int32_t n, const int32_t *rp, const int32_t *ci, const uint8_t *in, size_t esz,
                const std::vector<int32_t> &so, const std::vector<int32_t> &offs, std::vector<uint8_t> &out) {
  const int32_t ns = (int32_t)so.size() - 1;
  out.assign((size_t)so[ns] * kSlice * esz, 0);
  for (int32_t r = 0; r < n; ++r) {
    const int32_t c = r / kSlice, l = r % kSlice;
    int32_t k = so[c];
    for (int32_t q = rp[r]; q < rp[r + 1]; ++q) {  // both ascending: one merge pass
      while (offs[k] != ci[q] - r) ++k;
      std::memcpy(&out[((size_t)k * kSlice + l) * esz], in + (size_t)q * esz, esz);
    }
  }
}

bool is_block3(int32_t n, const int32_t *rp, const int32_t *ci, int64_t *blocks) {
  if (n <= 0 || n % 3) return false;
  int64_t nb = 0;
  for (int32_t R = 0; R < n / 3; ++R) {
    const int32_t r = 3 * R, len = rp[r + 1] - rp[r];
    if (len % 3 || rp[r + 2] - rp[r + 1] != len || rp[r + 3] - rp[r + 2] != len) return false;
    for (int32_t k = 0; k < len; k += 3) {
      const int32_t c = ci[rp[r] + k];
      if (c % 3) return false;
      for (int s = 0; s < 3; ++s)
        for (int j = 0; j < 3; ++j)
          if (ci[rp[r + s] + k + j] != c + j) return false;
    }
    nb += len / 3;
  }
  if (blocks) *blocks = nb;
  return true;
}

int64_t bsell_blocks(int32_t n, const int32_t *rp) {
  const int32_t nbr = n / 3;
  int64_t tot = 0;
  for (int32_t R0 = 0; R0 < nbr; R0 += kBSlice) {
    int32_t w = 0;
    for (int32_t R = R0; R < std::min(nbr, R0 + kBSlice); ++R) w = std::max(w, (rp[3 * R + 1] - rp[3 * R]) / 3);
    tot += (int64_t)w * kBSlice;
  }
  return tot;
}

void bsell_pattern(int32_t n, const int32_t *rp, const int32_t *ci, std::vector<int32_t> &bo,
                   std::vector<int32_t> &bcol) {
  const int32_t nbr = n / 3, ns = (nbr + kBSlice - 1) / kBSlice;
  bo.assign(ns + 1, 0);
  for (int32_t c = 0; c < ns; ++c) {
    int32_t w = 0;
    for (int32_t R = c * kBSlice; R < std::min(nbr, (c + 1) * kBSlice); ++R)
      w = std::max(w, (rp[3 * R + 1] - rp[3 * R]) / 3);
    bo[c + 1] = bo[c] + w;
  }
  bcol.resize((size_t)bo[ns] * kBSlice);
  for (int32_t c = 0; c < ns; ++c)
    for (int32_t r = 0; r < kBSlice; ++r) {
      const int32_t R = c * kBSlice + r;
      const int32_t nbk = R < nbr ? (rp[3 * R + 1] - rp[3 * R]) / 3 : 0;
      for (int32_t k = 0; k < bo[c + 1] - bo[c]; ++k)
        bcol[((size_t)bo[c] + k) * kBSlice + r] = k < nbk ? ci[rp[3 * R] + 3 * k] / 3 : (R < nbr ? R : 0);
    }
}

void bsell_bytes(int32_t n, const int32_t *rp, const uint8_t *in, size_t esz, const std::vector<int32_t> &bo,
                 std::vector<uint8_t> &out) {
  const int32_t nbr = n / 3, ns = (int32_t)bo.size() - 1;
  out.assign((size_t)bo[ns] * kBSlice * 9 * esz, 0);
  for (int32_t R = 0; R < nbr; ++R) {
    const int32_t c = R / kBSlice, r = R % kBSlice, nbk = (rp[3 * R + 1] - rp[3 * R]) / 3;
    for (int32_t k = 0; k < nbk; ++k)
      for (int s = 0; s < 3; ++s)
        for (int j = 0; j < 3; ++j) {
          const size_t pos = esz == 8 ? (((size_t)bo[c] + k) * 3 + j) * 3 * kBSlice + (size_t)s * kBSlice + r
                                      : (((size_t)bo[c] + k) * kBSlice + r) * 9 + 3 * s + j;
          std::memcpy(&out[pos * esz], in + (size_t)(rp[3 * R + s] + 3 * k + j) * esz, esz);
        }
  }
}

double bytes_per_iter(int32_t n, int64_t a, int64_t g, int adt, int gdt, int vdt) {
  const double sa = (double)pcgk::dtype_size(adt), sg = (double)pcgk::dtype_size(gdt),
               sv = (double)pcgk::dtype_size(vdt);
  return (double)a * (sa + 4) + 2.0 * (double)g * (sg + 4) + 3.0 * 4.0 * (n + 1.0) + 11.0 * n * sv;
}

}  // namespace pcgh

extern "C" {

int pcg_validate_csr(int32_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col, int require_diag) {
  return pcgh::validate_csr(n, nnz, rowptr, col, require_diag, nullptr);
}

int64_t pcg_g_nnz(int kind, int32_t n, const int32_t *rowptr, const int32_t *col) {
  if (n <= 0 || !rowptr || !col) return -1;
  return pcgh::g_nnz(kind, n, rowptr, col);
}

int pcg_build_g_host(int kind, uint64_t seed, int32_t n, const int32_t *rowptr, const int32_t *col,
                     const double *val, int32_t *g_rowptr, int32_t *g_col, double *g_val) {
  if (n <= 0 || !rowptr || !col || !val || !g_rowptr || !g_col || !g_val) return PCG_EINVAL;
  int rc = pcgh::validate_csr(n, rowptr[n], rowptr, col, 1, nullptr);
  if (rc) return rc;
  std::vector<int32_t> grp, gci;
  std::vector<double> gv;
  rc = pcgh::build_g(kind, seed, n, rowptr, col, val, grp, gci, gv);
  if (rc) return rc;
  std::memcpy(g_rowptr, grp.data(), sizeof(int32_t) * grp.size());
  std::memcpy(g_col, gci.data(), sizeof(int32_t) * gci.size());
  std::memcpy(g_val, gv.data(), sizeof(double) * gv.size());
  return PCG_OK;
}

int pcg_estimate_bytes(const pcg_config *cfg, int32_t n, int64_t nnz_a, int64_t nnz_g, size_t *bytes) {
  if (!cfg || !bytes || n <= 0 || nnz_a < 0 || nnz_g < 0) return PCG_EINVAL;
  const double sa = (double)pcgk::dtype_size(cfg->a_dtype), sg = (double)pcgk::dtype_size(cfg->g_dtype),
               sv = (double)pcgk::dtype_size(cfg->vec_dtype);
  const double pad = 1.125;  // sliced layouts keep padding within 1/8
  const double blocks = 8.0 * ((double)n / 32.0 + 2.0);  // row blocks or slice offsets
  double b = pad * (double)nnz_a * (sa + 4.0) + 4.0 * (n + 1.0) + blocks;        // A
  b += 2.0 * (pad * (double)nnz_g * (sg + 4.0) + 4.0 * (n + 1.0) + blocks);      // G, G^T
  b += (8.0 + 2.0) * (double)n * sv + 8.0 * (double)n;                           // vectors, staging
  b += 8.0 * 6.0 * 2.0 * 256.0 * std::max(cfg->grid_mult, 8);                         // partial sums
  if (cfg->refine) b += pad * 8.0 * (double)nnz_a + blocks + 3.0 * 8.0 * (double)n;  // FP64 view of A
  b += 256.0 * 32.0;                                                             // alignment of the carved arrays
  *bytes = (size_t)b;
  return PCG_OK;
}

double pcg_bytes_per_iter(int32_t n, int64_t nnz_a, int64_t nnz_g, int a_dtype, int g_dtype, int vec_dtype) {
  return pcgh::bytes_per_iter(n, nnz_a, nnz_g, a_dtype, g_dtype, vec_dtype);
}

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

static_assert(pcgh::kSlice == pcgk::kSliceRows, "slice height shared by host layout and kernels");
