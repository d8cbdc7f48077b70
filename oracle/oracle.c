/*
 * FP64 CPU oracle for preconditioned CG with a factorized sparse approximate
 * inverse, M^-1 = G G^T + eps I (paper Sec. 3.2.1, Eq. "major"; PCG in
 * Appendix A, Algorithm 1).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
 * HIP library is checked against. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it. It shares no code with the HIP
 * path: its own CSR SpMV, transpose, FSAI and PCG loop, written for obvious
 * correctness (plain loops, FP64 throughout, no blocking or fusion).
 *
 * Build with floating-point contraction off (-ffp-contract=off), so each
 * product and each sum is rounded on its own, in the order written here.
 * Inner products (dot products and norms) are the exception: each is the
 * exact sum of its products, rounded once (the reading is stated where the
 * accumulator is defined), so they do not depend on the order or on the
 * thread count.
 *
 * Pins (tests/test_oracle.py): dense brute-force matvec, adjoint identity,
 * the paper's two-hop locality formula for the apply (Eq. "spai-locality"),
 * finite termination, one-iteration convergence with G = L^-T, monotone
 * A-norm error, agreement with scipy's CG for G = I and G = D^-1/2,
 * power-of-two scale invariance, and the FSAI invariants. The FP32 products
 * (or_spmv_f32, or_spmv_t_f32) are pinned bit for bit against a float32
 * brute force that adds each row's products one at a time in numpy binary32
 * scalars, on data whose sums change with the order or with a wider
 * accumulator, and exactly on small integers. The exact inner product is
 * pinned against rational arithmetic (Python's Fraction) on cancelling,
 * wide-range, subnormal and overflowing data, ties to even and a sticky bit,
 * a subnormal result that a double rounding would get wrong, and for
 * independence from order and thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* status codes (same numeric meaning as the library's public ones) */
#define OR_OK 0
#define OR_NOT_CONVERGED 2
#define OR_EINVAL (-1)
#define OR_EBREAKDOWN (-4)

/* ---------------------------------------------------------------- SpMV */

/* y = A x. Each row is summed left to right in CSR order, starting at 0. */
void or_spmv(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, const double *x, double *y,
             int threads) {
#pragma omp parallel for num_threads(threads) schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s += v[k] * x[ci[k]];
    y[i] = s;
  }
}

/* y = G^T x for an nrows x ncols CSR matrix G, by scattering row i of G
 * scaled by x_i: (G^T x)_j = sum_i G_ij x_i, with i ascending. */
void or_spmv_t(int32_t nrows, int32_t ncols, const int32_t *rp, const int32_t *ci, const double *v,
               const double *x, double *y) {
  for (int32_t j = 0; j < ncols; ++j) y[j] = 0.0;
  for (int32_t i = 0; i < nrows; ++i)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) y[ci[k]] += v[k] * x[i];
}

/* Single-precision products for the mixed-precision path (vectors and
 * accumulation in FP32): the same definitions with float operands, each
 * product and sum rounded to FP32 in the order written. */
void or_spmv_f32(int32_t n, const int32_t *rp, const int32_t *ci, const float *v, const float *x, float *y) {
  for (int32_t i = 0; i < n; ++i) {
    float s = 0.0f;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s += v[k] * x[ci[k]];
    y[i] = s;
  }
}

void or_spmv_t_f32(int32_t nrows, int32_t ncols, const int32_t *rp, const int32_t *ci, const float *v,
                   const float *x, float *y) {
  for (int32_t j = 0; j < ncols; ++j) y[j] = 0.0f;
  for (int32_t i = 0; i < nrows; ++i)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) y[ci[k]] += v[k] * x[i];
}

/* CSR of the transpose by counting: out arrays sized ncols+1 / nnz. */
void or_transpose(int32_t nrows, int32_t ncols, const int32_t *rp, const int32_t *ci, const double *v,
                  int32_t *trp, int32_t *tci, double *tv) {
  for (int32_t j = 0; j <= ncols; ++j) trp[j] = 0;
  for (int32_t k = 0; k < rp[nrows]; ++k) trp[ci[k] + 1]++;
  for (int32_t j = 0; j < ncols; ++j) trp[j + 1] += trp[j];
  int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (ncols > 0 ? ncols : 1));
  for (int32_t j = 0; j < ncols; ++j) pos[j] = trp[j];
  for (int32_t i = 0; i < nrows; ++i)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      int32_t p = pos[ci[k]]++;
      tci[p] = i;
      tv[p] = v[k];
    }
  free(pos);
}

/* ------------------------------------------------- exact inner products */

/*
 * Inner products are the exact value of sum_i a_i b_i rounded once to the
 * nearest double, ties to even (a reading: the paper fixes neither the
 * precision nor the order of its dot products, and the correctly rounded
 * value is the one that does not depend on the order). Every finite double
 * is m 2^e with an integer 0 <= m < 2^53 and -1074 <= e <= 971, so every
 * product of two is an integer below 2^106 times 2^E, -2148 <= E <= 1942.
 * The accumulator is a fixed-point integer whose bit k weighs
 * 2^(k + XA_LSB): limb i holds the 32 bits [32 i, 32 i + 32) as a signed
 * 64-bit count, so each product adds at most 2^33 to a limb and 2^29
 * products fit before carries are propagated. Products with an infinite or
 * NaN factor are tracked apart and give the IEEE result of the sum (NaN,
 * +Inf or -Inf); finite factors are accumulated exactly even where their
 * product exceeds the largest double.
 */
#define XA_LSB (-2304)
#define XA_LIMBS 140 /* weights 2^-2304 .. 2^2175 */
#define XA_SPAN (1L << 29)

typedef struct {
  int64_t d[XA_LIMBS];
  int64_t adds;
  int nan, pinf, ninf;
} xacc;

static void xacc_init(xacc *a) { memset(a, 0, sizeof(*a)); }

/* carries: every limb but the top in [0, 2^32); the top keeps the sign */
static void xacc_carry(xacc *a) {
  for (int i = 0; i < XA_LIMBS - 1; ++i) {
    const int64_t c = a->d[i] >> 32; /* floor(d / 2^32) (gcc: arithmetic shift) */
    a->d[i] -= c * ((int64_t)1 << 32);
    a->d[i + 1] += c;
  }
  a->adds = 0;
}

/* v = (-1)^sign m 2^e for a finite double */
static void split_double(double v, int *sign, uint64_t *m, int *e) {
  uint64_t u;
  memcpy(&u, &v, 8);
  *sign = (int)(u >> 63);
  const int ex = (int)((u >> 52) & 0x7FF);
  const uint64_t fr = u & (((uint64_t)1 << 52) - 1);
  if (ex == 0) {
    *m = fr;
    *e = -1074;
  } else {
    *m = fr | ((uint64_t)1 << 52);
    *e = ex - 1075;
  }
}

/* a += x y, exactly (an infinite or NaN factor: the IEEE product) */
static void xacc_add_prod(xacc *a, double x, double y) {
  if (!isfinite(x) || !isfinite(y)) {
    const double p = x * y;
    if (isnan(p)) a->nan = 1;
    else if (p > 0) a->pinf = 1;
    else a->ninf = 1;
    return;
  }
  int sx, sy, ex, ey;
  uint64_t mx, my;
  split_double(x, &sx, &mx, &ex);
  split_double(y, &sy, &my, &ey);
  if (mx == 0 || my == 0) return;
  const unsigned __int128 P = (unsigned __int128)mx * my; /* < 2^106 */
  const int off = ex + ey - XA_LSB;                        /* >= 156 */
  const int li = off / 32, sh = off % 32;
  const int64_t sg = (sx ^ sy) ? -1 : 1;
  for (int k = 0; k < 4; ++k) {
    const uint64_t c = (uint64_t)(P >> (32 * k)) & 0xFFFFFFFFu; /* digit k of P */
    const uint64_t w = c << sh;                                 /* < 2^63 */
    a->d[li + k] += sg * (int64_t)(w & 0xFFFFFFFFu);
    a->d[li + k + 1] += sg * (int64_t)(w >> 32);
  }
  if (++a->adds >= XA_SPAN) xacc_carry(a);
}

/* a += b, exactly */
static void xacc_merge(xacc *a, const xacc *b) {
  xacc_carry(a);
  xacc t = *b;
  xacc_carry(&t);
  for (int i = 0; i < XA_LIMBS; ++i) a->d[i] += t.d[i];
  a->nan |= t.nan;
  a->pinf |= t.pinf;
  a->ninf |= t.ninf;
  xacc_carry(a);
}

/* the accumulated value rounded to the nearest double, ties to even */
static double xacc_round(const xacc *in) {
  if (in->nan || (in->pinf && in->ninf)) return NAN;
  if (in->pinf) return INFINITY;
  if (in->ninf) return -INFINITY;
  xacc a = *in;
  xacc_carry(&a);
  double sign = 1.0;
  if (a.d[XA_LIMBS - 1] < 0) { /* magnitude of a negative value */
    for (int i = 0; i < XA_LIMBS; ++i) a.d[i] = -a.d[i];
    xacc_carry(&a);
    sign = -1.0;
  }
  int t = XA_LIMBS - 1;
  while (t >= 0 && a.d[t] == 0) --t;
  if (t < 0) return 0.0; /* exactly zero */
  /* the top three limbs as one integer V, its weight 2^E, and whether any
   * lower bit is set (sticky); the top limb is nonzero, so V >= 2^64 */
  unsigned __int128 V = 0;
  for (int i = t; i >= t - 2; --i) V = (V << 32) | (uint64_t)(i >= 0 ? a.d[i] : 0);
  const int E = 32 * (t - 2) + XA_LSB;
  int sticky = 0;
  for (int i = 0; i < t - 2; ++i) sticky |= a.d[i] != 0;
  int L = 0; /* bit length of V */
  for (unsigned __int128 w = V; w; w >>= 1) ++L;
  if (L + E - 1 > 1023) return sign * INFINITY;
  int lsb = L + E - 53; /* weight of the last kept bit */
  if (lsb < -1074) lsb = -1074;
  const int shift = lsb - E; /* >= L - 53 >= 12 */
  uint64_t mant = (uint64_t)(V >> shift);
  const unsigned __int128 rem = V & ((((unsigned __int128)1) << shift) - 1);
  const unsigned __int128 half = ((unsigned __int128)1) << (shift - 1);
  if (rem > half || (rem == half && (sticky || (mant & 1)))) ++mant;
  return sign * ldexp((double)mant, lsb); /* mant <= 2^53: exact, or overflow to Inf */
}

/* ------------------------------------------------------------ vectors */

/* sum_i a_i b_i, exact, rounded once; threads only split the work (each
 * adds its part exactly, the parts are merged exactly), so the result is the
 * same for every thread count */
static double dot(int32_t n, const double *a, const double *b, int threads) {
  xacc acc;
  xacc_init(&acc);
  if (threads <= 1) {
    for (int32_t i = 0; i < n; ++i) xacc_add_prod(&acc, a[i], b[i]);
    return xacc_round(&acc);
  }
#pragma omp parallel num_threads(threads)
  {
    xacc part;
    xacc_init(&part);
#pragma omp for schedule(static)
    for (int32_t i = 0; i < n; ++i) xacc_add_prod(&part, a[i], b[i]);
#pragma omp critical
    xacc_merge(&acc, &part);
  }
  return xacc_round(&acc);
}

double or_dot(int32_t n, const double *a, const double *b) { return dot(n, a, b, 1); }
double or_dot_threads(int32_t n, const double *a, const double *b, int threads) { return dot(n, a, b, threads); }

/* s = G (G^T r) + eps r, with t = G^T r returned too (Eq. "major"). */
static void apply_precond(int32_t n, const int32_t *grp, const int32_t *gci, const double *gv, double eps,
                          const double *r, double *t, double *s, int threads) {
  or_spmv_t(n, n, grp, gci, gv, r, t);
  or_spmv(n, grp, gci, gv, t, s, threads);
#pragma omp parallel for num_threads(threads) schedule(static)
  for (int32_t i = 0; i < n; ++i) s[i] = s[i] + eps * r[i];
}

void or_apply_precond(int32_t n, const int32_t *grp, const int32_t *gci, const double *gv, double eps,
                      const double *r, double *s) {
  double *t = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
  apply_precond(n, grp, gci, gv, eps, r, t, s, 1);
  free(t);
}

/* r = b - A x */
static void residual(int32_t n, const int32_t *arp, const int32_t *aci, const double *av, const double *b,
                     const double *x, double *r, int threads) {
  or_spmv(n, arp, aci, av, x, r, threads);
#pragma omp parallel for num_threads(threads) schedule(static)
  for (int32_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
}

/* ----------------------------------------------------------------- PCG */

typedef struct {
  double eps;      /* shift of M^-1 = G G^T + eps I (absolute units) */
  double tol;      /* relative tolerance on ||b - A x|| / ||b|| (Sec. 4.1 metric) */
  int32_t maxit;   /* i_max of Algorithm 1 */
  int32_t rr_period; /* residual replacement period of Algorithm 1 (50); 0 = never */
  int32_t delta_form; /* 0: delta = r^T s;  1: delta = ||G^T r||^2 + eps ||r||^2 (same value) */
  int32_t stop_rule;  /* 0: ||r|| <= tol ||b||, confirmed on the true residual;
                         1: Algorithm 1's delta_new <= tol^2 delta_0;
                         2: ||r|| <= tol ||b|| on the recurrence alone (the inner
                            solves of iterative refinement, whose FP64 outer
                            residual is the check) */
  int32_t threads;
} or_opts;

typedef struct {
  int32_t status;   /* OR_OK, OR_NOT_CONVERGED, OR_EBREAKDOWN, OR_EINVAL */
  int32_t iters;
  int32_t restarts; /* times the recurrence claimed convergence but the true residual did not */
  int32_t pad;
  double relres_rec;  /* ||r|| / ||b|| of the recurrence residual at exit */
  double relres_true; /* ||b - A x|| / ||b|| at exit */
} or_result;

static int finite(double v) { return isfinite(v); }

static double precond_delta(int32_t n, const double *r, const double *t, const double *s, double eps, int form,
                            int threads) {
  if (form == 0) return dot(n, r, s, threads);
  return dot(n, t, t, threads) + eps * dot(n, r, r, threads);
}

/*
 * Preconditioned CG (Algorithm 1), read as the standard method of the template
 * it cites:
 *   - the "i divisible by 50" branch only chooses how r is formed (recomputed
 *     as b - A x, or updated as r - alpha q); s, delta, beta and d are updated
 *     on every iteration; replacement happens for i > 0 only;
 *   - stopping (stop_rule 0) uses the evaluation metric of Sec. 4.1,
 *     ||r|| <= tol ||b|| on the recurrence residual, checked at the top of the
 *     loop; when it holds, the true residual b - A x is formed; if that fails
 *     the test, r is replaced by it, s and delta are recomputed, d restarts
 *     from s, and the iteration continues;
 *   - x0 is whatever x holds on entry; b = 0 returns x = 0 with 0 iterations.
 * Optional histories: rhist[k] = ||r_k|| (recurrence, k = 0..iters) and
 * xhist[k*n .. k*n+n) = x_k.
 */
int or_pcg(int32_t n, const int32_t *arp, const int32_t *aci, const double *av, const int32_t *grp,
           const int32_t *gci, const double *gv, const double *b, double *x, const or_opts *o, or_result *res,
           double *rhist, double *xhist) {
  memset(res, 0, sizeof(*res));
  if (n < 0 || o->tol < 0 || o->maxit < 0) { res->status = OR_EINVAL; return OR_EINVAL; }
  const int th = o->threads > 0 ? o->threads : 1;
  const double nb = sqrt(dot(n, b, b, th));
  if (nb == 0.0) {
    for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
    if (xhist) memcpy(xhist, x, sizeof(double) * n);
    if (rhist) rhist[0] = 0.0;
    res->status = OR_OK;
    return OR_OK;
  }
  size_t bytes = sizeof(double) * (size_t)n;
  double *r = (double *)malloc(bytes), *t = (double *)malloc(bytes), *s = (double *)malloc(bytes);
  double *d = (double *)malloc(bytes), *q = (double *)malloc(bytes);
  int status = OR_NOT_CONVERGED;
  int32_t i = 0;

  residual(n, arp, aci, av, b, x, r, th);
  apply_precond(n, grp, gci, gv, o->eps, r, t, s, th);
  memcpy(d, s, bytes);
  double delta = precond_delta(n, r, t, s, o->eps, o->delta_form, th);
  const double delta0 = delta;
  double rnorm = sqrt(dot(n, r, r, th));
  if (rhist) rhist[0] = rnorm;
  if (xhist) memcpy(xhist, x, bytes);

  for (;;) {
    if (o->stop_rule == 0) {
      if (rnorm <= o->tol * nb) {
        residual(n, arp, aci, av, b, x, q, th); /* q as scratch: true residual */
        double tn = sqrt(dot(n, q, q, th));
        if (tn <= o->tol * nb) { status = OR_OK; break; }
        /* recurrence drifted: restart from the true residual */
        memcpy(r, q, bytes);
        rnorm = tn;
        apply_precond(n, grp, gci, gv, o->eps, r, t, s, th);
        delta = precond_delta(n, r, t, s, o->eps, o->delta_form, th);
        memcpy(d, s, bytes);
        res->restarts++;
      }
    } else if (o->stop_rule == 1) {
      if (!(delta > o->tol * o->tol * delta0)) { status = OR_OK; break; }
    } else {
      if (rnorm <= o->tol * nb) { status = OR_OK; break; }
    }
    if (i >= o->maxit) break;

    or_spmv(n, arp, aci, av, d, q, th);
    const double gamma = dot(n, d, q, th);
    if (!(gamma > 0.0) || !finite(gamma)) { status = OR_EBREAKDOWN; break; }
    const double alpha = delta / gamma;
#pragma omp parallel for num_threads(th) schedule(static)
    for (int32_t j = 0; j < n; ++j) x[j] = x[j] + alpha * d[j];
    if (o->rr_period > 0 && i > 0 && i % o->rr_period == 0) {
      residual(n, arp, aci, av, b, x, r, th);
    } else {
#pragma omp parallel for num_threads(th) schedule(static)
      for (int32_t j = 0; j < n; ++j) r[j] = r[j] - alpha * q[j];
    }
    rnorm = sqrt(dot(n, r, r, th));
    apply_precond(n, grp, gci, gv, o->eps, r, t, s, th);
    const double delta_old = delta;
    delta = precond_delta(n, r, t, s, o->eps, o->delta_form, th);
    if (!(delta >= 0.0) || !finite(delta)) { status = OR_EBREAKDOWN; i++; break; }
    const double beta = delta / delta_old;
#pragma omp parallel for num_threads(th) schedule(static)
    for (int32_t j = 0; j < n; ++j) d[j] = s[j] + beta * d[j];
    i++;
    if (rhist) rhist[i] = rnorm;
    if (xhist) memcpy(xhist + (size_t)i * n, x, bytes);
  }

  residual(n, arp, aci, av, b, x, q, th);
  res->relres_true = sqrt(dot(n, q, q, th)) / nb;
  res->relres_rec = rnorm / nb;
  res->iters = i;
  res->status = status;
  free(r); free(t); free(s); free(d); free(q);
  return status;
}

/* -------------------------------------------------- preconditioner builders */

/* Entry A_ij of a CSR matrix with sorted columns, or 0 (binary search). */
static double csr_get(const int32_t *rp, const int32_t *ci, const double *v, int32_t i, int32_t j) {
  int32_t lo = rp[i], hi = rp[i + 1];
  while (lo < hi) {
    const int32_t mid = lo + (hi - lo) / 2;
    if (ci[mid] < j) lo = mid + 1;
    else hi = mid;
  }
  return (lo < rp[i + 1] && ci[lo] == j) ? v[lo] : 0.0;
}

/* Number of entries with column <= row: the size of tril(A)'s pattern. */
int64_t or_tril_nnz(int32_t n, const int32_t *rp, const int32_t *ci) {
  int64_t c = 0;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] <= i) c++;
  return c;
}

/*
 * Classic factorized sparse approximate inverse (FSAI, Kolotilina and
 * Yeremin 1993, cited by the paper as a factorized SPAI): a lower-triangular
 * G_L on the pattern of tril(A) such that A^-1 ~ G_L^T G_L. For row i with
 * J = { j <= i : A_ij != 0 } (ascending, so i is last), solve A[J,J] y = e_i
 * by dense Cholesky and set row i of G_L on J to y / sqrt(y_i).
 * Output arrays are sized n+1 / or_tril_nnz. Returns OR_OK, or OR_EBREAKDOWN
 * when a local matrix is not positive definite (OR_EINVAL: no diagonal).
 * Rows are independent; `threads` only splits them (same result).
 */
static int fsai_row(int32_t i, const int32_t *rp, const int32_t *ci, const double *v, int32_t *gci, double *gv,
                    int32_t *J, double *S, double *y) {
  int m = 0;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
    if (ci[k] <= i) J[m++] = ci[k];
  if (m == 0 || J[m - 1] != i) return OR_EINVAL;
  for (int a = 0; a < m; ++a)
    for (int c = 0; c < m; ++c) S[a * m + c] = csr_get(rp, ci, v, J[a], J[c]);
  /* Cholesky S = L L^T, L stored in the lower triangle of S */
  for (int c = 0; c < m; ++c) {
    double dsum = S[c * m + c];
    for (int k = 0; k < c; ++k) dsum -= S[c * m + k] * S[c * m + k];
    if (!(dsum > 0.0)) return OR_EBREAKDOWN;
    double l = sqrt(dsum);
    S[c * m + c] = l;
    for (int a = c + 1; a < m; ++a) {
      double e = S[a * m + c];
      for (int k = 0; k < c; ++k) e -= S[a * m + k] * S[c * m + k];
      S[a * m + c] = e / l;
    }
  }
  /* forward: L z = e_last ; backward: L^T y = z */
  for (int a = 0; a < m; ++a) {
    double e = (a == m - 1) ? 1.0 : 0.0;
    for (int k = 0; k < a; ++k) e -= S[a * m + k] * y[k];
    y[a] = e / S[a * m + a];
  }
  for (int a = m - 1; a >= 0; --a) {
    double e = y[a];
    for (int k = a + 1; k < m; ++k) e -= S[k * m + a] * y[k];
    y[a] = e / S[a * m + a];
  }
  if (!(y[m - 1] > 0.0)) return OR_EBREAKDOWN;
  const double sc = sqrt(y[m - 1]);
  for (int a = 0; a < m; ++a) {
    gci[a] = J[a];
    gv[a] = y[a] / sc;
  }
  return OR_OK;
}

int or_fsai_lower(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t *grp, int32_t *gci,
                  double *gv, int threads) {
  int32_t mmax = 1;
  grp[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    int32_t m = 0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] <= i) m++;
    if (m > mmax) mmax = m;
    grp[i + 1] = grp[i] + m;
  }
  int rc = OR_OK;
#pragma omp parallel num_threads(threads > 0 ? threads : 1)
  {
    int32_t *J = (int32_t *)malloc(sizeof(int32_t) * mmax);
    double *S = (double *)malloc(sizeof(double) * (size_t)mmax * mmax);
    double *y = (double *)malloc(sizeof(double) * mmax);
    int my = OR_OK;
#pragma omp for schedule(dynamic, 256)
    for (int32_t i = 0; i < n; ++i) {
      const int r = fsai_row(i, rp, ci, v, gci + grp[i], gv + grp[i], J, S, y);
      if (r != OR_OK && my == OR_OK) my = r;
    }
#pragma omp critical
    if (my != OR_OK && rc == OR_OK) rc = my;
    free(J); free(S); free(y);
  }
  return rc;
}

/*
 * Block FSAI for systems with b unknowns per node (the paper's blocked
 * systems, Sec. 3.1, whose learned G carries one b x b block per nonzero
 * block of A, Sec. 3.2.2). A must be exactly b x b blocked: n = b N and the b
 * rows of block row I store the same complete column blocks. G_L is block
 * lower triangular on the block pattern of tril(A), every block full (zeros
 * included), with A^-1 ~ G_L^T G_L:
 *   for block row I with block columns J = { J <= I : A_IJ != 0 } (I last),
 *   solve A[J,J] X = E (E: the last b columns of the identity of size b|J|)
 *   by dense Cholesky; with X_II = C C^T (C lower, the Cholesky factor of
 *   X's last b x b block), block row I of G_L is C^-1 X^T.
 * Then each diagonal block of G_L A G_L^T is the identity, and
 * G_L^T G_L = sum_I X X_II^-1 X^T does not depend on the choice of C. With
 * b = 1 this is the scalar FSAI above. Output: CSR sized n+1 / b^2 times the
 * block count of tril (rows of a block row list the same columns).
 */
static int bfsai_blockrow(int32_t I, int b, const int32_t *rp, const int32_t *ci, const double *v, int32_t *gci,
                          double *gv, int32_t rowlen, int32_t *J, double *S, double *X, double *C) {
  const int32_t r = b * I;
  int m = 0; /* block columns of the tril part of block row I */
  for (int32_t k = rp[r]; k < rp[r + 1]; k += b)
    if (ci[k] / b <= I) J[m++] = ci[k] / b;
  if (m == 0 || J[m - 1] != I) return OR_EINVAL;
  const int M = b * m;
  for (int a = 0; a < M; ++a)
    for (int c = 0; c < M; ++c) S[a * M + c] = csr_get(rp, ci, v, b * J[a / b] + a % b, b * J[c / b] + c % b);
  for (int c = 0; c < M; ++c) { /* S = L L^T, L in the lower triangle */
    double dsum = S[c * M + c];
    for (int k = 0; k < c; ++k) dsum -= S[c * M + k] * S[c * M + k];
    if (!(dsum > 0.0)) return OR_EBREAKDOWN;
    const double l = sqrt(dsum);
    S[c * M + c] = l;
    for (int a = c + 1; a < M; ++a) {
      double e = S[a * M + c];
      for (int k = 0; k < c; ++k) e -= S[a * M + k] * S[c * M + k];
      S[a * M + c] = e / l;
    }
  }
  for (int q = 0; q < b; ++q) { /* column q of X: L z = e_(M-b+q), L^T x = z */
    double *x = X + (size_t)q * M;
    for (int a = 0; a < M; ++a) {
      double e = (a == M - b + q) ? 1.0 : 0.0;
      for (int k = 0; k < a; ++k) e -= S[a * M + k] * x[k];
      x[a] = e / S[a * M + a];
    }
    for (int a = M - 1; a >= 0; --a) {
      double e = x[a];
      for (int k = a + 1; k < M; ++k) e -= S[k * M + a] * x[k];
      x[a] = e / S[a * M + a];
    }
  }
  for (int p = 0; p < b; ++p) /* X_II = C C^T (C lower) */
    for (int q = 0; q <= p; ++q) {
      double e = X[(size_t)q * M + M - b + p];
      for (int k = 0; k < q; ++k) e -= C[p * b + k] * C[q * b + k];
      if (p == q) {
        if (!(e > 0.0)) return OR_EBREAKDOWN;
        C[p * b + p] = sqrt(e);
      } else {
        C[p * b + q] = e / C[q * b + q];
      }
    }
  for (int a = 0; a < M; ++a) /* W = C^-1 X^T, column a by forward substitution */
    for (int p = 0; p < b; ++p) {
      double e = X[(size_t)p * M + a];
      for (int k = 0; k < p; ++k) e -= C[p * b + k] * gv[(size_t)k * rowlen + a];
      gv[(size_t)p * rowlen + a] = e / C[p * b + p];
    }
  for (int p = 0; p < b; ++p)
    for (int a = 0; a < M; ++a) gci[(size_t)p * rowlen + a] = b * J[a / b] + a % b;
  return OR_OK;
}

/* Row pointers of the block FSAI's pattern (b^2 per tril block); -1 when A
 * is not exactly b x b blocked. */
int64_t or_bfsai_pattern(int32_t n, const int32_t *rp, const int32_t *ci, int b, int32_t *grp) {
  if (b < 1 || n % b) return -1;
  grp[0] = 0;
  for (int32_t I = 0; I < n / b; ++I) {
    const int32_t r = b * I, len = rp[r + 1] - rp[r];
    if (len % b) return -1;
    int32_t m = 0;
    for (int s = 0; s < b; ++s) {
      if (rp[r + s + 1] - rp[r + s] != len) return -1;
      for (int32_t k = 0; k < len; k += b) {
        const int32_t c0 = ci[rp[r + s] + k];
        if (c0 % b) return -1;
        for (int j = 0; j < b; ++j)
          if (ci[rp[r + s] + k + j] != c0 + j || ci[rp[r] + k + j] != c0 + j) return -1;
        if (s == 0 && c0 / b <= I) m++;
      }
    }
    for (int s = 0; s < b; ++s) grp[r + s + 1] = grp[r + s] + b * m;
  }
  return grp[n];
}

int or_fsai_block_lower(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int b, const int32_t *grp,
                        int32_t *gci, double *gv, int threads) {
  int32_t mmax = 1;
  for (int32_t I = 0; I < n / b; ++I) {
    const int32_t m = (grp[b * I + 1] - grp[b * I]) / b;
    if (m > mmax) mmax = m;
  }
  const int Mx = b * mmax;
  int rc = OR_OK;
#pragma omp parallel num_threads(threads > 0 ? threads : 1)
  {
    int32_t *J = (int32_t *)malloc(sizeof(int32_t) * mmax);
    double *S = (double *)malloc(sizeof(double) * (size_t)Mx * Mx);
    double *X = (double *)malloc(sizeof(double) * (size_t)Mx * b);
    double *C = (double *)malloc(sizeof(double) * (size_t)b * b);
    int my = OR_OK;
#pragma omp for schedule(dynamic, 64)
    for (int32_t I = 0; I < n / b; ++I) {
      const int32_t r = b * I, rowlen = grp[r + 1] - grp[r];
      const int e = bfsai_blockrow(I, b, rp, ci, v, gci + grp[r], gv + grp[r], rowlen, J, S, X, C);
      if (e != OR_OK && my == OR_OK) my = e;
    }
#pragma omp critical
    if (my != OR_OK && rc == OR_OK) rc = my;
    free(J); free(S); free(X); free(C);
  }
  return rc;
}

/*
 * The fixed lower-triangular G of the small 2D Poisson workload: on tril(A)'s
 * pattern, G_ii = 1/sqrt(A_ii) and G_ij = -0.25 A_ij / sqrt(A_ii A_jj) for
 * j < i. Output arrays sized n+1 / or_tril_nnz.
 */
int or_g_cfg1(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t *grp, int32_t *gci,
              double *gv) {
  double *dg = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
  for (int32_t i = 0; i < n; ++i) {
    dg[i] = csr_get(rp, ci, v, i, i);
    if (!(dg[i] > 0.0)) { free(dg); return OR_EINVAL; }
  }
  int64_t p = 0;
  grp[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      int32_t j = ci[k];
      if (j > i) continue;
      gci[p] = j;
      gv[p] = (j == i) ? 1.0 / sqrt(dg[i]) : -0.25 * v[k] / sqrt(dg[i] * dg[j]);
      p++;
    }
    grp[i + 1] = (int32_t)p;
  }
  free(dg);
  return OR_OK;
}

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
