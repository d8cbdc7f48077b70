/*
 * Seeded synthetic input generators for the preconditioned-CG path.
 *
 * This module produces the linear systems (A, b) and the random draws that the
 * workloads need. It contains none of the solver's arithmetic: no SpMV, no CG,
 * no preconditioner construction. Both the HIP library's tests and the FP64
 * oracle take their inputs from here, so it is the only code they share.
 *
 * Random numbers: one counter-based generator built on SplitMix64 (Steele,
 * Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA
 * 2014). The i-th draw of stream `stream` under seed `seed` is the (i+1)-th
 * output of a SplitMix64 sequence whose initial state is
 *     key(seed, stream) = mix(mix(seed + GAMMA) + (stream + 1) * GAMMA),
 * i.e. bits(seed, stream, i) = mix(key + (i + 1) * GAMMA), with mix() the
 * SplitMix64 output finaliser and GAMMA = 0x9E3779B97F4A7C15. Draws do not
 * depend on evaluation order or threading.
 *   u01(i)    = ((bits >> 11) + 1) * 2^-53, in (0, 1]
 *   normal(i) = sqrt(-2 ln u01(2i)) * cos(2 pi u01(2i+1))   (Box-Muller)
 *
 * Matrices are CSR with int32 row pointers and int32 column indices, columns
 * sorted ascending and unique within each row, FP64 values, diagonal present.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GEN_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t gen_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t gen_key(uint64_t seed, uint64_t stream) {
  return gen_mix(gen_mix(seed + GEN_GAMMA) + (stream + 1) * GEN_GAMMA);
}

uint64_t gen_bits(uint64_t seed, uint64_t stream, uint64_t i) {
  return gen_mix(gen_key(seed, stream) + (i + 1) * GEN_GAMMA);
}

static inline double u01_k(uint64_t key, uint64_t i) {
  uint64_t v = gen_mix(key + (i + 1) * GEN_GAMMA);
  return (double)((v >> 11) + 1) * 0x1.0p-53;
}

static inline double normal_k(uint64_t key, uint64_t i) {
  double u1 = u01_k(key, 2 * i), u2 = u01_k(key, 2 * i + 1);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925287 * u2);
}

double gen_u01(uint64_t seed, uint64_t stream, uint64_t i) { return u01_k(gen_key(seed, stream), i); }
double gen_normal(uint64_t seed, uint64_t stream, uint64_t i) { return normal_k(gen_key(seed, stream), i); }

void gen_u01_vec(uint64_t seed, uint64_t stream, int64_t n, double *out) {
  uint64_t key = gen_key(seed, stream);
  for (int64_t i = 0; i < n; ++i) out[i] = u01_k(key, (uint64_t)i);
}

/* Draws at arbitrary indices: out[k] = u01(seed, stream, idx[k]). */
void gen_u01_at(uint64_t seed, uint64_t stream, int64_t n, const uint64_t *idx, double *out) {
  uint64_t key = gen_key(seed, stream);
  for (int64_t k = 0; k < n; ++k) out[k] = u01_k(key, idx[k]);
}

void gen_normal_vec(uint64_t seed, uint64_t stream, int64_t n, double *out) {
  uint64_t key = gen_key(seed, stream);
  for (int64_t i = 0; i < n; ++i) out[i] = normal_k(key, (uint64_t)i);
}

/* ------------------------------------------------------------------------ */
/* Poisson on a d-dimensional grid (d = 2 or 3), N interior points per side, */
/* Dirichlet boundary eliminated, lexicographic x-fastest ordering, no h^2   */
/* scaling. Every cell face f carries a coefficient k_f = exp(sigma * Z_f),  */
/* Z_f ~ N(0,1) from stream `coef_stream` at the face id below; faces to the */
/* boundary exist too and only add to the diagonal. A_ij = -k_f for the face */
/* between i and j, A_ii = sum of the 2d faces around i. sigma = 0 gives the */
/* constant stencil (A_ii = 2d, A_ij = -1).                                  */
/* Face ids (axis a, face coordinate fa in [0, N], others in [0, N)):        */
/*   x-faces: fx + (N+1)*(y + N*z)                                           */
/*   y-faces: off_y + x + N*(fy + (N+1)*z),  off_y = (N+1)*N^(d-1)           */
/*   z-faces: off_z + x + N*(y + N*fz),      off_z = 2*(N+1)*N^2             */
/* ------------------------------------------------------------------------ */

int64_t gen_poisson_nnz(int dim, int64_t N) {
  if (dim == 2) return 5 * N * N - 4 * N;
  return 7 * N * N * N - 6 * N * N;
}

static inline double face_coef(uint64_t key, double sigma, uint64_t id) {
  if (sigma == 0.0) return 1.0;
  return exp(sigma * normal_k(key, id));
}

/* Returns nnz, or -1 on bad arguments. Arrays are caller-allocated with
 * n+1 / nnz entries (n = N^dim, nnz = gen_poisson_nnz). */
int64_t gen_poisson(int dim, int64_t N, double sigma, uint64_t seed, uint64_t coef_stream,
                    int32_t *rowptr, int32_t *col, double *val) {
  if ((dim != 2 && dim != 3) || N < 1) return -1;
  uint64_t key = gen_key(seed, coef_stream);
  const int64_t Nz = (dim == 3) ? N : 1;
  const int64_t n = N * N * Nz;
  const uint64_t offy = (uint64_t)((N + 1) * N * Nz);
  const uint64_t offz = (uint64_t)(2 * (N + 1) * N * N);
  int64_t k = 0;
  rowptr[0] = 0;
  for (int64_t z = 0; z < Nz; ++z)
    for (int64_t y = 0; y < N; ++y)
      for (int64_t x = 0; x < N; ++x) {
        const int64_t i = x + N * (y + N * z);
        /* faces: lower/upper in each axis */
        double kxl = face_coef(key, sigma, (uint64_t)(x + (N + 1) * (y + N * z)));
        double kxu = face_coef(key, sigma, (uint64_t)(x + 1 + (N + 1) * (y + N * z)));
        double kyl = face_coef(key, sigma, offy + (uint64_t)(x + N * (y + (N + 1) * z)));
        double kyu = face_coef(key, sigma, offy + (uint64_t)(x + N * (y + 1 + (N + 1) * z)));
        double kzl = 0.0, kzu = 0.0;
        if (dim == 3) {
          kzl = face_coef(key, sigma, offz + (uint64_t)(x + N * (y + N * z)));
          kzu = face_coef(key, sigma, offz + (uint64_t)(x + N * (y + N * (z + 1))));
        }
        double diag = kxl + kxu + kyl + kyu;
        if (dim == 3) diag += kzl + kzu;
        if (dim == 3 && z > 0) { col[k] = (int32_t)(i - N * N); val[k++] = -kzl; }
        if (y > 0) { col[k] = (int32_t)(i - N); val[k++] = -kyl; }
        if (x > 0) { col[k] = (int32_t)(i - 1); val[k++] = -kxl; }
        col[k] = (int32_t)i; val[k++] = diag;
        if (x < N - 1) { col[k] = (int32_t)(i + 1); val[k++] = -kxu; }
        if (y < N - 1) { col[k] = (int32_t)(i + N); val[k++] = -kyu; }
        if (dim == 3 && z < N - 1) { col[k] = (int32_t)(i + N * N); val[k++] = -kzu; }
        rowptr[i + 1] = (int32_t)k;
      }
  (void)n;
  return k;
}

/* ------------------------------------------------------------------------ */
/* Random geometric graph Laplacian plus diagonal shift.                     */
/* n points uniform in the unit square (stream `pts_stream`: x = u(2k),      */
/* y = u(2k+1)); an edge joins points closer than r = sqrt(8/(pi (n-1))), so */
/* the expected degree away from the boundary is 8; its weight is            */
/* 0.1 + 9.9 u(min(k,m) * n + max(k,m)) from stream `w_stream` (original     */
/* point ids, so the matrix is symmetric). A = D - W + shift * I. Nodes are  */
/* renumbered by grid cell (cells of side >= r, row-major), ties by point id,*/
/* for locality. Output arrays are malloc'ed; release with gen_free.         */
/* ------------------------------------------------------------------------ */
int64_t gen_rgg_laplacian(int64_t n, double shift, uint64_t seed, uint64_t pts_stream, uint64_t w_stream,
                          int32_t **rowptr_out, int32_t **col_out, double **val_out) {
  if (n < 2) return -1;
  uint64_t kp = gen_key(seed, pts_stream), kw = gen_key(seed, w_stream);
  double *px = (double *)malloc(sizeof(double) * n), *py = (double *)malloc(sizeof(double) * n);
  for (int64_t k = 0; k < n; ++k) { px[k] = u01_k(kp, 2 * k); py[k] = u01_k(kp, 2 * k + 1); }
  const double r = sqrt(8.0 / (3.14159265358979323846 * (double)(n - 1)));
  const double r2 = r * r;
  int64_t nc = (int64_t)floor(1.0 / r);
  if (nc < 1) nc = 1;
  const int64_t ncell = nc * nc;
  int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * n);
  int64_t *cstart = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  for (int64_t k = 0; k < n; ++k) {
    int64_t cx = (int64_t)(px[k] * nc), cy = (int64_t)(py[k] * nc);
    if (cx >= nc) cx = nc - 1;
    if (cy >= nc) cy = nc - 1;
    cell[k] = cx + nc * cy;
    cstart[cell[k] + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
  int64_t *order = (int64_t *)malloc(sizeof(int64_t) * n); /* new index -> point id */
  int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * n);  /* point id -> new index */
  {
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ncell);
    memcpy(fill, cstart, sizeof(int64_t) * ncell);
    for (int64_t k = 0; k < n; ++k) { order[fill[cell[k]]] = k; perm[k] = fill[cell[k]]++; }
    free(fill);
  }
  /* two passes over the neighbour search: count, then fill */
  int32_t *rowptr = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
  rowptr[0] = 0;
  for (int pass = 0; pass < 2; ++pass) {
    int32_t *col = pass ? *col_out : NULL;
    double *val = pass ? *val_out : NULL;
    int64_t cap = 64, *nb = (int64_t *)malloc(sizeof(int64_t) * cap);
    double *nw = (double *)malloc(sizeof(double) * cap);
    for (int64_t i = 0; i < n; ++i) {
      int64_t k = order[i];
      int64_t cx = cell[k] % nc, cy = cell[k] / nc, cnt = 0;
      double wsum = 0.0;
      for (int64_t yy = cy - 1; yy <= cy + 1; ++yy)
        for (int64_t xx = cx - 1; xx <= cx + 1; ++xx) {
          if (xx < 0 || yy < 0 || xx >= nc || yy >= nc) continue;
          int64_t c = xx + nc * yy;
          for (int64_t t = cstart[c]; t < cstart[c + 1]; ++t) {
            int64_t m = order[t];
            if (m == k) continue;
            double dx = px[m] - px[k], dy = py[m] - py[k];
            if (dx * dx + dy * dy >= r2) continue;
            if (cnt == cap) {
              cap *= 2;
              nb = (int64_t *)realloc(nb, sizeof(int64_t) * cap);
              nw = (double *)realloc(nw, sizeof(double) * cap);
            }
            int64_t lo = k < m ? k : m, hi = k < m ? m : k;
            double w = 0.1 + 9.9 * u01_k(kw, (uint64_t)lo * (uint64_t)n + (uint64_t)hi);
            nb[cnt] = perm[m]; nw[cnt] = w; cnt++;
          }
        }
      if (!pass) { rowptr[i + 1] = rowptr[i] + (int32_t)(cnt + 1); continue; }
      /* insertion sort of the row by new column index; add the diagonal */
      for (int64_t a = 1; a < cnt; ++a) {
        int64_t cb = nb[a]; double cw = nw[a]; int64_t b = a - 1;
        while (b >= 0 && nb[b] > cb) { nb[b + 1] = nb[b]; nw[b + 1] = nw[b]; --b; }
        nb[b + 1] = cb; nw[b + 1] = cw;
      }
      for (int64_t a = 0; a < cnt; ++a) wsum += nw[a];
      int64_t p = rowptr[i];
      int diag_done = 0;
      for (int64_t a = 0; a < cnt; ++a) {
        if (!diag_done && nb[a] > i) { col[p] = (int32_t)i; val[p++] = wsum + shift; diag_done = 1; }
        col[p] = (int32_t)nb[a]; val[p++] = -nw[a];
      }
      if (!diag_done) { col[p] = (int32_t)i; val[p++] = wsum + shift; }
    }
    free(nb); free(nw);
    if (!pass) {
      *col_out = (int32_t *)malloc(sizeof(int32_t) * (size_t)rowptr[n]);
      *val_out = (double *)malloc(sizeof(double) * (size_t)rowptr[n]);
    }
  }
  *rowptr_out = rowptr;
  free(px); free(py); free(cell); free(cstart); free(order); free(perm);
  return rowptr[n];
}

void gen_free(void *p) { free(p); }

/* ------------------------------------------------------------------------ */
/* Linear-elasticity-like block system: trilinear (Q1) hexahedral finite     */
/* elements on the unit cube, (N+1)^3 elements of side h = 1/(N+1), all      */
/* boundary nodes clamped, leaving N^3 free nodes with 3 dof each, ordered   */
/* node-major (lexicographic x-fastest) and dof-minor. Isotropic material    */
/* with Poisson ratio nu; each element's Young's modulus is exp(sigma Z_e),  */
/* Z_e ~ N(0,1) from stream `e_stream` at element id ex + (N+1)(ey + (N+1)ez)*/
/* Element stiffness by 2x2x2 Gauss quadrature. Every free node couples to   */
/* the free nodes of its 3x3x3 neighbourhood: nnz = 9 (3N-2)^3.              */
/* ------------------------------------------------------------------------ */

/* Reference element stiffness for E = 1 (24 x 24, local node a = ax+2ay+4az,
 * dof-minor), on a cube of side h. */
static void q1_ref_stiffness(double nu, double h, double K[24][24]) {
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  double D[6][6] = {{0}};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) D[a][b] = lam + (a == b ? 2.0 * mu : 0.0);
  D[3][3] = D[4][4] = D[5][5] = mu;
  memset(K, 0, sizeof(double) * 24 * 24);
  const double g = 1.0 / sqrt(3.0);
  const double detJ = (h / 2) * (h / 2) * (h / 2);
  for (int q = 0; q < 8; ++q) {
    double xi[3] = {(q & 1) ? g : -g, (q & 2) ? g : -g, (q & 4) ? g : -g};
    double dN[8][3];
    for (int a = 0; a < 8; ++a) {
      double s[3] = {(a & 1) ? 1.0 : -1.0, (a & 2) ? 1.0 : -1.0, (a & 4) ? 1.0 : -1.0};
      for (int d = 0; d < 3; ++d) {
        double p = s[d] / 2.0;
        for (int e = 0; e < 3; ++e)
          if (e != d) p *= (1.0 + s[e] * xi[e]) / 2.0;
        dN[a][d] = p * (2.0 / h);
      }
    }
    double B[6][24] = {{0}};
    for (int a = 0; a < 8; ++a) {
      B[0][3 * a + 0] = dN[a][0];
      B[1][3 * a + 1] = dN[a][1];
      B[2][3 * a + 2] = dN[a][2];
      B[3][3 * a + 0] = dN[a][1]; B[3][3 * a + 1] = dN[a][0];
      B[4][3 * a + 1] = dN[a][2]; B[4][3 * a + 2] = dN[a][1];
      B[5][3 * a + 0] = dN[a][2]; B[5][3 * a + 2] = dN[a][0];
    }
    double DB[6][24];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 24; ++j) {
        double s = 0.0;
        for (int k = 0; k < 6; ++k) s += D[i][k] * B[k][j];
        DB[i][j] = s;
      }
    for (int i = 0; i < 24; ++i)
      for (int j = 0; j < 24; ++j) {
        double s = 0.0;
        for (int k = 0; k < 6; ++k) s += B[k][i] * DB[k][j];
        K[i][j] += s * detJ;
      }
  }
}

int64_t gen_elasticity_nnz(int64_t N) { int64_t m = 3 * N - 2; return 9 * m * m * m; }

int64_t gen_elasticity(int64_t N, double sigma, double nu, uint64_t seed, uint64_t e_stream,
                       int32_t *rowptr, int32_t *col, double *val) {
  if (N < 1 || !(nu > -1.0 && nu < 0.5)) return -1;
  static double K[24][24];
  const int64_t M = N + 1; /* elements per side; nodes per side N + 2 */
  const double h = 1.0 / (double)M;
  q1_ref_stiffness(nu, h, K);
  uint64_t key = gen_key(seed, e_stream);
  double *E = (double *)malloc(sizeof(double) * M * M * M);
  for (int64_t e = 0; e < M * M * M; ++e) E[e] = (sigma == 0.0) ? 1.0 : exp(sigma * normal_k(key, (uint64_t)e));
  int64_t k = 0;
  rowptr[0] = 0;
  for (int64_t zi = 1; zi <= N; ++zi)
    for (int64_t yi = 1; yi <= N; ++yi)
      for (int64_t xi = 1; xi <= N; ++xi) {
        const int64_t ni = (xi - 1) + N * ((yi - 1) + N * (zi - 1));
        for (int c = 0; c < 3; ++c) {
          for (int64_t dz = -1; dz <= 1; ++dz)
            for (int64_t dy = -1; dy <= 1; ++dy)
              for (int64_t dx = -1; dx <= 1; ++dx) {
                int64_t xj = xi + dx, yj = yi + dy, zj = zi + dz;
                if (xj < 1 || yj < 1 || zj < 1 || xj > N || yj > N || zj > N) continue;
                const int64_t nj = (xj - 1) + N * ((yj - 1) + N * (zj - 1));
                double blk[3] = {0.0, 0.0, 0.0};
                int64_t ex0 = (xi > xj ? xi : xj) - 1, ex1 = (xi < xj ? xi : xj);
                int64_t ey0 = (yi > yj ? yi : yj) - 1, ey1 = (yi < yj ? yi : yj);
                int64_t ez0 = (zi > zj ? zi : zj) - 1, ez1 = (zi < zj ? zi : zj);
                for (int64_t ez = ez0; ez <= ez1; ++ez)
                  for (int64_t ey = ey0; ey <= ey1; ++ey)
                    for (int64_t ex = ex0; ex <= ex1; ++ex) {
                      int li = (int)((xi - ex) + 2 * (yi - ey) + 4 * (zi - ez));
                      int lj = (int)((xj - ex) + 2 * (yj - ey) + 4 * (zj - ez));
                      double Ee = E[ex + M * (ey + M * ez)];
                      for (int cc = 0; cc < 3; ++cc) blk[cc] += Ee * K[3 * li + c][3 * lj + cc];
                    }
                for (int cc = 0; cc < 3; ++cc) { col[k] = (int32_t)(3 * nj + cc); val[k++] = blk[cc]; }
              }
          rowptr[3 * ni + c + 1] = (int32_t)k;
        }
      }
  free(E);
  return k;
}
