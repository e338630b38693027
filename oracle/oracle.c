/* FP64 CPU oracle of the SPH hot path (paper Sec. 2.1, Sec. 3.2, Sec. 4).
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path. It shares
 * no code, header, table or constant with the HIP library.
 *
 * Everything here is the plain definition, written for a reader to check by
 * eye: every neighbour sum is taken over an explicit, ascending list of
 * neighbour indices, so the brute-force and cell-list modes produce
 * bit-identical results (the cell list only restricts candidates).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math, no
 * contraction: every expression rounds as written).
 *
 * Readings where the paper is silent (listed in the design notes):
 *  - kernel: cubic-spline M4 with support radius H = gamma_k h (Sec. 2.1
 *    names the cubic spline; gamma_k = 1.825742 makes (4 pi/3)(gamma_k eta)^3
 *    about 48 neighbours at eta = 1.2348).
 *  - h_ij: density uses h_i (gather); the force uses the grad-h form with
 *    separate W(h_i) and W(h_j) terms; gradh = 0 with uniform h reduces it to
 *    the momentum equation of Sec. 2.1 as printed.
 *  - the momentum equation's "grad rho / rho" is read as "grad P / rho".
 *  - viscosity: signal-velocity artificial viscosity, no limiter.
 *  - the self pair is in the density sums and out of the force sums.
 *  - support test is strict: r < H.
 *  - a pair at zero separation with j != i (coincident stored positions)
 *    has the zero vector as its direction: it counts, exerts no force and
 *    its signal velocity is c_i + c_j.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Kernel (Sec. 2.1: cubic spline, compact support)                          */
/* ------------------------------------------------------------------------ */

/* Normalised 3D kernels on the unit support, u = r / H (Sec. 2.1 names the
 * cubic spline and Wendland families): kernel ORC_KERNEL_M4, the M4 cubic
 * spline; ORC_KERNEL_WENDLAND_C2, the Wendland C2 function
 * (21 / 2 pi) (1 - u)^4 (1 + 4 u). */
double orc_kernel_w(int kernel, double u) {
  if (!(u < 1.0)) return 0.0;
  double t = 1.0 - u;
  if (kernel == ORC_KERNEL_WENDLAND_C2) return (21.0 / (2.0 * ORC_PI)) * t * t * t * t * (1.0 + 4.0 * u);
  if (u < 0.5) return (8.0 / ORC_PI) * (1.0 - 6.0 * u * u + 6.0 * u * u * u);
  return (16.0 / ORC_PI) * t * t * t;
}

/* d(w_hat)/du */
double orc_kernel_dw(int kernel, double u) {
  if (!(u < 1.0)) return 0.0;
  double t = 1.0 - u;
  if (kernel == ORC_KERNEL_WENDLAND_C2) return -(210.0 / ORC_PI) * u * t * t * t;
  if (u < 0.5) return (8.0 / ORC_PI) * (-12.0 * u + 18.0 * u * u);
  return -(48.0 / ORC_PI) * t * t;
}

double orc_w_hat(double u) { return orc_kernel_w(ORC_KERNEL_M4, u); }
double orc_dw_hat(double u) { return orc_kernel_dw(ORC_KERNEL_M4, u); }

/* W(r, h) = w_hat(r / H) / H^3 with H = gamma_k h (Eq. interpolant, Eq. density) */
double orc_W(double r, double h, double gamma_k) { return orc_W_k(ORC_KERNEL_M4, r, h, gamma_k); }
double orc_W_k(int kernel, double r, double h, double gamma_k) {
  double H = gamma_k * h;
  return orc_kernel_w(kernel, r / H) / (H * H * H);
}

/* dW/dh at fixed r: -gamma_k (3 w_hat(u) + u w_hat'(u)) / H^4 */
double orc_dWdh(double r, double h, double gamma_k) { return orc_dWdh_k(ORC_KERNEL_M4, r, h, gamma_k); }
double orc_dWdh_k(int kernel, double r, double h, double gamma_k) {
  double H = gamma_k * h;
  double u = r / H;
  return -gamma_k * (3.0 * orc_kernel_w(kernel, u) + u * orc_kernel_dw(kernel, u)) / (H * H * H * H);
}

/* |grad_i W(r_ij, h)| along e_ij = (x_i - x_j)/r: w_hat'(u) / H^4 (Eq. gradient) */
static double orc_gradW(int kernel, double r, double h, double gamma_k) {
  double H = gamma_k * h;
  if (!(r < H)) return 0.0;
  return orc_kernel_dw(kernel, r / H) / (H * H * H * H);
}

/* ------------------------------------------------------------------------ */
/* Binning (the cell list of Sec. 2.2's spatial search structures)           */
/* ------------------------------------------------------------------------ */

static int cell_axis(double xw, int n_c) {
  double t = floor(xw * (double)n_c);
  int c = (t != t) ? 0 : (int)t;          /* NaN -> 0: inputs are validated */
  if (c > n_c - 1) c = n_c - 1;
  if (c < 0) c = 0;
  return c;
}

/* wrap into the periodic unit box */
static double wrap01(double x) { return x - floor(x); }

/* cell[i]: linear cell id cx + n_c (cy + n_c cz) of particle i (input order);
 * cell_start[C+1], perm[N]: particles of cell c are perm[cell_start[c] ..
 * cell_start[c+1]-1], in increasing input index; off[3i+k]: x_k - c_k / n_c
 * in FP64 after wrapping. Any output pointer may be NULL. */
int orc_bin(int n, const double *x, int n_c, int32_t *cell, int32_t *cell_start,
            int32_t *perm, double *off) {
  if (n < 0 || n_c < 1) return -1;
  int C = n_c * n_c * n_c;
  int32_t *cid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t *start = (int32_t *)calloc((size_t)C + 1, sizeof(int32_t));
  for (int i = 0; i < n; ++i) {
    int cc[3];
    for (int k = 0; k < 3; ++k) {
      double xw = wrap01(x[3 * i + k]);
      cc[k] = cell_axis(xw, n_c);
      if (off) off[3 * i + k] = xw - (double)cc[k] / (double)n_c;
    }
    cid[i] = cc[0] + n_c * (cc[1] + n_c * cc[2]);
    start[cid[i] + 1] += 1;
  }
  for (int c = 0; c < C; ++c) start[c + 1] += start[c];
  if (perm) {
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)C);
    memcpy(fill, start, sizeof(int32_t) * (size_t)C);
    for (int i = 0; i < n; ++i) perm[fill[cid[i]]++] = i;   /* stable */
    free(fill);
  }
  if (cell) memcpy(cell, cid, sizeof(int32_t) * (size_t)n);
  if (cell_start) memcpy(cell_start, start, sizeof(int32_t) * ((size_t)C + 1));
  free(cid);
  free(start);
  return 0;
}

/* Sub-cell order inside each cell: with R = 2^sub_bits sub-cells per axis,
 * the sub-cell index along an axis is floor(x_w * n_c * R) - c * R (FP64,
 * clamped to [0, R-1]), and particles of a cell are ordered by the Morton
 * code of (sx, sy, sz) (bit b of sx at 3b, of sy at 3b+1, of sz at 3b+2),
 * then by input index. key = cell * R^3 + morton; sub_start[C R^3 + 1] is the
 * CSR index of the keys. sub_bits = 0 gives the plain (cell, index) order. */
static uint32_t morton3(int sx, int sy, int sz, int bits) {
  uint32_t m = 0;
  for (int b = 0; b < bits; ++b) {
    m |= (uint32_t)((sx >> b) & 1) << (3 * b);
    m |= (uint32_t)((sy >> b) & 1) << (3 * b + 1);
    m |= (uint32_t)((sz >> b) & 1) << (3 * b + 2);
  }
  return m;
}

int orc_bin_sub(int n, const double *x, int n_c, int sub_bits, int32_t *key,
                int32_t *sub_start, int32_t *perm) {
  if (n < 0 || n_c < 1 || sub_bits < 0 || sub_bits > 4) return -1;
  int R = 1 << sub_bits;
  int64_t S = (int64_t)n_c * n_c * n_c * R * R * R;
  if (S >= (1LL << 31)) return -1;
  int32_t *k = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t *start = (int32_t *)calloc((size_t)S + 1, sizeof(int32_t));
  for (int i = 0; i < n; ++i) {
    int cc[3], ss[3];
    for (int a = 0; a < 3; ++a) {
      double xw = wrap01(x[3 * i + a]);
      cc[a] = cell_axis(xw, n_c);
      double t = floor(xw * (double)(n_c * R));
      int sa = (t != t) ? 0 : (int)(t - (double)cc[a] * R);
      if (sa < 0) sa = 0;
      if (sa > R - 1) sa = R - 1;
      ss[a] = sa;
    }
    int c = cc[0] + n_c * (cc[1] + n_c * cc[2]);
    k[i] = (int32_t)((int64_t)c * R * R * R + morton3(ss[0], ss[1], ss[2], sub_bits));
    start[k[i] + 1] += 1;
  }
  for (int64_t c = 0; c < S; ++c) start[c + 1] += start[c];
  if (perm) {
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)S);
    memcpy(fill, start, sizeof(int32_t) * (size_t)S);
    for (int i = 0; i < n; ++i) perm[fill[k[i]]++] = i;   /* stable */
    free(fill);
  }
  if (key) memcpy(key, k, sizeof(int32_t) * (size_t)n);
  if (sub_start) memcpy(sub_start, start, sizeof(int32_t) * ((size_t)S + 1));
  free(k);
  free(start);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Neighbour lists                                                           */
/* ------------------------------------------------------------------------ */

/* minimum-image separation x_i - x_j in the periodic unit box */
static double sep2(const double *x, int i, int j, double d[3]) {
  for (int k = 0; k < 3; ++k) {
    double t = x[3 * i + k] - x[3 * j + k];
    d[k] = t - nearbyint(t);
  }
  return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

typedef struct { int32_t *idx; int n, cap; } nlist;

static void nl_push(nlist *l, int j) {
  if (l->n == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 128;
    l->idx = (int32_t *)realloc(l->idx, sizeof(int32_t) * (size_t)l->cap);
  }
  l->idx[l->n++] = j;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

typedef struct {
  int n, n_c;
  int32_t *cell, *start, *perm;
} cellgrid;

static int grid_build(cellgrid *g, int n, const double *x, int n_c) {
  g->n = n;
  g->n_c = n_c;
  int C = n_c * n_c * n_c;
  g->cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  g->start = (int32_t *)malloc(sizeof(int32_t) * ((size_t)C + 1));
  g->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  return orc_bin(n, x, n_c, g->cell, g->start, g->perm, NULL);
}

static void grid_free(cellgrid *g) {
  free(g->cell);
  free(g->start);
  free(g->perm);
}

/* kind 0: density list {j : r_ij < H_i}, self included.
 * kind 1: force list {j != i : r_ij < max(H_i, H_j)}.
 * jmask (NULL: every j) restricts j to the particles with jmask[j] != 0, so
 * a sum over a subset of pairs (one cell pair) is the same expression.
 * The list comes back sorted by ascending j. */
static void neighbours(int kind, int i, int n, const double *x, const double *h,
                       double gamma_k, int mode, const cellgrid *g,
                       const uint8_t *jmask, nlist *out) {
  out->n = 0;
  double Hi = gamma_k * h[i];
  double d[3];
  if (mode == 0) {
    for (int j = 0; j < n; ++j) {
      if (jmask && !jmask[j]) continue;
      double r2 = sep2(x, i, j, d);
      double r = sqrt(r2);
      if (kind == 0) {
        if (r < Hi) nl_push(out, j);
      } else {
        double Hj = gamma_k * h[j];
        if (j != i && (r < Hi || r < Hj)) nl_push(out, j);
      }
    }
  } else {
    int n_c = g->n_c;
    int ci = g->cell[i];
    int cx = ci % n_c, cy = (ci / n_c) % n_c, cz = ci / (n_c * n_c);
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int nx = (cx + dx + n_c) % n_c, ny = (cy + dy + n_c) % n_c,
              nz = (cz + dz + n_c) % n_c;
          int cn = nx + n_c * (ny + n_c * nz);
          for (int t = g->start[cn]; t < g->start[cn + 1]; ++t) {
            int j = g->perm[t];
            if (jmask && !jmask[j]) continue;
            double r2 = sep2(x, i, j, d);
            double r = sqrt(r2);
            if (kind == 0) {
              if (r < Hi) nl_push(out, j);
            } else {
              double Hj = gamma_k * h[j];
              if (j != i && (r < Hi || r < Hj)) nl_push(out, j);
            }
          }
        }
    qsort(out->idx, (size_t)out->n, sizeof(int32_t), cmp_i32);
  }
}

/* the cell list finds every neighbour only if the cell side is >= max H */
static int grid_ok(int n, const double *h, double gamma_k, int n_c) {
  if (n_c < 3) return 0;
  double side = 1.0 / (double)n_c;
  for (int i = 0; i < n; ++i)
    if (!(gamma_k * h[i] <= side)) return 0;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Density loop (Eq. density) with dRho/dh, weighted neighbour number,       */
/* grad-h factor, pressure and sound speed                                   */
/* ------------------------------------------------------------------------ */

int orc_density(int n, const double *x, const double *m, const double *h,
                const double *u, const orc_params *p, int mode, int n_c,
                const int32_t *sel, int nsel, const uint8_t *jmask, double *rho,
                double *wcount, double *rho_dh, double *f, double *P, double *c,
                int32_t *nngb) {
  cellgrid g;
  memset(&g, 0, sizeof g);
  if (mode == 1) {
    if (!grid_ok(n, h, p->gamma_k, n_c)) return -2;
    grid_build(&g, n, x, n_c);
  }
  int cnt = sel ? nsel : n;
#pragma omp parallel
  {
    nlist l = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
    for (int s = 0; s < cnt; ++s) {
      int i = sel ? sel[s] : s;
      neighbours(0, i, n, x, h, p->gamma_k, mode, &g, jmask, &l);
      double rho_i = 0.0, S = 0.0, dh = 0.0, d[3];
      for (int t = 0; t < l.n; ++t) {
        int j = l.idx[t];
        double r = sqrt(sep2(x, i, j, d));
        double Hi = p->gamma_k * h[i];
        rho_i += m[j] * orc_W_k(p->kernel, r, h[i], p->gamma_k);
        S += orc_kernel_w(p->kernel, r / Hi);
        dh += m[j] * orc_dWdh_k(p->kernel, r, h[i], p->gamma_k);
      }
      /* grad-h term Omega_i = 1 + (h_i / (3 rho_i)) d rho_i / d h_i,
       * from h = eta (m / rho)^(1/3) */
      double omega = 1.0 + h[i] * dh / (3.0 * rho_i);
      rho[s] = rho_i;
      if (wcount) wcount[s] = (4.0 * ORC_PI / 3.0) * S;
      if (rho_dh) rho_dh[s] = dh;
      if (f) f[s] = p->gradh ? 1.0 / omega : 1.0;
      /* ideal gas: P = (gamma - 1) rho u, c = sqrt(gamma P / rho) */
      if (P) P[s] = (p->gamma - 1.0) * rho_i * u[i];
      if (c) c[s] = sqrt(p->gamma * (p->gamma - 1.0) * u[i]);
      if (nngb) nngb[s] = l.n;
    }
    free(l.idx);
  }
  if (mode == 1) grid_free(&g);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Force loop (Eq. momentum and Eq. energy of Sec. 2.1, discrete form):      */
/*   dv_i/dt = -sum_j m_j (A_i g_i + A_j g_j + Pi_ij gbar_ij) e_ij           */
/*   du_i/dt =  sum_j m_j (A_i g_i + Pi_ij gbar_ij / 2) (v_ij . e_ij)        */
/* with A_k = f_k P_k / rho_k^2, g_k = |grad W(r_ij, h_k)| (signed),         */
/* gbar = (g_i + g_j) / 2, Pi_ij the signal-velocity viscosity.              */
/* rho, f, P, c are arrays over all particles (input order).                 */
/* ------------------------------------------------------------------------ */

int orc_force(int n, const double *x, const double *v, const double *m,
              const double *h, const double *rho, const double *f,
              const double *P, const double *c, const orc_params *p, int mode,
              int n_c, const int32_t *sel, int nsel, const uint8_t *jmask, double *a,
              double *du, double *vsig, int32_t *nforce) {
  cellgrid g;
  memset(&g, 0, sizeof g);
  if (mode == 1) {
    if (!grid_ok(n, h, p->gamma_k, n_c)) return -2;
    grid_build(&g, n, x, n_c);
  }
  int cnt = sel ? nsel : n;
#pragma omp parallel
  {
    nlist l = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
    for (int s = 0; s < cnt; ++s) {
      int i = sel ? sel[s] : s;
      neighbours(1, i, n, x, h, p->gamma_k, mode, &g, jmask, &l);
      double ai[3] = {0.0, 0.0, 0.0}, dui = 0.0, vs = 0.0, d[3];
      double fi = p->gradh ? f[i] : 1.0;
      double Ai = fi * P[i] / (rho[i] * rho[i]);
      for (int t = 0; t < l.n; ++t) {
        int j = l.idx[t];
        double r = sqrt(sep2(x, i, j, d));
        /* coincident positions (j != i, r = 0): the pair direction is taken
         * as the zero vector, the limit of the pair terms as r -> 0
         * averaged over directions; the pair counts, exerts no force and
         * does no work, and its signal velocity is c_i + c_j */
        double e[3] = {0.0, 0.0, 0.0};
        if (r > 0.0)
          for (int k = 0; k < 3; ++k) e[k] = d[k] / r;
        double fj = p->gradh ? f[j] : 1.0;
        double Aj = fj * P[j] / (rho[j] * rho[j]);
        double gi = orc_gradW(p->kernel, r, h[i], p->gamma_k);
        double gj = orc_gradW(p->kernel, r, h[j], p->gamma_k);
        double w = (v[3 * i + 0] - v[3 * j + 0]) * e[0] +
                   (v[3 * i + 1] - v[3 * j + 1]) * e[1] +
                   (v[3 * i + 2] - v[3 * j + 2]) * e[2];
        double mu = w < 0.0 ? w : 0.0;
        double vsig_ij = c[i] + c[j] - p->beta * mu;
        double Pi = -p->alpha * vsig_ij * mu / (rho[i] + rho[j]);
        double gbar = 0.5 * (gi + gj);
        double K = Ai * gi + Aj * gj + Pi * gbar;
        for (int k = 0; k < 3; ++k) ai[k] -= m[j] * K * e[k];
        dui += m[j] * (Ai * gi * w + 0.5 * Pi * gbar * w);
        if (vsig_ij > vs) vs = vsig_ij;
      }
      for (int k = 0; k < 3; ++k) a[3 * s + k] = ai[k];
      du[s] = dui;
      if (vsig) vsig[s] = vs;
      if (nforce) nforce[s] = l.n;
    }
    free(l.idx);
  }
  if (mode == 1) grid_free(&g);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Smoothing lengths adapted to the local density (Sec. 2.1: h follows the   */
/* density so that the neighbour number stays about constant), from         */
/* h = eta (m / rho)^(1/3). The density sum gathers with h_i, so rho_i is a  */
/* function of particle i's own h: each particle solves                      */
/*   f(h) = h - eta (m / rho(h))^(1/3) = 0                                   */
/* by Newton steps, f'(h) = 1 + (h_t / (3 rho)) drho/dh with                 */
/* h_t = eta (m / rho(h))^(1/3); a step that f' <= 0 would make is replaced  */
/* by h_t; every new h is limited to [h/2, 2h] and to h_max; the iteration   */
/* stops after the first step with |h_new - h| < tol h (h_new is kept) that  */
/* the h_max limit did not cut.                                              */
/* iters[s] = steps taken (max_iter + 1: not converged).                     */
/* ------------------------------------------------------------------------ */

static void density_at(int i, double hi, int n, const double *x, const double *m,
                       double gamma_k, int kernel, int mode, const cellgrid *g, nlist *l,
                       double *rho, double *drho_dh) {
  /* neighbours of i for support gamma_k hi: a local h array view */
  double d[3];
  double Hi = gamma_k * hi;
  l->n = 0;
  if (mode == 0) {
    for (int j = 0; j < n; ++j) {
      double r = sqrt(sep2(x, i, j, d));
      if (r < Hi) nl_push(l, j);
    }
  } else {
    int n_c = g->n_c;
    int ci = g->cell[i];
    int cx = ci % n_c, cy = (ci / n_c) % n_c, cz = ci / (n_c * n_c);
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int cn = ((cx + dx + n_c) % n_c) + n_c * (((cy + dy + n_c) % n_c) +
                                                     n_c * ((cz + dz + n_c) % n_c));
          for (int t = g->start[cn]; t < g->start[cn + 1]; ++t) {
            int j = g->perm[t];
            double r = sqrt(sep2(x, i, j, d));
            if (r < Hi) nl_push(l, j);
          }
        }
    qsort(l->idx, (size_t)l->n, sizeof(int32_t), cmp_i32);
  }
  double r_sum = 0.0, dh = 0.0;
  for (int t = 0; t < l->n; ++t) {
    int j = l->idx[t];
    double r = sqrt(sep2(x, i, j, d));
    r_sum += m[j] * orc_W_k(kernel, r, hi, gamma_k);
    dh += m[j] * orc_dWdh_k(kernel, r, hi, gamma_k);
  }
  *rho = r_sum;
  *drho_dh = dh;
}

int orc_smoothing_length(int n, const double *x, const double *m, const double *h0,
                         double eta, const orc_params *p, int mode, int n_c, double h_max,
                         double tol, int max_iter, const int32_t *sel, int nsel,
                         double *h_out, int32_t *iters) {
  cellgrid g;
  memset(&g, 0, sizeof g);
  if (mode == 1) {
    if (n_c < 3 || !(p->gamma_k * h_max <= 1.0 / (double)n_c)) return -2;
    grid_build(&g, n, x, n_c);
  }
  int cnt = sel ? nsel : n;
#pragma omp parallel
  {
    nlist l = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
    for (int s = 0; s < cnt; ++s) {
      int i = sel ? sel[s] : s;
      double h = h0[i] < h_max ? h0[i] : h_max;
      int it = 0;
      for (; it < max_iter; ++it) {
        double rho, drho;
        density_at(i, h, n, x, m, p->gamma_k, p->kernel, mode, &g, &l, &rho, &drho);
        double ht = eta * cbrt(m[i] / rho);
        double f = h - ht;
        double fp = 1.0 + ht / (3.0 * rho) * drho;
        double hn = fp > 0.0 ? h - f / fp : ht;
        if (hn < 0.5 * h) hn = 0.5 * h;
        if (hn > 2.0 * h) hn = 2.0 * h;
        int capped = hn > h_max;
        if (capped) hn = h_max;
        int done = !capped && fabs(hn - h) < tol * h;
        h = hn;
        if (done) break;
      }
      h_out[s] = h;
      if (iters) iters[s] = it < max_iter ? it + 1 : max_iter + 1;
    }
    free(l.idx);
  }
  if (mode == 1) grid_free(&g);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Kick and drift (linear kernels, Alg. 1 CallLinear): kick v and u, then    */
/* drift x with the kicked velocity and wrap into the periodic box.          */
/* ------------------------------------------------------------------------ */

void orc_kick_drift(int n, double *x, double *v, double *u, const double *a,
                    const double *du, double dt_kick, double dt_drift) {
  for (int i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) v[3 * i + k] = v[3 * i + k] + a[3 * i + k] * dt_kick;
    u[i] = u[i] + du[i] * dt_kick;
    for (int k = 0; k < 3; ++k) {
      double xn = x[3 * i + k] + v[3 * i + k] * dt_drift;
      x[3 * i + k] = xn - floor(xn);
    }
  }
}

void orc_reduce(int n, const double *m, const double *v, const double *a,
                const double *du, double *out) {
  for (int k = 0; k < 6; ++k) out[k] = 0.0;
  for (int i = 0; i < n; ++i) {
    double va = 0.0, an = 0.0;
    for (int k = 0; k < 3; ++k) {
      out[k] += m[i] * a[3 * i + k];
      va += v[3 * i + k] * a[3 * i + k];
      an += a[3 * i + k] * a[3 * i + k];
    }
    out[3] += m[i] * (va + du[i]);
    out[4] += m[i] * sqrt(an);
    out[5] += m[i] * (fabs(va) + fabs(du[i]));
  }
}

/* ------------------------------------------------------------------------ */
/* Quantisers (Sec. 3.2, Table 2: the 32- and 16-bit rows are IEEE single    */
/* and half; bfloat16 keeps single's 8-bit exponent). Round to nearest,      */
/* ties to even, written from the IEEE-754 encodings.                        */
/* ------------------------------------------------------------------------ */

static uint32_t f32_bits(float v) {
  uint32_t b;
  memcpy(&b, &v, 4);
  return b;
}

static float bits_f32(uint32_t b) {
  float v;
  memcpy(&v, &b, 4);
  return v;
}

/* round the integer sig right by s bits, ties to even */
static uint32_t rne_shift(uint32_t sig, int s) {
  if (s <= 0) return sig;
  if (s >= 32) return 0;
  uint32_t q = sig >> s;
  uint32_t rem = sig & ((1u << s) - 1u);
  uint32_t half = 1u << (s - 1);
  if (rem > half || (rem == half && (q & 1u))) q += 1u;
  return q;
}

uint16_t orc_f32_to_f16(float v) {
  uint32_t b = f32_bits(v);
  uint16_t sign = (uint16_t)((b >> 16) & 0x8000u);
  uint32_t E = (b >> 23) & 0xffu, M = b & 0x7fffffu;
  if (E == 0xffu) return (uint16_t)(sign | (M ? 0x7e00u : 0x7c00u));  /* NaN, Inf */
  if (E == 0u) return sign;   /* FP32 subnormals are below half of 2^-24 */
  int e = (int)E - 127;       /* value = 1.M * 2^e */
  uint32_t sig = (1u << 23) | M;
  if (e >= -14) {             /* normal half: 10 fraction bits */
    uint32_t q = rne_shift(sig, 13);          /* 11 bits incl. hidden one */
    int he = e + 15;
    if (q == (1u << 11)) { q >>= 1; he += 1; }
    if (he >= 31) return (uint16_t)(sign | 0x7c00u);
    return (uint16_t)(sign | ((uint32_t)he << 10) | (q & 0x3ffu));
  }
  /* subnormal half: value / 2^-24 = sig * 2^(e + 1 - 23 + 23) */
  int s = -(e + 1);           /* sig * 2^(e+1) = sig >> s */
  uint32_t q = rne_shift(sig, s);
  return (uint16_t)(sign | q); /* q == 0x400 encodes the smallest normal */
}

float orc_f16_to_f32(uint16_t h) {
  uint32_t sign = ((uint32_t)h & 0x8000u) << 16;
  uint32_t E = (h >> 10) & 0x1fu, M = h & 0x3ffu;
  if (E == 0x1fu) return bits_f32(sign | 0x7f800000u | (M << 13));
  if (E == 0u) {
    float mag = (float)M * 0x1p-24f;          /* exact */
    return sign ? -mag : mag;
  }
  return bits_f32(sign | ((E - 15u + 127u) << 23) | (M << 13));
}

uint16_t orc_f32_to_bf16(float v) {
  uint32_t b = f32_bits(v);
  uint32_t E = (b >> 23) & 0xffu, M = b & 0x7fffffu;
  if (E == 0xffu && M) return (uint16_t)(((b >> 16) & 0x8000u) | 0x7fc0u);
  /* keep the top 16 bits, round the low 16 to nearest even; a carry into
   * the exponent (up to infinity) is the correct rounding */
  uint32_t q = rne_shift(b & 0x7fffffffu, 16);
  return (uint16_t)(((b >> 16) & 0x8000u) | q);
}

float orc_bf16_to_f32(uint16_t h) { return bits_f32((uint32_t)h << 16); }

void orc_quant_array(int64_t n, const float *in, uint16_t *out, int dtype) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    out[i] = dtype == ORC_BF16 ? orc_f32_to_bf16(in[i]) : orc_f32_to_f16(in[i]);
}

void orc_dequant_array(int64_t n, const uint16_t *in, float *out, int dtype) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    out[i] = dtype == ORC_BF16 ? orc_bf16_to_f32(in[i]) : orc_f16_to_f32(in[i]);
}

/* truncate_mantissa(T) storage (Sec. 3.2, Table 2), T bits in total: where T
 * is an IEEE size (64, 32, 16) that format is used; otherwise the smallest
 * IEEE layout wider than T keeps its sign and exponent fields and the top
 * T - 1 - e bits of its mantissa (e = 11, 8, 5 for 33..63, 17..31, 9..15),
 * the lower bits being cut off (rounding toward zero). A value reaches its
 * base layout by the IEEE conversion (round to nearest even): FP64 -> FP32
 * for T <= 32, then FP32 -> half for T <= 16. Written on the bit patterns:
 * the stored code is the top T bits of the base pattern. */
static double trunc_roundtrip(double v, int T, int scale) {
  if (T >= 64) return v;
  if (T >= 33) {
    uint64_t b;
    double s = ldexp(v, scale);
    memcpy(&b, &s, 8);
    b = (b >> (64 - T)) << (64 - T);
    memcpy(&s, &b, 8);
    return ldexp(s, -scale);
  }
  float s = ldexpf((float)v, scale);
  if (T >= 17) {
    uint32_t b = f32_bits(s);
    b = (b >> (32 - T)) << (32 - T);
    return (double)ldexpf(bits_f32(b), -scale);
  }
  uint16_t h = orc_f32_to_f16(s);
  h = (uint16_t)((h >> (16 - T)) << (16 - T));
  return (double)ldexpf(orc_f16_to_f32(h), -scale);
}

/* stored value of v: RNE to FP32, times 2^scale (exact), RNE to the storage
 * format; read back: widen to FP32, times 2^-scale. FP64 storage is exact. */
static float roundtrip32(double v, int dtype, int scale) {
  if (dtype >= ORC_TRUNC) return (float)trunc_roundtrip(v, dtype - ORC_TRUNC, scale);
  float q32 = (float)v;
  if (dtype == ORC_F32) return q32;
  float s = ldexpf(q32, scale);
  float back = dtype == ORC_BF16 ? orc_bf16_to_f32(orc_f32_to_bf16(s))
                                 : orc_f16_to_f32(orc_f32_to_f16(s));
  return ldexpf(back, -scale);
}

double orc_roundtrip(double v, int dtype, int scale) {
  if (dtype == ORC_F64) return v;
  if (dtype >= ORC_TRUNC) return trunc_roundtrip(v, dtype - ORC_TRUNC, scale);
  return (double)roundtrip32(v, dtype, scale);
}

/* Offsets of the stored positions from their anchor (Sec. 3.2's anchor
 * and delta: a value is kept as a quantised difference from an anchor the
 * reader reconstructs). The anchor of a particle in cell c is
 *   anchor 0:      the cell corner c / n_c, per axis;
 *   anchor 1 + b:  the centre of its sub-cell of side 1 / (n_c 2^b),
 *                  (c 2^b + a + 1/2) / (n_c 2^b), with the sub-cell index
 *                  a = floor(x_w n_c 2^b) - c 2^b clamped to [0, 2^b - 1]
 *                  (b = 0: the cell centre; b <= 2),
 * all in FP64 on the wrapped position x_w. off = x_w - anchor in FP64;
 * code = a_x + 4 a_y + 16 a_z (0 for anchor 0 and 1). Either output may be
 * NULL. */
static int anchor_of(double xw, int c, int n_c, int anchor, double *o) {
  if (anchor == 0) {
    *o = (double)c / (double)n_c;
    return 0;
  }
  int R = 1 << (anchor - 1);
  double t = floor(xw * (double)(n_c * R));
  int a = (t != t) ? 0 : (int)(t - (double)c * R);
  if (a < 0) a = 0;
  if (a > R - 1) a = R - 1;
  *o = ((double)c * R + a + 0.5) / ((double)n_c * R);
  return a;
}

int orc_pos_offsets(int n, const double *x, int n_c, int anchor, double *off, uint8_t *code) {
  if (n < 0 || n_c < 1 || anchor < 0 || anchor > 3) return -1;
  for (int i = 0; i < n; ++i) {
    int cc = 0;
    for (int k = 0; k < 3; ++k) {
      double xw = wrap01(x[3 * i + k]), o;
      int a = anchor_of(xw, cell_axis(xw, n_c), n_c, anchor, &o);
      if (off) off[3 * i + k] = xw - o;
      cc |= a << (2 * k);
    }
    if (code) code[i] = (uint8_t)cc;
  }
  return 0;
}

int orc_dequantise_set(int n, const double *x, const double *v, const double *m,
                       const double *h, const double *u, int n_c, int pos_dt,
                       int vel_dt, int mhu_dt, const int32_t *scales, int pos_anchor,
                       double *xq, double *vq, double *mq, double *hq, double *uq) {
  if (pos_anchor < 0 || pos_anchor > 3) return -1;
  int s_m = scales ? scales[0] : 0, s_h = scales ? scales[1] : 0, s_u = scales ? scales[2] : 0;
  for (int i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) {
      double xw = wrap01(x[3 * i + k]), o;
      anchor_of(xw, cell_axis(xw, n_c), n_c, pos_anchor, &o);
      xq[3 * i + k] = o + orc_roundtrip(xw - o, pos_dt, 0);
      vq[3 * i + k] = orc_roundtrip(v[3 * i + k], vel_dt, 0);
    }
    mq[i] = orc_roundtrip(m[i], mhu_dt, s_m);
    hq[i] = orc_roundtrip(h[i], mhu_dt, s_h);
    uq[i] = orc_roundtrip(u[i], mhu_dt, s_u);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Pairs near the support boundary. A neighbour count taken in another        */
/* precision (or with positions rounded differently) can differ from the     */
/* FP64 count of this oracle only through pairs whose separation lies within */
/* that precision's rounding of the support radius. For each selected i:      */
/*   near_d = #{j : |r_ij - H_i| < eps_rel H_i + eps_abs}                      */
/*   near_f = #{j != i : |r_ij - H_i| < tol_i or |r_ij - H_j| < tol_j}         */
/* with tol_k = eps_rel H_k + eps_abs; r_ij is the FP64 minimum-image         */
/* separation (the same expression as in the density and force sums).        */
/* Pairs beyond the 27 cells around i's cell are not candidates of a cell    */
/* list and are not counted (mode 1); brute force (mode 0) counts all.       */
/* ------------------------------------------------------------------------ */
int orc_near_support(int n, const double *x, const double *h, double gamma_k, int mode,
                     int n_c, const int32_t *sel, int nsel, double eps_rel, double eps_abs,
                     int32_t *near_d, int32_t *near_f) {
  cellgrid g;
  memset(&g, 0, sizeof g);
  if (mode == 1) {
    if (!grid_ok(n, h, gamma_k, n_c)) return -2;
    grid_build(&g, n, x, n_c);
  }
  int cnt = sel ? nsel : n;
#pragma omp parallel for schedule(dynamic, 64)
  for (int s = 0; s < cnt; ++s) {
    int i = sel ? sel[s] : s;
    double Hi = gamma_k * h[i], ti = eps_rel * Hi + eps_abs, d[3];
    int nd = 0, nf = 0;
    int lo = 0, hi = n, C = mode == 1 ? 27 : 1;
    for (int q = 0; q < C; ++q) {
      if (mode == 1) {
        int ci = g.cell[i];
        int cx = ci % n_c, cy = (ci / n_c) % n_c, cz = ci / (n_c * n_c);
        int cn = ((cx + q % 3 - 1 + n_c) % n_c) +
                 n_c * (((cy + (q / 3) % 3 - 1 + n_c) % n_c) + n_c * ((cz + q / 9 - 1 + n_c) % n_c));
        lo = g.start[cn];
        hi = g.start[cn + 1];
      }
      for (int t = lo; t < hi; ++t) {
        int j = mode == 1 ? g.perm[t] : t;
        double r = sqrt(sep2(x, i, j, d));
        double Hj = gamma_k * h[j], tj = eps_rel * Hj + eps_abs;
        int near_i = fabs(r - Hi) < ti;
        if (near_i) nd++;
        if (j != i && (near_i || fabs(r - Hj) < tj)) nf++;
      }
    }
    if (near_d) near_d[s] = nd;
    if (near_f) near_f[s] = nf;
  }
  if (mode == 1) grid_free(&g);
  return 0;
}

/* threads the following OpenMP parallel regions use (n >= 1) */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* threads an OpenMP parallel region of the oracle uses */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
