/*
 * dirac_oracle.c -- CPU FP64 oracle for the spacetime finite-element Dirac solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * executes this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the HIP
 * path.  Everything is complex128, written for obviousness rather than speed.
 *
 * Paper: "A Spacetime Finite Elements Method to Solve the Dirac Equation"
 * (arXiv:2103.14588).
 *
 * What is computed, and where the paper defines it:
 *   - Q1 Lagrange tensor basis on each spacetime element: Sec. 2.2, eqs.
 *     (lag_el1)-(lag_el4) (read as products of 1D hats, with 1/h^2 normalisation).
 *   - Element matrices D^t, D^x, D^0 and their gamma combination
 *     i g^0 D^t + i g^x D^x - m I D^0: App. A, eq. (diracWeak1p1), extended to
 *     2+1 and 3+1 the way App. A states (one derivative matrix per axis).
 *   - Element-by-element summation into the global block matrix D_w: Sec. 2.2
 *     (sum of element stiffness matrices) and eq. (Dw).
 *   - Removal of the t=0 test rows and the move of the t=0 columns to the right
 *     hand side, D_w22 Psi = -D_w21 Psi_0: Sec. 2.1, eqs. (dirac_weakIVP),
 *     (bp:dirac); Alg. 1 steps 3-5.
 *   - Scalar potential coupling: Sec. 4.3 (Klein paradox operator), with the sign
 *     convention H = alpha.p + beta m + V (minimal coupling i d_t -> i d_t - V).
 *   - GMRES (Saad-Schultz), Sec. 2.2 and Alg. 1 step 6, here restarted GMRES(m)
 *     with two-pass classical Gram-Schmidt, complex Givens rotations and right
 *     preconditioning.
 *
 * Readings where the paper is silent (listed with the others in the design notes):
 *   - space is periodic; time nodes are tau = 0..n_t with tau = 0 known; the
 *     last time slice keeps its (one-sided) test rows, so the system is square;
 *   - potential integrated with 2-point Gauss-Legendre per axis; step is strict
 *     (V = V0 iff x > x0);
 *   - unknown numbering r = (tau-1)*S + spatial index with axis 1 fastest;
 *     component index r*nc + c.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
  int32_t d;      /* spatial dimensions 1..3 */
  int32_t nc;     /* spinor components: 2 for d <= 2, 4 for d = 3 */
  int32_t n[4];   /* n[0] time elements, n[1..d] spatial elements */
  double len[4];  /* len[0] = T, len[1..d] = box lengths */
  double m;       /* mass */
  int32_t vkind;  /* 0 none, 1 step V0*[x > x0], 2 smooth V0/2 (1 + tanh((x - x0)/lw)) */
  double v0, x0, lw;
} orc_problem;

/* ------------------------------------------------------------------ gammas */
/* Gamma matrices, row-major nc x nc.  1+1: the pair written in App. A.
 * 2+1: g0 = s3, g1 = i s2, g2 = -i s1 (reduces to the App. A pair).
 * 3+1: Dirac representation.  All satisfy {g^mu, g^nu} = 2 eta^{mu nu},
 * eta = diag(+,-,-,-). */
int orc_gamma(int d, int mu, cplx *g) {
  int nc = (d == 3) ? 4 : 2;
  memset(g, 0, sizeof(cplx) * nc * nc);
  if (mu < 0 || mu > d) return -1;
  if (nc == 2) {
    if (mu == 0) { g[0] = 1; g[3] = -1; }
    else if (mu == 1) { g[1] = 1; g[2] = -1; }
    else { g[1] = -I; g[2] = -I; }
    return 0;
  }
  /* Pauli matrices */
  cplx s[3][4] = {{0, 1, 1, 0}, {0, -I, I, 0}, {1, 0, 0, -1}};
  if (mu == 0) {
    g[0] = 1; g[5] = 1; g[10] = -1; g[15] = -1;
    return 0;
  }
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++) {
      g[a * 4 + (b + 2)] = s[mu - 1][a * 2 + b];      /* upper right:  sigma_k */
      g[(a + 2) * 4 + b] = -s[mu - 1][a * 2 + b];     /* lower left:  -sigma_k */
    }
  return 0;
}

/* ------------------------------------------------------------------ basics */
static int problem_ok(const orc_problem *p) {
  if (p->d < 1 || p->d > 3) return 0;
  if (p->nc != ((p->d == 3) ? 4 : 2)) return 0;
  if (p->n[0] < 1) return 0;
  for (int a = 1; a <= p->d; a++) if (p->n[a] < 2) return 0;
  for (int a = 0; a <= p->d; a++) if (!(p->len[a] > 0)) return 0;
  return 1;
}

int64_t orc_spatial_nodes(const orc_problem *p) {
  int64_t s = 1;
  for (int a = 1; a <= p->d; a++) s *= p->n[a];
  return s;
}

int64_t orc_nrows(const orc_problem *p) { return (int64_t)p->n[0] * orc_spatial_nodes(p); }

/* potential energy V(x) along spatial axis 1 (Sec. 4.3 and its smooth step) */
double orc_potential(const orc_problem *p, double x) {
  if (p->vkind == 1) return (x > p->x0) ? p->v0 : 0.0;
  if (p->vkind == 2) return 0.5 * p->v0 * (1.0 + tanh((x - p->x0) / p->lw));
  return 0.0;
}

/* 1D hat functions on [0, h]: phi_0 = 1 - s/h, phi_1 = s/h */
static double hat(int b, double s, double h) { return b ? s / h : 1.0 - s / h; }
static double dhat(int b, double h) { return b ? 1.0 / h : -1.0 / h; }

/* 1D element integrals by 2-point Gauss-Legendre (exact for these quadratics):
 * mass[b][a] = int phi_b phi_a, conv[b][a] = int phi_b phi_a'
 * (row b = test function, column a = trial function). */
static void elem1d(double h, double mass[2][2], double conv[2][2]) {
  const double g = 1.0 / sqrt(3.0);
  double q[2] = {0.5 * h * (1 - g), 0.5 * h * (1 + g)};
  for (int b = 0; b < 2; b++)
    for (int a = 0; a < 2; a++) {
      mass[b][a] = 0; conv[b][a] = 0;
      for (int k = 0; k < 2; k++) {
        mass[b][a] += 0.5 * h * hat(b, q[k], h) * hat(a, q[k], h);
        conv[b][a] += 0.5 * h * hat(b, q[k], h) * dhat(a, h);
      }
    }
}

/* Element block matrix for element e (e[0] time index, e[1..d] spatial).
 * Local node beta has bit a = offset along axis a (bit 0 = time).
 * B[((beta * nloc) + alpha) * nc*nc + i*nc + j] =
 *     sum_mu i g^mu D^mu_{beta alpha} - m D^0_{beta alpha} delta_ij - g^0 P_{beta alpha}
 * with D^mu = prod_a (a == mu ? conv_a : mass_a) and
 * P_{beta alpha} = int V phi_beta phi_alpha by tensor 2-point Gauss over the element. */
void orc_element_matrix(const orc_problem *p, const int32_t *e, cplx *B) {
  const int D = p->d + 1, nc = p->nc, nloc = 1 << D;
  double mass[4][2][2], conv[4][2][2], h[4];
  for (int a = 0; a < D; a++) {
    h[a] = p->len[a] / p->n[a];
    elem1d(h[a], mass[a], conv[a]);
  }
  cplx gam[4][16];
  for (int mu = 0; mu < D; mu++) orc_gamma(p->d, mu, gam[mu]);
  const double g = 1.0 / sqrt(3.0);
  for (int be = 0; be < nloc; be++)
    for (int al = 0; al < nloc; al++) {
      double Dmu[4], D0 = 1.0;
      for (int mu = 0; mu < D; mu++) {
        double v = 1.0;
        for (int a = 0; a < D; a++) {
          int bb = (be >> a) & 1, aa = (al >> a) & 1;
          v *= (a == mu) ? conv[a][bb][aa] : mass[a][bb][aa];
        }
        Dmu[mu] = v;
      }
      for (int a = 0; a < D; a++) D0 *= mass[a][(be >> a) & 1][(al >> a) & 1];
      /* potential: tensor Gauss points, all D axes */
      double P = 0.0;
      if (p->vkind != 0) {
        for (int q = 0; q < nloc; q++) {
          double w = 1.0, phib = 1.0, phia = 1.0, x1 = 0.0;
          for (int a = 0; a < D; a++) {
            double s = 0.5 * h[a] * (1 + (((q >> a) & 1) ? g : -g));
            w *= 0.5 * h[a];
            phib *= hat((be >> a) & 1, s, h[a]);
            phia *= hat((al >> a) & 1, s, h[a]);
            if (a == 1) x1 = e[1] * h[1] + s;
          }
          P += w * orc_potential(p, x1) * phib * phia;
        }
      }
      cplx *blk = B + ((size_t)be * nloc + al) * nc * nc;
      for (int i = 0; i < nc; i++)
        for (int j = 0; j < nc; j++) {
          cplx v = 0;
          for (int mu = 0; mu < D; mu++) v += I * gam[mu][i * nc + j] * Dmu[mu];
          if (i == j) v -= p->m * D0;
          v -= gam[0][i * nc + j] * P;
          blk[i * nc + j] = v;
        }
    }
}

/* global node coordinates of local node beta of element e; returns time index */
static void local_to_global(const orc_problem *p, const int32_t *e, int beta, int32_t *g) {
  const int D = p->d + 1;
  for (int a = 0; a < D; a++) {
    int32_t c = e[a] + ((beta >> a) & 1);
    if (a > 0) c %= p->n[a];   /* periodic space */
    g[a] = c;
  }
}

static int64_t spatial_index(const orc_problem *p, const int32_t *g) {
  int64_t s = 0, stride = 1;
  for (int a = 1; a <= p->d; a++) { s += g[a] * stride; stride *= p->n[a]; }
  return s;
}

/* ------------------------------------------------------------- assembly */
/* Block-row matrix: row r has cols[rowptr[r]..rowptr[r+1]) (column nodes,
 * ascending) and nc*nc blocks, row-major. */
typedef struct {
  orc_problem p;
  int64_t nrows, nnzb;
  int64_t *rowptr, *col;
  cplx *val;
  /* columns at tau = 0 (moved to the right-hand side) */
  int64_t nrows0, nnzb0;   /* rows of the tau = 1 slice only */
  int64_t *rowptr0, *col0;
  cplx *val0;
} orc_matrix;

typedef struct {
  int64_t *cnt, *col;
  cplx *val;
  int cap, nb;
} staging;

static void stage_add(staging *s, int64_t row, int64_t col, const cplx *blk) {
  int64_t base = row * s->cap;
  int64_t k;
  for (k = 0; k < s->cnt[row]; k++)
    if (s->col[base + k] == col) break;
  if (k == s->cnt[row]) {
    if (k >= s->cap) { fprintf(stderr, "oracle: row capacity exceeded\n"); abort(); }
    s->col[base + k] = col;
    memset(s->val + (base + k) * s->nb, 0, sizeof(cplx) * s->nb);
    s->cnt[row]++;
  }
  for (int q = 0; q < s->nb; q++) s->val[(base + k) * s->nb + q] += blk[q];
}

static void stage_to_csr(staging *s, int64_t nrows, int64_t **rowptr, int64_t **col, cplx **val,
                         int64_t *nnzb) {
  *rowptr = malloc(sizeof(int64_t) * (nrows + 1));
  (*rowptr)[0] = 0;
  for (int64_t r = 0; r < nrows; r++) (*rowptr)[r + 1] = (*rowptr)[r] + s->cnt[r];
  *nnzb = (*rowptr)[nrows];
  *col = malloc(sizeof(int64_t) * (*nnzb > 0 ? *nnzb : 1));
  *val = malloc(sizeof(cplx) * s->nb * (*nnzb > 0 ? *nnzb : 1));
  for (int64_t r = 0; r < nrows; r++) {
    int64_t base = r * s->cap, n = s->cnt[r];
    /* insertion sort of the row by column */
    int idx[81];
    for (int k = 0; k < n; k++) idx[k] = k;
    for (int a = 1; a < n; a++) {
      int t = idx[a], b = a - 1;
      while (b >= 0 && s->col[base + idx[b]] > s->col[base + t]) { idx[b + 1] = idx[b]; b--; }
      idx[b + 1] = t;
    }
    for (int k = 0; k < n; k++) {
      (*col)[(*rowptr)[r] + k] = s->col[base + idx[k]];
      memcpy(*val + ((*rowptr)[r] + k) * s->nb, s->val + (base + idx[k]) * s->nb,
             sizeof(cplx) * s->nb);
    }
  }
}

/* Assemble by looping over every spacetime element and adding its element
 * matrix into the global block matrix (scatter-add). */
orc_matrix *orc_build(const orc_problem *p) {
  if (!problem_ok(p)) return NULL;
  const int D = p->d + 1, nc = p->nc, nloc = 1 << D;
  int cap = 1;
  for (int a = 0; a < D; a++) cap *= 3;
  const int64_t S = orc_spatial_nodes(p), nrows = orc_nrows(p);
  staging st = {calloc(nrows, sizeof(int64_t)), malloc(sizeof(int64_t) * nrows * cap),
                malloc(sizeof(cplx) * nrows * cap * nc * nc), cap, nc * nc};
  staging s0 = {calloc(S, sizeof(int64_t)), malloc(sizeof(int64_t) * S * cap),
                malloc(sizeof(cplx) * S * cap * nc * nc), cap, nc * nc};
  if (!st.cnt || !st.col || !st.val || !s0.cnt || !s0.col || !s0.val) {
    fprintf(stderr, "oracle: out of memory\n");
    abort();
  }
  cplx *B = malloc(sizeof(cplx) * nloc * nloc * nc * nc);
  int64_t nelem = 1;
  for (int a = 0; a < D; a++) nelem *= p->n[a];
  for (int64_t el = 0; el < nelem; el++) {
    /* element ordering: time slowest, spatial axis 1 fastest */
    int32_t e[4] = {0, 0, 0, 0};
    int64_t tt = el % S;
    for (int a = 1; a <= p->d; a++) { e[a] = tt % p->n[a]; tt /= p->n[a]; }
    e[0] = (int32_t)(el / S);
    orc_element_matrix(p, e, B);
    for (int be = 0; be < nloc; be++) {
      int32_t gb[4];
      local_to_global(p, e, be, gb);
      if (gb[0] == 0) continue;   /* t = 0 test rows are removed */
      int64_t row = (int64_t)(gb[0] - 1) * S + spatial_index(p, gb);
      for (int al = 0; al < nloc; al++) {
        int32_t ga[4];
        local_to_global(p, e, al, ga);
        const cplx *blk = B + ((size_t)be * nloc + al) * nc * nc;
        if (ga[0] == 0) {
          /* known t = 0 column: only rows of slice tau = 1 touch it */
          stage_add(&s0, row, spatial_index(p, ga), blk);
        } else {
          stage_add(&st, row, (int64_t)(ga[0] - 1) * S + spatial_index(p, ga), blk);
        }
      }
    }
  }
  free(B);
  orc_matrix *A = calloc(1, sizeof(orc_matrix));
  A->p = *p;
  A->nrows = nrows;
  stage_to_csr(&st, nrows, &A->rowptr, &A->col, &A->val, &A->nnzb);
  A->nrows0 = S;
  stage_to_csr(&s0, S, &A->rowptr0, &A->col0, &A->val0, &A->nnzb0);
  free(st.cnt); free(st.col); free(st.val);
  free(s0.cnt); free(s0.col); free(s0.val);
  return A;
}

void orc_free(orc_matrix *A) {
  if (!A) return;
  free(A->rowptr); free(A->col); free(A->val);
  free(A->rowptr0); free(A->col0); free(A->val0);
  free(A);
}

int64_t orc_nnzb(const orc_matrix *A) { return A->nnzb; }
int64_t orc_nnzb0(const orc_matrix *A) { return A->nnzb0; }

void orc_export(const orc_matrix *A, int64_t *rowptr, int64_t *col, cplx *val) {
  int nb = A->p.nc * A->p.nc;
  memcpy(rowptr, A->rowptr, sizeof(int64_t) * (A->nrows + 1));
  memcpy(col, A->col, sizeof(int64_t) * A->nnzb);
  memcpy(val, A->val, sizeof(cplx) * nb * A->nnzb);
}

void orc_export0(const orc_matrix *A, int64_t *rowptr, int64_t *col, cplx *val) {
  int nb = A->p.nc * A->p.nc;
  memcpy(rowptr, A->rowptr0, sizeof(int64_t) * (A->nrows0 + 1));
  memcpy(col, A->col0, sizeof(int64_t) * A->nnzb0);
  memcpy(val, A->val0, sizeof(cplx) * nb * A->nnzb0);
}

/* One block row of the matrix computed on its own, by summing the element
 * matrices of the elements that contain the row node.  Used to check single
 * rows of very large assembled operators.  Writes at most 3^D columns (sorted
 * ascending) and their blocks; returns the count.  Columns at tau = 0 are
 * returned as -(spatial index) - 1. */
int orc_row(const orc_problem *p, int64_t r, int64_t *cols, cplx *blocks) {
  if (!problem_ok(p)) return -1;
  const int D = p->d + 1, nc = p->nc, nloc = 1 << D, nb = nc * nc;
  const int64_t S = orc_spatial_nodes(p);
  int32_t g[4] = {0, 0, 0, 0};
  g[0] = (int32_t)(r / S) + 1;
  int64_t s = r % S;
  for (int a = 1; a <= p->d; a++) { g[a] = s % p->n[a]; s /= p->n[a]; }
  int64_t lc[81];
  cplx lv[81 * 16];
  int cnt = 0;
  cplx *B = malloc(sizeof(cplx) * nloc * nloc * nb);
  for (int be = 0; be < nloc; be++) {
    /* element in which the row node is local node be */
    int32_t e[4];
    int ok = 1;
    for (int a = 0; a < D; a++) {
      int32_t c = g[a] - ((be >> a) & 1);
      if (a == 0) { if (c < 0 || c >= p->n[0]) ok = 0; }
      else c = (c + p->n[a]) % p->n[a];
      e[a] = c;
    }
    if (!ok) continue;
    orc_element_matrix(p, e, B);
    for (int al = 0; al < nloc; al++) {
      int32_t ga[4];
      local_to_global(p, e, al, ga);
      int64_t c = (ga[0] == 0) ? -spatial_index(p, ga) - 1
                               : (int64_t)(ga[0] - 1) * S + spatial_index(p, ga);
      int k;
      for (k = 0; k < cnt; k++) if (lc[k] == c) break;
      if (k == cnt) { lc[cnt] = c; memset(lv + cnt * nb, 0, sizeof(cplx) * nb); cnt++; }
      for (int q = 0; q < nb; q++) lv[k * nb + q] += B[((size_t)be * nloc + al) * nb + q];
    }
  }
  free(B);
  /* sort by column */
  for (int a = 1; a < cnt; a++) {
    int64_t tc = lc[a];
    cplx tv[16];
    memcpy(tv, lv + a * nb, sizeof(cplx) * nb);
    int b = a - 1;
    while (b >= 0 && lc[b] > tc) {
      lc[b + 1] = lc[b];
      memcpy(lv + (b + 1) * nb, lv + b * nb, sizeof(cplx) * nb);
      b--;
    }
    lc[b + 1] = tc;
    memcpy(lv + (b + 1) * nb, tv, sizeof(cplx) * nb);
  }
  memcpy(cols, lc, sizeof(int64_t) * cnt);
  memcpy(blocks, lv, sizeof(cplx) * nb * cnt);
  return cnt;
}

/* ------------------------------------------------------------- products */
void orc_spmv(const orc_matrix *A, const cplx *x, cplx *y) {
  const int nc = A->p.nc, nb = nc * nc;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < A->nrows; r++) {
    cplx acc[4] = {0, 0, 0, 0};
    for (int64_t k = A->rowptr[r]; k < A->rowptr[r + 1]; k++)
      for (int i = 0; i < nc; i++)
        for (int j = 0; j < nc; j++) acc[i] += A->val[k * nb + i * nc + j] * x[A->col[k] * nc + j];
    for (int i = 0; i < nc; i++) y[r * nc + i] = acc[i];
  }
}

/* b = -A_{:,t0} psi0 (Sec. 2.1, eq. (dirac_weakIVP)); rows outside tau = 1 are zero */
void orc_rhs(const orc_matrix *A, const cplx *psi0, cplx *b) {
  const int nc = A->p.nc, nb = nc * nc;
  memset(b, 0, sizeof(cplx) * A->nrows * nc);
  for (int64_t r = 0; r < A->nrows0; r++)
    for (int64_t k = A->rowptr0[r]; k < A->rowptr0[r + 1]; k++)
      for (int i = 0; i < nc; i++)
        for (int j = 0; j < nc; j++) b[r * nc + i] -= A->val0[k * nb + i * nc + j] * psi0[A->col0[k] * nc + j];
}

/* ---------------------------------------------------- small dense helpers */
/* Gauss-Jordan inverse with partial pivoting of an n x n complex matrix.
 * Returns 0 on success, -1 if a pivot is exactly zero. */
static int small_inverse(int n, const cplx *a, cplx *inv) {
  cplx m[16 * 2];
  for (int i = 0; i < n; i++)
    for (int j = 0; j < 2 * n; j++)
      m[i * 2 * n + j] = (j < n) ? a[i * n + j] : (j - n == i ? 1.0 : 0.0);
  for (int c = 0; c < n; c++) {
    int piv = c;
    for (int r = c + 1; r < n; r++) if (cabs(m[r * 2 * n + c]) > cabs(m[piv * 2 * n + c])) piv = r;
    if (cabs(m[piv * 2 * n + c]) == 0.0) return -1;
    if (piv != c)
      for (int j = 0; j < 2 * n; j++) { cplx t = m[c * 2 * n + j]; m[c * 2 * n + j] = m[piv * 2 * n + j]; m[piv * 2 * n + j] = t; }
    cplx d = m[c * 2 * n + c];
    for (int j = 0; j < 2 * n; j++) m[c * 2 * n + j] /= d;
    for (int r = 0; r < n; r++) {
      if (r == c) continue;
      cplx f = m[r * 2 * n + c];
      for (int j = 0; j < 2 * n; j++) m[r * 2 * n + j] -= f * m[c * 2 * n + j];
    }
  }
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) inv[i * n + j] = m[i * 2 * n + n + j];
  return 0;
}

static double norm1(int n, const cplx *a) {
  double best = 0;
  for (int j = 0; j < n; j++) {
    double s = 0;
    for (int i = 0; i < n; i++) s += cabs(a[i * n + j]);
    if (s > best) best = s;
  }
  return best;
}

/* Node-block Jacobi: inverse of each diagonal nc x nc block.  A block whose
 * 1-norm condition number exceeds 1e12 (or that is singular) is replaced by the
 * identity and counted.  Returns that count. */
int64_t orc_block_jacobi(const orc_matrix *A, cplx *inv) {
  const int nc = A->p.nc, nb = nc * nc;
  int64_t bad = 0;
  for (int64_t r = 0; r < A->nrows; r++) {
    const cplx *blk = NULL;
    for (int64_t k = A->rowptr[r]; k < A->rowptr[r + 1]; k++)
      if (A->col[k] == r) blk = A->val + k * nb;
    cplx *out = inv + r * nb;
    int ok = blk && small_inverse(nc, blk, out) == 0;
    if (ok && norm1(nc, blk) * norm1(nc, out) > 1e12) ok = 0;
    if (!ok) {
      bad++;
      for (int i = 0; i < nc; i++)
        for (int j = 0; j < nc; j++) out[i * nc + j] = (i == j) ? 1.0 : 0.0;
    }
  }
  return bad;
}

static void apply_block_jacobi(const orc_matrix *A, const cplx *inv, const cplx *in, cplx *out) {
  const int nc = A->p.nc, nb = nc * nc;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < A->nrows; r++)
    for (int i = 0; i < nc; i++) {
      cplx s = 0;
      for (int j = 0; j < nc; j++) s += inv[r * nb + i * nc + j] * in[r * nc + j];
      out[r * nc + i] = s;
    }
}

/* ------------------------------------------------- spectral solve (V const) */
/* Exact inverse of the operator with the potential replaced by a constant
 * vbar, on the periodic uniform mesh: spatial discrete Fourier transform by
 * its definition (O(n^2) per line), then, for every spatial mode, the
 * block-tridiagonal system along time solved by block Gaussian elimination
 * without pivoting (block Thomas), then the inverse transform.
 *
 * Symbols: the 1D periodic mass matrix has eigenvalue h (2 + cos th)/3 and the
 * 1D derivative matrix i sin th on the mode exp(i th j), th = 2 pi k / n. */
static void dft_axis(const orc_problem *p, int axis, int sign, cplx *v) {
  const int nc = p->nc, n = p->n[axis];
  int64_t inner = nc, outer = 1;
  for (int a = 1; a < axis; a++) inner *= p->n[a];
  for (int a = axis + 1; a <= p->d; a++) outer *= p->n[a];
  outer *= p->n[0];
  cplx *tw = malloc(sizeof(cplx) * n);
  for (int k = 0; k < n; k++) tw[k] = cexp(sign * 2.0 * M_PI * I * (double)k / (double)n);
#pragma omp parallel
  {
    cplx *line = malloc(sizeof(cplx) * n);
#pragma omp for collapse(2) schedule(static)
    for (int64_t o = 0; o < outer; o++)
      for (int64_t q = 0; q < inner; q++) {
        cplx *base = v + o * n * inner + q;
        for (int j = 0; j < n; j++) line[j] = base[(int64_t)j * inner];
        for (int k = 0; k < n; k++) {
          cplx s = 0;
          for (int j = 0; j < n; j++) s += line[j] * tw[(int64_t)j * k % n];
          base[(int64_t)k * inner] = s;
        }
      }
    free(line);
  }
  free(tw);
}

static void matmul(int n, const cplx *a, const cplx *b, cplx *c) {
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) {
      cplx s = 0;
      for (int k = 0; k < n; k++) s += a[i * n + k] * b[k * n + j];
      c[i * n + j] = s;
    }
}
static void matvec(int n, const cplx *a, const cplx *x, cplx *y) {
  for (int i = 0; i < n; i++) {
    cplx s = 0;
    for (int k = 0; k < n; k++) s += a[i * n + k] * x[k];
    y[i] = s;
  }
}

/* Per-mode time blocks: row tau couples tau-1 (L), tau (Dg) and tau+1 (U).
 * The operator restricted to a spatial mode is
 *   i g^0 mus C_t + S M_t,  S = sum_a i g^a (i sin th_a) prod_{b!=a} mu_b - (m + vbar g^0) mus,
 * with C_t rows (1/2)[-1, 0, 1] and M_t rows (h_t/6)[1, 4, 1]; the last row is
 * (1/2)[-1, 1] and (h_t/6)[1, 2]. */
static void mode_blocks(const orc_problem *p, const int32_t *k, double vbar, cplx *L, cplx *Dg,
                        cplx *Dl, cplx *U) {
  const int nc = p->nc, d = p->d;
  double mu[4], ht = p->len[0] / p->n[0];
  cplx cs[4];
  for (int a = 1; a <= d; a++) {
    double h = p->len[a] / p->n[a], th = 2.0 * M_PI * k[a] / p->n[a];
    mu[a] = h * (2.0 + cos(th)) / 3.0;
    cs[a] = I * sin(th);
  }
  double mus = 1.0;
  for (int a = 1; a <= d; a++) mus *= mu[a];
  cplx g[4][16], S[16], T[16];
  for (int a = 0; a <= d; a++) orc_gamma(d, a, g[a]);
  for (int i = 0; i < nc * nc; i++) {
    cplx s = 0;
    for (int a = 1; a <= d; a++) {
      double other = 1.0;
      for (int b = 1; b <= d; b++) if (b != a) other *= mu[b];
      s += I * g[a][i] * cs[a] * other;
    }
    s -= vbar * g[0][i] * mus;
    if (i / nc == i % nc) s -= p->m * mus;
    S[i] = s;
    T[i] = I * g[0][i] * mus;
  }
  for (int i = 0; i < nc * nc; i++) {
    L[i] = -0.5 * T[i] + ht / 6.0 * S[i];
    U[i] = 0.5 * T[i] + ht / 6.0 * S[i];
    Dg[i] = 4.0 * ht / 6.0 * S[i];
    Dl[i] = 0.5 * T[i] + 2.0 * ht / 6.0 * S[i];
  }
}

/* out = A(vbar)^{-1} in.  Returns 0, or -1 if a Thomas pivot is singular. */
int orc_spectral_solve(const orc_problem *p, double vbar, const cplx *in, cplx *out) {
  if (!problem_ok(p)) return -1;
  const int nc = p->nc, nb = nc * nc, nt = p->n[0];
  const int64_t S = orc_spatial_nodes(p), N = orc_nrows(p) * nc;
  memcpy(out, in, sizeof(cplx) * N);
  for (int a = 1; a <= p->d; a++) dft_axis(p, a, -1, out);
  int fail = 0;
#pragma omp parallel for schedule(static) reduction(| : fail)
  for (int64_t s = 0; s < S; s++) {
    int32_t k[4] = {0, 0, 0, 0};
    int64_t t = s;
    for (int a = 1; a <= p->d; a++) { k[a] = t % p->n[a]; t /= p->n[a]; }
    cplx L[16], Dg[16], Dl[16], U[16];
    mode_blocks(p, k, vbar, L, Dg, Dl, U);
    cplx *piv = malloc(sizeof(cplx) * nt * nb);  /* inverses of eliminated pivots */
    cplx *y = malloc(sizeof(cplx) * nt * nc);
    cplx tmp[16], tmp2[16], vv[4];
    for (int tau = 0; tau < nt; tau++) {
      const cplx *Dt = (tau == nt - 1) ? Dl : Dg;
      cplx Dp[16], rv[4];
      for (int i = 0; i < nc; i++) rv[i] = out[((int64_t)tau * S + s) * nc + i];
      if (tau == 0) {
        memcpy(Dp, Dt, sizeof(cplx) * nb);
      } else {
        matmul(nc, L, piv + (tau - 1) * nb, tmp);    /* L Dp^{-1}_{tau-1} */
        matmul(nc, tmp, U, tmp2);
        for (int i = 0; i < nb; i++) Dp[i] = Dt[i] - tmp2[i];
        matvec(nc, tmp, y + (tau - 1) * nc, vv);
        for (int i = 0; i < nc; i++) rv[i] -= vv[i];
      }
      if (small_inverse(nc, Dp, piv + tau * nb) != 0) fail = 1;
      memcpy(y + tau * nc, rv, sizeof(cplx) * nc);
    }
    cplx xn[4], xprev[4];
    for (int tau = nt - 1; tau >= 0; tau--) {
      cplx rv[4];
      memcpy(rv, y + tau * nc, sizeof(cplx) * nc);
      if (tau < nt - 1) {
        matvec(nc, U, xprev, vv);
        for (int i = 0; i < nc; i++) rv[i] -= vv[i];
      }
      matvec(nc, piv + tau * nb, rv, xn);
      for (int i = 0; i < nc; i++) out[((int64_t)tau * S + s) * nc + i] = xn[i];
      memcpy(xprev, xn, sizeof(cplx) * nc);
    }
    free(piv);
    free(y);
  }
  for (int a = 1; a <= p->d; a++) dft_axis(p, a, +1, out);
  double scale = 1.0 / (double)S;
  for (int64_t i = 0; i < N; i++) out[i] *= scale;
  return fail ? -1 : 0;
}

/* ------------------------------------------------------------------ GMRES */
typedef void (*orc_pc_fn)(const cplx *in, cplx *out, void *ctx);

typedef struct {
  int32_t iters, restarts, converged, breakdown;
  double relres;      /* true relative residual at exit */
  double est;         /* last Arnoldi residual estimate / ||b|| */
} orc_stats;

static double vnorm(int64_t n, const cplx *x) {
  double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t i = 0; i < n; i++) s += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
  return sqrt(s);
}

static cplx vdot(int64_t n, const cplx *u, const cplx *v) {  /* sum conj(u) v */
  double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
  for (int64_t i = 0; i < n; i++) {
    cplx t = conj(u[i]) * v[i];
    re += creal(t);
    im += cimag(t);
  }
  return re + I * im;
}

typedef struct {
  const orc_matrix *A;
  int kind;           /* 0 none, 1 node-block Jacobi, 2 spectral(vbar), 3 callback */
  cplx *bj;
  double vbar;
  orc_pc_fn fn;
  void *ctx;
} pc_state;

static void pc_apply(pc_state *pc, const cplx *in, cplx *out, int64_t N) {
  if (pc->kind == 1) apply_block_jacobi(pc->A, pc->bj, in, out);
  else if (pc->kind == 2) orc_spectral_solve(&pc->A->p, pc->vbar, in, out);
  else if (pc->kind == 3) pc->fn(in, out, pc->ctx);
  else memcpy(out, in, sizeof(cplx) * N);
}

/* Restarted GMRES(m) / FGMRES(m) with right preconditioning, CGS2 and complex
 * Givens rotations.  x holds the initial guess on entry.  hist (may be NULL,
 * length >= max_it) receives the residual estimate / ||b|| after every
 * Arnoldi step.  flexible != 0 keeps the preconditioned vectors Z and updates
 * x += Z y; otherwise x += M^{-1} (V y). */
int orc_gmres(const orc_matrix *A, int pc_kind, double vbar, orc_pc_fn fn, void *ctx,
              const cplx *b, cplx *x, int restart, int max_it, double rtol, int flexible,
              orc_stats *st, double *hist) {
  const int nc = A->p.nc;
  const int64_t N = A->nrows * nc;
  const int m = restart;
  pc_state pc = {A, pc_kind, NULL, vbar, fn, ctx};
  if (pc_kind == 1) {
    pc.bj = malloc(sizeof(cplx) * A->nrows * nc * nc);
    orc_block_jacobi(A, pc.bj);
  }
  cplx *V = malloc(sizeof(cplx) * N * (m + 1));
  cplx *Z = flexible ? malloc(sizeof(cplx) * N * m) : NULL;
  cplx *w = malloc(sizeof(cplx) * N), *z = malloc(sizeof(cplx) * N), *r = malloc(sizeof(cplx) * N);
  cplx *H = calloc((size_t)(m + 1) * m, sizeof(cplx));  /* H[i*m + j] */
  cplx *cs = malloc(sizeof(cplx) * m), *sn = malloc(sizeof(cplx) * m), *g = malloc(sizeof(cplx) * (m + 1));
  cplx *yv = malloc(sizeof(cplx) * m), *h1 = malloc(sizeof(cplx) * (m + 1));
  memset(st, 0, sizeof(*st));
  double bnorm = vnorm(N, b);
  if (bnorm == 0.0) {
    memset(x, 0, sizeof(cplx) * N);
    st->converged = 1;
    goto done;
  }
  int its = 0;
  for (;;) {
    /* true residual */
    orc_spmv(A, x, r);
    for (int64_t i = 0; i < N; i++) r[i] = b[i] - r[i];
    double beta = vnorm(N, r);
    st->relres = beta / bnorm;
    if (!isfinite(beta)) { st->breakdown = 1; break; }
    if (st->relres <= rtol) { st->converged = 1; break; }
    if (its >= max_it) break;
    st->restarts++;
    for (int64_t i = 0; i < N; i++) V[i] = r[i] / beta;
    memset(H, 0, sizeof(cplx) * (m + 1) * m);
    memset(g, 0, sizeof(cplx) * (m + 1));
    g[0] = beta;
    int k = 0, stop = 0;
    for (int j = 0; j < m && its < max_it; j++) {
      cplx *vj = V + (int64_t)j * N, *zj = flexible ? Z + (int64_t)j * N : z;
      pc_apply(&pc, vj, zj, N);
      orc_spmv(A, zj, w);
      double w0 = vnorm(N, w);
      /* CGS2: two full classical Gram-Schmidt passes */
      for (int pass = 0; pass < 2; pass++) {
        for (int i = 0; i <= j; i++) h1[i] = vdot(N, V + (int64_t)i * N, w);
        for (int i = 0; i <= j; i++) {
          const cplx *vi = V + (int64_t)i * N;
#pragma omp parallel for schedule(static)
          for (int64_t q = 0; q < N; q++) w[q] -= h1[i] * vi[q];
          H[i * m + j] += h1[i];
        }
      }
      double hn = vnorm(N, w);
      H[(j + 1) * m + j] = hn;
      its++;
      k = j + 1;
      int happy = hn <= 1e-14 * w0;
      if (!happy)
        for (int64_t q = 0; q < N; q++) V[(int64_t)(j + 1) * N + q] = w[q] / hn;
      /* apply previous rotations to column j */
      for (int i = 0; i < j; i++) {
        cplx a = H[i * m + j], bb = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * bb;
        H[(i + 1) * m + j] = -conj(sn[i]) * a + cs[i] * bb;
      }
      /* new rotation zeroing H[j+1][j] */
      {
        cplx a = H[j * m + j], bb = H[(j + 1) * m + j];
        double rho = sqrt(creal(a) * creal(a) + cimag(a) * cimag(a) + creal(bb) * creal(bb) + cimag(bb) * cimag(bb));
        cplx c, s;
        if (cabs(a) == 0.0) { c = 0.0; s = 1.0; }
        else { c = cabs(a) / rho; s = (a / cabs(a)) * conj(bb) / rho; }
        cs[j] = c; sn[j] = s;
        H[j * m + j] = c * a + s * bb;
        H[(j + 1) * m + j] = 0.0;
        cplx gj = g[j];
        g[j] = c * gj;
        g[j + 1] = -conj(s) * gj;
      }
      double est = cabs(g[j + 1]) / bnorm;
      st->est = est;
      if (hist) hist[its - 1] = est;
      if (!isfinite(est)) { st->breakdown = 1; stop = 1; break; }
      if (est <= rtol || happy) { stop = 1; break; }
    }
    (void)stop;
    /* back substitution R y = g */
    for (int i = k - 1; i >= 0; i--) {
      cplx s = g[i];
      for (int q = i + 1; q < k; q++) s -= H[i * m + q] * yv[q];
      yv[i] = s / H[i * m + i];
    }
    if (flexible) {
      for (int i = 0; i < k; i++) {
        const cplx *zi = Z + (int64_t)i * N;
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < N; q++) x[q] += yv[i] * zi[q];
      }
    } else {
      memset(w, 0, sizeof(cplx) * N);
      for (int i = 0; i < k; i++) {
        const cplx *vi = V + (int64_t)i * N;
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < N; q++) w[q] += yv[i] * vi[q];
      }
      pc_apply(&pc, w, z, N);
      for (int64_t q = 0; q < N; q++) x[q] += z[q];
    }
    if (st->breakdown) break;
  }
  st->iters = its;
done:
  free(V); free(Z); free(w); free(z); free(r); free(H); free(cs); free(sn); free(g); free(yv); free(h1);
  free(pc.bj);
  return st->converged ? 0 : (st->breakdown ? -3 : 1);
}

/* ---------------------------------------------------------------- BiCGSTAB */
/* BiCGSTAB (van der Vorst, SIAM J. Sci. Stat. Comput. 13 (1992)), the second
 * Krylov solver of the paper's parallel runs (Sec. 4.4, Tables 1-3), with right
 * preconditioning so that r is the residual of the original system:
 *   r = b - A x, rh = r, rho_old = alpha = omega = 1, p = v = 0
 *   each iteration:
 *     rho = rh^H r;  beta = (rho / rho_old) (alpha / omega)
 *     p = r + beta (p - omega v);  ph = M^{-1} p;  v = A ph
 *     alpha = rho / (rh^H v);  s = r - alpha v
 *     sh = M^{-1} s;  t = A sh;  omega = (t^H s) / (t^H t)  (0 if t = 0)
 *     x += alpha ph + omega sh;  r = s - omega t
 * The stop test uses the updated residual; when it passes, the true residual
 * b - A x decides, and if that fails (the two drifted apart) the iteration
 * restarts from the true residual with rh = r.  A zero rho or rh^H v also
 * restarts (from the true residual); a restart that is immediately hit again
 * ends the solve as a breakdown.  hist (may be NULL, length >= max_it)
 * receives ||r|| / ||b|| after every iteration; st->restarts counts the starts. */
int orc_bicgstab(const orc_matrix *A, int pc_kind, double vbar, orc_pc_fn fn, void *ctx,
                 const cplx *b, cplx *x, int max_it, double rtol, orc_stats *st, double *hist) {
  const int nc = A->p.nc;
  const int64_t N = A->nrows * nc;
  pc_state pc = {A, pc_kind, NULL, vbar, fn, ctx};
  if (pc_kind == 1) {
    pc.bj = malloc(sizeof(cplx) * A->nrows * nc * nc);
    orc_block_jacobi(A, pc.bj);
  }
  cplx *r = malloc(sizeof(cplx) * N), *rh = malloc(sizeof(cplx) * N), *p = malloc(sizeof(cplx) * N);
  cplx *v = malloc(sizeof(cplx) * N), *ph = malloc(sizeof(cplx) * N), *s = malloc(sizeof(cplx) * N);
  cplx *sh = malloc(sizeof(cplx) * N), *t = malloc(sizeof(cplx) * N);
  memset(st, 0, sizeof(*st));
  const double bnorm = vnorm(N, b);
  int its = 0, fresh = 0;
  cplx rho_old = 1, alpha = 1, omega = 1;
  if (bnorm == 0.0) {
    memset(x, 0, sizeof(cplx) * N);
    st->converged = 1;
    goto done;
  }
  for (;;) {
    /* (re)start from the true residual */
    orc_spmv(A, x, r);
    for (int64_t i = 0; i < N; i++) r[i] = b[i] - r[i];
    const double rn = vnorm(N, r);
    st->relres = rn / bnorm;
    if (!isfinite(rn)) { st->breakdown = 1; break; }
    if (st->relres <= rtol) { st->converged = 1; break; }
    if (its >= max_it) break;
    if (fresh) { st->breakdown = 1; break; }  /* restarted and broke down at once */
    st->restarts++;
    fresh = 1;
    memcpy(rh, r, sizeof(cplx) * N);
    memset(p, 0, sizeof(cplx) * N);
    memset(v, 0, sizeof(cplx) * N);
    rho_old = alpha = omega = 1;
    int restart = 0;
    while (its < max_it) {
      const cplx rho = vdot(N, rh, r);
      if (rho == 0) { restart = 1; break; }
      const cplx beta = (rho / rho_old) * (alpha / omega);
      for (int64_t i = 0; i < N; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
      pc_apply(&pc, p, ph, N);
      orc_spmv(A, ph, v);
      const cplx rv = vdot(N, rh, v);
      if (rv == 0) { restart = 1; break; }
      alpha = rho / rv;
      for (int64_t i = 0; i < N; i++) s[i] = r[i] - alpha * v[i];
      pc_apply(&pc, s, sh, N);
      orc_spmv(A, sh, t);
      const double tt = creal(vdot(N, t, t));
      omega = tt > 0.0 ? vdot(N, t, s) / tt : 0.0;
      for (int64_t i = 0; i < N; i++) {
        x[i] += alpha * ph[i] + omega * sh[i];
        r[i] = s[i] - omega * t[i];
      }
      rho_old = rho;
      its++;
      fresh = 0;
      const double est = vnorm(N, r) / bnorm;
      st->est = est;
      if (hist) hist[its - 1] = est;
      if (!isfinite(est)) { st->breakdown = 1; break; }
      if (est <= rtol) { restart = 1; break; }
      if (omega == 0) { restart = 1; break; }
    }
    if (st->breakdown) break;
    if (!restart && its >= max_it) {
      /* cap reached inside the loop: report the true residual */
      orc_spmv(A, x, r);
      for (int64_t i = 0; i < N; i++) r[i] = b[i] - r[i];
      st->relres = vnorm(N, r) / bnorm;
      st->converged = st->relres <= rtol;
      break;
    }
  }
  st->iters = its;
done:
  free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t);
  free(pc.bj);
  return st->converged ? 0 : (st->breakdown ? -3 : 1);
}

/* Dense copy of the block matrix (tiny meshes only) for checks against a
 * textbook dense solver. */
void orc_dense(const orc_matrix *A, cplx *dense) {
  const int nc = A->p.nc, nb = nc * nc;
  const int64_t N = A->nrows * nc;
  memset(dense, 0, sizeof(cplx) * N * N);
  for (int64_t r = 0; r < A->nrows; r++)
    for (int64_t k = A->rowptr[r]; k < A->rowptr[r + 1]; k++)
      for (int i = 0; i < nc; i++)
        for (int j = 0; j < nc; j++)
          dense[(r * nc + i) * N + A->col[k] * nc + j] += A->val[k * nb + i * nc + j];
}

/* Dense LU with partial pivoting, solving a x = b in place (a is destroyed).
 * Returns 0 or -1 on an exactly zero pivot. */
int orc_dense_solve(int64_t n, cplx *a, cplx *b) {
  for (int64_t c = 0; c < n; c++) {
    int64_t piv = c;
    for (int64_t r = c + 1; r < n; r++) if (cabs(a[r * n + c]) > cabs(a[piv * n + c])) piv = r;
    if (cabs(a[piv * n + c]) == 0.0) return -1;
    if (piv != c) {
      for (int64_t j = 0; j < n; j++) { cplx t = a[c * n + j]; a[c * n + j] = a[piv * n + j]; a[piv * n + j] = t; }
      cplx t = b[c]; b[c] = b[piv]; b[piv] = t;
    }
    for (int64_t r = c + 1; r < n; r++) {
      cplx f = a[r * n + c] / a[c * n + c];
      if (f == 0) continue;
      for (int64_t j = c; j < n; j++) a[r * n + j] -= f * a[c * n + j];
      b[r] -= f * b[c];
    }
  }
  for (int64_t i = n - 1; i >= 0; i--) {
    cplx s = b[i];
    for (int64_t j = i + 1; j < n; j++) s -= a[i * n + j] * b[j];
    b[i] = s / a[i * n + i];
  }
  return 0;
}
