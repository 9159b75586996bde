/*
 * hmat_oracle.c -- plain FP64 CPU oracle for the collocation single-layer
 * H-matrix path of Bauer & Bebendorf, "Adaptive H-Matrix Computations in
 * Linear Elasticity" (arXiv 2205.04752).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no source
 * with the HIP path (paper_2205_04752_amd/) and includes none of its headers.
 * It is deliberately slow and literal: every routine follows the definition
 * it cites, with no blocking, fusion or reordering beyond that definition.
 *
 * What it computes (each item names the passage it follows):
 *   - Kelvin fundamental solution S_K (Sec. 4.1, Kelvin's solution tensor).
 *   - Collocation entries for piecewise-constant trial functions
 *     (Sec. 2, collocation method; Sec. 4.2, basis of S^0_h; DOF order
 *     t = [t_i^(1), t_i^(2), t_i^(3)]_i, so DOF 3i+a).
 *       j != i : degree-5 seven-point rule of Radon (Stroud T2:5-1).
 *       j == i : the triangle is split at the collocation point into three
 *                sub-triangles, each mapped to the unit square by Duffy's
 *                transformation, with n x n Gauss-Legendre points (n = 16).
 *   - Cluster tree by bounding-box bisection (Sec. 2.1, binary cluster tree),
 *     admissibility min(diam X_t, diam X_s) <= eta dist(X_t, X_s) with
 *     dist > 0 (Sec. 2.1, eq. adm), block partition as the leaves of the
 *     block-cluster tree (Sec. 2.1), sparsity constant c_sp (Sec. 2.1).
 *   - ACA with partial pivoting (Sec. 2.2, Algorithm 1), stop rule read as
 *     ||u_k|| ||v_k|| <= eps ||S_k||_F (the printed constant is negative for
 *     eta >= 1), pivot ties broken by a fuzzy argmax, vanishing rows
 *     collected in Z.
 *   - H-matrix-vector product y = sum_far U_b (V_b^T x_s) + sum_near D_b x_s
 *     (Sec. 2, outer-product representation; Sec. 2.2, H(P,k)).
 *   - Dense assembly and a matrix-free brute-force product y = A x.
 *   - GMRES(m) of Saad and Schultz (modified Gram-Schmidt, Givens rotations,
 *     x0 = 0, convergence on the explicit residual) -- not in the paper,
 *     which solves its saddle-point system with Bramble-Pasciak CG.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (see build.py).
 * -ffp-contract=off keeps the geometry and the admissibility test in plain
 * IEEE binary64 arithmetic, operation by operation as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int or_version(void) { return 1; }

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Kelvin's solution tensor (Sec. 4.1):
 *   S_ab(r) = 1/(8 pi) (1/E) (1+nu)/(1-nu) [ (3-4nu) delta_ab/|r| + r_a r_b/|r|^3 ]
 * for r != 0. Output row-major 3x3. */
void or_kelvin(const double r[3], double E, double nu, double S[9]) {
  double cK = (1.0 / (8.0 * OR_PI)) * (1.0 / E) * ((1.0 + nu) / (1.0 - nu));
  double rho = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  double rho3 = rho * rho * rho;
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      double d = (a == b) ? 1.0 : 0.0;
      S[3 * a + b] = cK * ((3.0 - 4.0 * nu) * d / rho + r[a] * r[b] / rho3);
    }
}

/* ------------------------------------------------------------------------ */
/* Radon's degree-5 seven-point rule on a triangle (Stroud T2:5-1), given as
 * barycentric points and weights summing to 1:
 *   (1/3,1/3,1/3) with 9/40;
 *   the three placements of (a1,b1,b1), b1 = (6+sqrt15)/21, a1 = 1-2 b1, weight (155+sqrt15)/1200;
 *   the three placements of (a2,b2,b2), b2 = (6-sqrt15)/21, a2 = 1-2 b2, weight (155-sqrt15)/1200.
 * Placement order: vertex 0 carries a, then vertex 1, then vertex 2. */
void or_rule_radon7(double bary[21], double w[7]) {
  double s15 = sqrt(15.0);
  double b1 = (6.0 + s15) / 21.0, a1 = 1.0 - 2.0 * b1;
  double b2 = (6.0 - s15) / 21.0, a2 = 1.0 - 2.0 * b2;
  double w1 = (155.0 + s15) / 1200.0, w2 = (155.0 - s15) / 1200.0;
  bary[0] = bary[1] = bary[2] = 1.0 / 3.0;
  w[0] = 9.0 / 40.0;
  for (int m = 0; m < 3; m++) {
    for (int c = 0; c < 3; c++) {
      bary[3 * (1 + m) + c] = (c == m) ? a1 : b1;
      bary[3 * (4 + m) + c] = (c == m) ? a2 : b2;
    }
    w[1 + m] = w1;
    w[4 + m] = w2;
  }
}

/* n-point Gauss-Legendre rule on [-1,1]: nodes are the roots of P_n, found by
 * Newton's method on the three-term recurrence
 *   (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1};
 * weights w = 2 / ((1-x^2) P_n'(x)^2). Nodes ascending. */
void or_gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; i++) {
    /* i-th root counted from the right end */
    double z = cos(OR_PI * ((double)i + 0.75) / ((double)n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; it++) {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < n; k++) {
        double p2 = ((2.0 * k + 1.0) * z * p1 - (double)k * p0) / (double)(k + 1);
        p0 = p1;
        p1 = p2;
      }
      /* p1 = P_n(z), p0 = P_{n-1}(z) */
      dp = (double)n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < n; k++) {
        double p2 = ((2.0 * k + 1.0) * z * p1 - (double)k * p0) / (double)(k + 1);
        p0 = p1;
        p1 = p2;
      }
      dp = (double)n * (z * p1 - p0) / (z * z - 1.0);
    }
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

/* ------------------------------------------------------------------------ */
/* Mesh context: geometry of the triangulation (Sec. 4.2) and material. */
typedef struct {
  int nv, nt;
  double* V;    /* [nv][3] */
  int* T;       /* [nt][3] */
  double E, nu;
  double* cen;  /* [nt][3] collocation points (centroids) */
  double* area; /* [nt] */
  double* qn;   /* [nt][7][3] quadrature nodes */
  double* qw;   /* [nt][7] weights times area */
  int ngl;      /* Gauss-Legendre order for the self term */
  double glx[64], glw[64]; /* rule on [0,1] */
} or_ctx;

/* Centroid ((p0+p1)+p2)/3 and area |(p1-p0) x (p2-p0)|/2 of triangle i. */
static void tri_geometry(const or_ctx* c, int i, double cen[3], double* area) {
  const double* p0 = c->V + 3 * c->T[3 * i + 0];
  const double* p1 = c->V + 3 * c->T[3 * i + 1];
  const double* p2 = c->V + 3 * c->T[3 * i + 2];
  for (int d = 0; d < 3; d++) cen[d] = ((p0[d] + p1[d]) + p2[d]) / 3.0;
  double e1[3], e2[3], n[3];
  for (int d = 0; d < 3; d++) {
    e1[d] = p1[d] - p0[d];
    e2[d] = p2[d] - p0[d];
  }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  *area = 0.5 * sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
}

static void set_gl(or_ctx* c, int n) {
  double x[64], w[64];
  or_gauss_legendre(n, x, w);
  for (int k = 0; k < n; k++) {
    c->glx[k] = 0.5 * (1.0 + x[k]);
    c->glw[k] = 0.5 * w[k];
  }
  c->ngl = n;
}

/* Returns NULL on invalid input (index out of range, zero-area triangle). */
or_ctx* or_ctx_new(int nv, int nt, const double* V, const int* T, double E, double nu) {
  if (nv <= 0 || nt <= 0) return NULL;
  for (int i = 0; i < 3 * nt; i++)
    if (T[i] < 0 || T[i] >= nv) return NULL;
  or_ctx* c = (or_ctx*)calloc(1, sizeof(or_ctx));
  c->nv = nv;
  c->nt = nt;
  c->E = E;
  c->nu = nu;
  c->V = (double*)malloc(sizeof(double) * 3 * nv);
  c->T = (int*)malloc(sizeof(int) * 3 * nt);
  memcpy(c->V, V, sizeof(double) * 3 * nv);
  memcpy(c->T, T, sizeof(int) * 3 * nt);
  c->cen = (double*)malloc(sizeof(double) * 3 * nt);
  c->area = (double*)malloc(sizeof(double) * nt);
  c->qn = (double*)malloc(sizeof(double) * 21 * nt);
  c->qw = (double*)malloc(sizeof(double) * 7 * nt);
  double bary[21], w[7];
  or_rule_radon7(bary, w);
  for (int i = 0; i < nt; i++) {
    tri_geometry(c, i, c->cen + 3 * i, c->area + i);
    if (!(c->area[i] > 0.0)) {
      free(c->V); free(c->T); free(c->cen); free(c->area); free(c->qn); free(c->qw); free(c);
      return NULL;
    }
    const double* p0 = c->V + 3 * c->T[3 * i + 0];
    const double* p1 = c->V + 3 * c->T[3 * i + 1];
    const double* p2 = c->V + 3 * c->T[3 * i + 2];
    for (int q = 0; q < 7; q++) {
      for (int d = 0; d < 3; d++)
        c->qn[21 * i + 3 * q + d] =
            (bary[3 * q + 0] * p0[d] + bary[3 * q + 1] * p1[d]) + bary[3 * q + 2] * p2[d];
      c->qw[7 * i + q] = w[q] * c->area[i];
    }
  }
  set_gl(c, 16);
  return c;
}

void or_ctx_free(or_ctx* c) {
  if (!c) return;
  free(c->V); free(c->T); free(c->cen); free(c->area); free(c->qn); free(c->qw);
  free(c);
}

void or_ctx_set_self_order(or_ctx* c, int n) {
  if (n >= 1 && n <= 64) set_gl(c, n);
}

void or_ctx_geometry(const or_ctx* c, double* cen, double* area, double* qn, double* qw) {
  if (cen) memcpy(cen, c->cen, sizeof(double) * 3 * c->nt);
  if (area) memcpy(area, c->area, sizeof(double) * c->nt);
  if (qn) memcpy(qn, c->qn, sizeof(double) * 21 * c->nt);
  if (qw) memcpy(qw, c->qw, sizeof(double) * 7 * c->nt);
}

/* Self term: integral over tau_i of S(c_i - y) dy. tau_i is split at c into
 * T_m = (c, p_m, p_{m+1}); on T_m, y(s,t) = c + s[(p_m - c) + t(p_{m+1} - p_m)]
 * with Jacobian 2|T_m| s, s,t in [0,1], Gauss-Legendre in s and t. */
static void self_block(const or_ctx* c, int i, double out[9]) {
  const double* x = c->cen + 3 * i;
  for (int k = 0; k < 9; k++) out[k] = 0.0;
  for (int m = 0; m < 3; m++) {
    const double* pa = c->V + 3 * c->T[3 * i + m];
    const double* pb = c->V + 3 * c->T[3 * i + (m + 1) % 3];
    double ea[3], eb[3], n[3];
    for (int d = 0; d < 3; d++) {
      ea[d] = pa[d] - x[d];
      eb[d] = pb[d] - pa[d];
    }
    n[0] = ea[1] * eb[2] - ea[2] * eb[1];
    n[1] = ea[2] * eb[0] - ea[0] * eb[2];
    n[2] = ea[0] * eb[1] - ea[1] * eb[0];
    double jac2 = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]); /* = 2 |T_m| */
    for (int ks = 0; ks < c->ngl; ks++) {
      double s = c->glx[ks];
      for (int kt = 0; kt < c->ngl; kt++) {
        double t = c->glx[kt];
        double y[3], r[3], S[9];
        for (int d = 0; d < 3; d++) {
          y[d] = x[d] + s * (ea[d] + t * eb[d]);
          r[d] = x[d] - y[d];
        }
        or_kelvin(r, c->E, c->nu, S);
        double wgt = c->glw[ks] * c->glw[kt] * jac2 * s;
        for (int k = 0; k < 9; k++) out[k] += wgt * S[k];
      }
    }
  }
}

/* A[3i+a, 3j+b] for a,b = 0..2 (row-major 3x3): collocation at c_i of the
 * piecewise-constant basis function of tau_j (Sec. 2, collocation; Sec. 4.2). */
void or_entry_block(const or_ctx* c, int i, int j, double out[9]) {
  if (i == j) {
    self_block(c, i, out);
    return;
  }
  const double* x = c->cen + 3 * i;
  for (int k = 0; k < 9; k++) out[k] = 0.0;
  for (int q = 0; q < 7; q++) {
    double r[3], S[9];
    for (int d = 0; d < 3; d++) r[d] = x[d] - c->qn[21 * j + 3 * q + d];
    or_kelvin(r, c->E, c->nu, S);
    for (int k = 0; k < 9; k++) out[k] += c->qw[7 * j + q] * S[k];
  }
}

/* Arbitrary DOF entries A[rows[k], cols[k]]. */
void or_entries(const or_ctx* c, int n, const int64_t* rows, const int64_t* cols, double* out) {
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n; k++) {
    double b[9];
    int64_t r = rows[k], s = cols[k];
    or_entry_block(c, (int)(r / 3), (int)(s / 3), b);
    out[k] = b[3 * (r % 3) + (s % 3)];
  }
}

/* Dense A (3nt x 3nt, row-major). */
void or_dense(const or_ctx* c, double* A) {
  int64_t N = 3 * (int64_t)c->nt;
#pragma omp parallel for schedule(dynamic, 4)
  for (int i = 0; i < c->nt; i++) {
    for (int j = 0; j < c->nt; j++) {
      double b[9];
      or_entry_block(c, i, j, b);
      for (int a = 0; a < 3; a++)
        for (int d = 0; d < 3; d++) A[(3 * (int64_t)i + a) * N + 3 * (int64_t)j + d] = b[3 * a + d];
    }
  }
}

/* Matrix-free y_r = A x_r for the triangles listed in tri_rows (all if NULL),
 * nrhs vectors of length 3nt with leading dimension 3nt; y is [nrhs][3*nrows]. */
void or_brute_matvec_rows(const or_ctx* c, int nrows, const int* tri_rows, int nrhs,
                          const double* x, double* y) {
  int64_t N = 3 * (int64_t)c->nt;
  int n = tri_rows ? nrows : c->nt;
#pragma omp parallel for schedule(dynamic, 8)
  for (int ii = 0; ii < n; ii++) {
    int i = tri_rows ? tri_rows[ii] : ii;
    double* acc = (double*)calloc(3 * (size_t)nrhs, sizeof(double));
    for (int j = 0; j < c->nt; j++) {
      double b[9];
      or_entry_block(c, i, j, b);
      for (int r = 0; r < nrhs; r++)
        for (int a = 0; a < 3; a++)
          for (int d = 0; d < 3; d++) acc[3 * r + a] += b[3 * a + d] * x[r * N + 3 * (int64_t)j + d];
    }
    for (int r = 0; r < nrhs; r++)
      for (int a = 0; a < 3; a++) y[(int64_t)r * 3 * n + 3 * (int64_t)ii + a] = acc[3 * r + a];
    free(acc);
  }
}

/* ------------------------------------------------------------------------ */
/* ACA with partial pivoting (Sec. 2.2, Algorithm 1) on an m x n block given
 * by row and column callbacks. Conventions:
 *   - first row i_1 = 0; later rows i_{k+1} = fuzzy argmax over rows not in
 *     Z of |u_k|;
 *   - column j_k = fuzzy argmax of |v~_k|;
 *   - fuzzy argmax = lowest index whose magnitude is >= (1 - 1e-10) * max;
 *   - v~ vanishes if max|v~| == 0 (k = 0) or max|v~| <= 1e-14 ||S_k||_F;
 *   - ||S_k||_F^2 = ||S_{k-1}||_F^2 + 2 sum_{l<k} (u_l.u_k)(v_l.v_k) + |u_k|^2 |v_k|^2;
 *   - stop when |u_k| |v_k| <= eps ||S_k||_F (cross kept), when k = min(m,n),
 *     or when Z holds every row;
 *   - rows fall into ncls classes (row i in class i mod ncls: the three
 *     displacement components of a tensor block; 1 for a plain matrix). The
 *     accuracy test only stops ACA once every class has had a row in Z.
 *     Otherwise the next row is the lowest unused row of the lowest class
 *     not yet visited; if that row's remainder vanishes, the test counts as
 *     passed. (On coplanar clusters the Kelvin tensor decouples into
 *     in-plane and normal parts, and pivoting that never visits one class
 *     would miss its part of the block.)
 *   - cycle = 1 (step-limited runs only, eps = 0): the row rule of
 *     cycle_next below replaces partial pivoting and the class probes.
 * U is m x k and V is n x k, both column-major, returned through *pU / *pV
 * (malloc'd, grown as needed). Pivots are recorded in prow/pcol (capacity
 * min(m,n)). stop: 1 = threshold, 2 = rank = min(m,n), 3 = Z full. */
typedef void (*or_rowfn)(void* u, int i, double* out);
typedef void (*or_colfn)(void* u, int j, double* out);

static int fuzzy_argmax(const double* v, int n, const unsigned char* skip) {
  double mx = -1.0;
  for (int i = 0; i < n; i++)
    if (!(skip && skip[i]) && fabs(v[i]) > mx) mx = fabs(v[i]);
  if (mx < 0.0) return -1;
  double thr = (1.0 - 1e-10) * mx;
  for (int i = 0; i < n; i++)
    if (!(skip && skip[i]) && fabs(v[i]) >= thr) return i;
  return -1;
}

/* Lowest unused row of the lowest row class not in `visited`; -1 if none. */
static int class_probe(const unsigned char* Z, int m, int ncls, int visited) {
  for (int c = 0; c < ncls; c++) {
    if (visited & (1 << c)) continue;
    for (int r = c; r < m; r += ncls)
      if (!Z[r]) return r;
  }
  return -1;
}

/* Row rule of the step-limited runs (cycle = 1; the adaptive
 * multiplication's look-ahead, which has no accuracy test that could send ACA
 * to an unvisited class): the rows cycle through the classes. After a step at
 * row i -- a new cross, or a row whose remainder vanished -- the next row
 * comes from the first class c among i+1, i+2, i (mod ncls) that still has
 * rows outside Z: the fuzzy argmax over those rows of |u_l|, where u_l is the
 * latest cross whose largest magnitude on those rows exceeds 1e-12 times its
 * largest magnitude over all rows; if no cross qualifies, the lowest of
 * those rows. Returns -1 when Z holds every row. On coplanar clusters the
 * classes of the in-plane and normal components are decoupled, and each
 * gets its share of the steps; on coupled blocks u_l is the latest cross, as
 * in plain partial pivoting, restricted to the class. */
static int cycle_next(const double* U, int k, int m, const unsigned char* Z, int ncls, int i) {
  for (int dc = 1; dc <= ncls; dc++) {
    const int c = (i % ncls + dc) % ncls;
    int lowest = -1;
    for (int r = c; r < m; r += ncls)
      if (!Z[r]) { lowest = r; break; }
    if (lowest < 0) continue;
    for (int l = k - 1; l >= 0; l--) {
      const double* u = U + (size_t)l * m;
      double all = 0.0, cls = 0.0;
      for (int r = 0; r < m; r++)
        if (fabs(u[r]) > all) all = fabs(u[r]);
      for (int r = c; r < m; r += ncls)
        if (!Z[r] && fabs(u[r]) > cls) cls = fabs(u[r]);
      if (!(cls > 1e-12 * all)) continue;
      const double thr = (1.0 - 1e-10) * cls;
      for (int r = c; r < m; r += ncls)
        if (!Z[r] && fabs(u[r]) >= thr) return r;
    }
    return lowest;
  }
  return -1;
}

static int aca_core(int m, int n, or_rowfn rowf, or_colfn colf, void* user, double eps,
                    int kcap, int ncls, int cycle, double** pU, double** pV, int* prow, int* pcol,
                    int* stop, double* ratio) {
  int kmax = m < n ? m : n;
  const int allcls = (1 << ncls) - 1;
  int visited = 0, pending = 0;
  int cap = 8 < kmax ? 8 : kmax;
  double* U = (double*)malloc(sizeof(double) * (size_t)m * cap);
  double* V = (double*)malloc(sizeof(double) * (size_t)n * cap);
  unsigned char* Z = (unsigned char*)calloc((size_t)m, 1);
  double* vt = (double*)malloc(sizeof(double) * n);
  double* ut = (double*)malloc(sizeof(double) * m);
  int nZ = 0, k = 0, i = 0;
  double S2 = 0.0;
  *stop = 0;
  *ratio = 0.0;
  for (;;) {
    rowf(user, i, vt);
    for (int l = 0; l < k; l++) {
      double uil = U[(size_t)l * m + i];
      for (int c = 0; c < n; c++) vt[c] -= uil * V[(size_t)l * n + c];
    }
    if (!Z[i]) { Z[i] = 1; nZ++; }
    visited |= 1 << (i % ncls);
    double mx = 0.0;
    for (int c = 0; c < n; c++)
      if (fabs(vt[c]) > mx) mx = fabs(vt[c]);
    int vanished = (k == 0) ? (mx == 0.0) : (mx <= 1e-14 * sqrt(S2));
    if (vanished) {
      if (nZ == m) { *stop = 3; break; }
      if (pending && visited == allcls) { *stop = 1; break; }
      if (cycle) {
        i = cycle_next(U, k, m, Z, ncls, i);
      } else if (pending) {
        i = class_probe(Z, m, ncls, visited);
        if (i < 0) { *stop = 1; break; }
      } else if (k == 0) {
        i = 0;
        while (Z[i]) i++;
      } else {
        i = fuzzy_argmax(U + (size_t)(k - 1) * m, m, Z);
      }
      continue;
    }
    int j = fuzzy_argmax(vt, n, NULL);
    double piv = vt[j];
    if (k == cap) {
      cap = (2 * cap < kmax) ? 2 * cap : kmax;
      U = (double*)realloc(U, sizeof(double) * (size_t)m * cap);
      V = (double*)realloc(V, sizeof(double) * (size_t)n * cap);
    }
    double* v = V + (size_t)k * n;
    for (int c = 0; c < n; c++) v[c] = vt[c] / piv;
    colf(user, j, ut);
    for (int l = 0; l < k; l++) {
      double vjl = V[(size_t)l * n + j];
      for (int r = 0; r < m; r++) ut[r] -= vjl * U[(size_t)l * m + r];
    }
    double* u = U + (size_t)k * m;
    memcpy(u, ut, sizeof(double) * m);
    prow[k] = i;
    pcol[k] = j;
    double uu = 0.0, vv = 0.0, cross = 0.0;
    for (int r = 0; r < m; r++) uu += u[r] * u[r];
    for (int c = 0; c < n; c++) vv += v[c] * v[c];
    for (int l = 0; l < k; l++) {
      double a = 0.0, b = 0.0;
      for (int r = 0; r < m; r++) a += U[(size_t)l * m + r] * u[r];
      for (int c = 0; c < n; c++) b += V[(size_t)l * n + c] * v[c];
      cross += a * b;
    }
    k++;
    S2 = S2 + 2.0 * cross + uu * vv;
    double lhs = sqrt(uu) * sqrt(vv), rhs = eps * sqrt(S2);
    *ratio = rhs > 0.0 ? lhs / rhs : INFINITY;
    pending = 0;
    if (lhs <= rhs) {
      if (visited == allcls) { *stop = 1; break; }
      pending = 1;
    }
    if (k == kmax) { *stop = 2; break; }
    if (nZ == m) { *stop = 3; break; }
    if (kcap > 0 && k == kcap) { *stop = 4; break; }
    if (cycle) {
      i = cycle_next(U, k, m, Z, ncls, i);
    } else if (pending) {
      i = class_probe(Z, m, ncls, visited);
      if (i < 0) { *stop = 1; break; }
    } else {
      i = fuzzy_argmax(u, m, Z);
    }
  }
  free(Z); free(vt); free(ut);
  *pU = U;
  *pV = V;
  return k;
}

/* ACA on a dense row-major m x n matrix (for synthetic tests). U, V must hold
 * m*min(m,n) and n*min(m,n) doubles; returns the rank. */
typedef struct { int m, n; const double* A; } dense_src;
static void dense_row(void* u, int i, double* out) {
  dense_src* s = (dense_src*)u;
  memcpy(out, s->A + (size_t)i * s->n, sizeof(double) * s->n);
}
static void dense_col(void* u, int j, double* out) {
  dense_src* s = (dense_src*)u;
  for (int r = 0; r < s->m; r++) out[r] = s->A[(size_t)r * s->n + j];
}
int or_aca_dense(int m, int n, const double* A, double eps, double* U, double* V, int* prow,
                 int* pcol, int* stop, double* ratio) {
  dense_src s = {m, n, A};
  double *Ui, *Vi;
  int k = aca_core(m, n, dense_row, dense_col, &s, eps, 0, 1, 0, &Ui, &Vi, prow, pcol, stop, ratio);
  memcpy(U, Ui, sizeof(double) * (size_t)m * k);
  memcpy(V, Vi, sizeof(double) * (size_t)n * k);
  free(Ui); free(Vi);
  return k;
}

/* The step-limited run (no accuracy test, class-cycling rows) on a dense
 * row-major m x n matrix whose rows fall into ncls classes: at most kcap
 * crosses. U, V must hold m*min(m,n,kcap) and n*min(m,n,kcap) doubles;
 * returns the rank (stop: 2 = min(m,n), 3 = Z full, 4 = kcap). */
int or_aca_dense_steps(int m, int n, const double* A, int kcap, int ncls, double* U, double* V,
                       int* prow, int* pcol, int* stop) {
  dense_src s = {m, n, A};
  double *Ui, *Vi, ratio;
  int k = aca_core(m, n, dense_row, dense_col, &s, 0.0, kcap, ncls, 1, &Ui, &Vi, prow, pcol, stop,
                   &ratio);
  memcpy(U, Ui, sizeof(double) * (size_t)m * k);
  memcpy(V, Vi, sizeof(double) * (size_t)n * k);
  free(Ui); free(Vi);
  return k;
}

/* ------------------------------------------------------------------------ */
/* Cluster tree, admissibility, partition (Sec. 2.1). */
typedef struct {
  int off, len, son0, son1, level;
  double lo[3], hi[3]; /* box of all vertices of the cluster's triangles (support X_t) */
} or_cluster;

typedef struct {
  int t, s;   /* cluster ids */
  int far;    /* 1 admissible (low-rank), 0 non-admissible (dense) */
} or_block;

typedef struct {
  or_ctx* c;
  double eta, eps;
  int leaf;
  int ncl, capcl;
  or_cluster* cl;
  int* order;
  int nb, capb;
  or_block* blk;
  /* filled by or_h_fill */
  int filled;
  int* rank;
  double** U;
  double** Vf;
  double** D;
  int** prow;
  int** pcol;
  int* stop;
  double* ratio;
  double t_plan, t_near, t_aca;
} or_hmat;

static int new_cluster(or_hmat* h) {
  if (h->ncl == h->capcl) {
    h->capcl = h->capcl ? 2 * h->capcl : 64;
    h->cl = (or_cluster*)realloc(h->cl, sizeof(or_cluster) * h->capcl);
  }
  return h->ncl++;
}

/* Bisection of the centroid bounding box along its longest axis (ties to the
 * lower axis index) at the midpoint; son 0 keeps coordinates <= mid, order
 * kept stable. A cluster of at most `leaf` triangles, or with zero extent, is
 * a leaf. */
static int build_tree(or_hmat* h, int* perm, int* tmp, int off, int len, int level) {
  int id = new_cluster(h);
  or_cluster* C = &h->cl[id];
  C->off = off;
  C->len = len;
  C->son0 = C->son1 = -1;
  C->level = level;
  for (int d = 0; d < 3; d++) {
    C->lo[d] = INFINITY;
    C->hi[d] = -INFINITY;
  }
  for (int p = off; p < off + len; p++)
    for (int v = 0; v < 3; v++) {
      const double* x = h->c->V + 3 * h->c->T[3 * perm[p] + v];
      for (int d = 0; d < 3; d++) {
        if (x[d] < C->lo[d]) C->lo[d] = x[d];
        if (x[d] > C->hi[d]) C->hi[d] = x[d];
      }
    }
  if (len <= h->leaf) return id;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int p = off; p < off + len; p++)
    for (int d = 0; d < 3; d++) {
      double x = h->c->cen[3 * perm[p] + d];
      if (x < lo[d]) lo[d] = x;
      if (x > hi[d]) hi[d] = x;
    }
  int ax = 0;
  for (int d = 1; d < 3; d++)
    if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
  if (!(hi[ax] - lo[ax] > 0.0)) return id;
  double mid = 0.5 * (lo[ax] + hi[ax]);
  int n0 = 0;
  for (int p = off; p < off + len; p++)
    if (h->c->cen[3 * perm[p] + ax] <= mid) tmp[n0++] = perm[p];
  int n1 = n0;
  for (int p = off; p < off + len; p++)
    if (!(h->c->cen[3 * perm[p] + ax] <= mid)) tmp[n1++] = perm[p];
  if (n0 == 0 || n0 == len) return id;
  memcpy(perm + off, tmp, sizeof(int) * len);
  int s0 = build_tree(h, perm, tmp, off, n0, level + 1);
  int s1 = build_tree(h, perm, tmp, off + n0, len - n0, level + 1);
  h->cl[id].son0 = s0;
  h->cl[id].son1 = s1;
  return id;
}

static double box_diam(const or_cluster* a) {
  double dx = a->hi[0] - a->lo[0], dy = a->hi[1] - a->lo[1], dz = a->hi[2] - a->lo[2];
  return sqrt(dx * dx + dy * dy + dz * dz);
}

static double box_dist(const or_cluster* a, const or_cluster* b) {
  double g[3];
  for (int d = 0; d < 3; d++) {
    double g1 = b->lo[d] - a->hi[d];
    double g2 = a->lo[d] - b->hi[d];
    double gg = g1 > g2 ? g1 : g2;
    g[d] = gg > 0.0 ? gg : 0.0;
  }
  return sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
}

/* eq. adm read as: dist > 0 and min(diam X_t, diam X_s) <= eta dist(X_t, X_s). */
static int admissible(const or_hmat* h, int t, int s) {
  double dist = box_dist(&h->cl[t], &h->cl[s]);
  if (!(dist > 0.0)) return 0;
  double dt = box_diam(&h->cl[t]), ds = box_diam(&h->cl[s]);
  double dm = dt < ds ? dt : ds;
  return dm <= h->eta * dist;
}

static void push_block(or_hmat* h, int t, int s, int far) {
  if (h->nb == h->capb) {
    h->capb = h->capb ? 2 * h->capb : 256;
    h->blk = (or_block*)realloc(h->blk, sizeof(or_block) * h->capb);
  }
  h->blk[h->nb].t = t;
  h->blk[h->nb].s = s;
  h->blk[h->nb].far = far;
  h->nb++;
}

/* Leaves of the block-cluster tree: descend from (root, root), sons visited
 * (t0,s0), (t0,s1), (t1,s0), (t1,s1); admissible -> low-rank leaf; else if t
 * or s is a leaf cluster -> dense leaf; else recurse. */
static void partition(or_hmat* h, int t, int s) {
  if (admissible(h, t, s)) {
    push_block(h, t, s, 1);
    return;
  }
  const or_cluster* T = &h->cl[t];
  const or_cluster* S = &h->cl[s];
  if (T->son0 < 0 || S->son0 < 0) {
    push_block(h, t, s, 0);
    return;
  }
  int t0 = T->son0, t1 = T->son1, s0 = S->son0, s1 = S->son1;
  partition(h, t0, s0);
  partition(h, t0, s1);
  partition(h, t1, s0);
  partition(h, t1, s1);
}

static const or_hmat* g_sort_h;
static int cmp_block(const void* a, const void* b) {
  const or_block* x = (const or_block*)a;
  const or_block* y = (const or_block*)b;
  int xr = g_sort_h->cl[x->t].off, yr = g_sort_h->cl[y->t].off;
  if (xr != yr) return xr < yr ? -1 : 1;
  int xc = g_sort_h->cl[x->s].off, yc = g_sort_h->cl[y->s].off;
  return xc < yc ? -1 : (xc > yc ? 1 : 0);
}

or_hmat* or_h_plan(or_ctx* c, double eta, int leaf) {
  if (!c || !(eta > 0.0) || leaf < 1) return NULL;
  double t0 = now_s();
  or_hmat* h = (or_hmat*)calloc(1, sizeof(or_hmat));
  h->c = c;
  h->eta = eta;
  h->leaf = leaf;
  int* perm = (int*)malloc(sizeof(int) * c->nt);
  int* tmp = (int*)malloc(sizeof(int) * c->nt);
  for (int i = 0; i < c->nt; i++) perm[i] = i;
  build_tree(h, perm, tmp, 0, c->nt, 0);
  free(tmp);
  h->order = perm;
  partition(h, 0, 0);
  g_sort_h = h;
  qsort(h->blk, h->nb, sizeof(or_block), cmp_block);
  h->t_plan = now_s() - t0;
  return h;
}

int or_h_nclusters(const or_hmat* h) { return h->ncl; }
/* info: off, len, son0, son1, level */
void or_h_cluster(const or_hmat* h, int id, int info[5], double box[6]) {
  const or_cluster* C = &h->cl[id];
  info[0] = C->off; info[1] = C->len; info[2] = C->son0; info[3] = C->son1; info[4] = C->level;
  for (int d = 0; d < 3; d++) { box[d] = C->lo[d]; box[3 + d] = C->hi[d]; }
}
void or_h_order(const or_hmat* h, int* order) { memcpy(order, h->order, sizeof(int) * h->c->nt); }
int or_h_nblocks(const or_hmat* h) { return h->nb; }
/* info: row_off, row_len, col_off, col_len (triangles), far, rank, stop, t id, s id */
void or_h_block(const or_hmat* h, int b, int info[9], double* ratio) {
  const or_block* B = &h->blk[b];
  info[0] = h->cl[B->t].off; info[1] = h->cl[B->t].len;
  info[2] = h->cl[B->s].off; info[3] = h->cl[B->s].len;
  info[4] = B->far;
  info[5] = h->filled && B->far ? h->rank[b] : 0;
  info[6] = h->filled && B->far ? h->stop[b] : 0;
  info[7] = B->t; info[8] = B->s;
  if (ratio) *ratio = h->filled && B->far ? h->ratio[b] : 0.0;
}

/* Sparsity constant c_sp (Sec. 2.1): max number of partition blocks sharing
 * a row cluster or a column cluster. */
int or_h_csp(const or_hmat* h) {
  int* r = (int*)calloc(h->ncl, sizeof(int));
  int* s = (int*)calloc(h->ncl, sizeof(int));
  int mx = 0;
  for (int b = 0; b < h->nb; b++) {
    r[h->blk[b].t]++;
    s[h->blk[b].s]++;
  }
  for (int i = 0; i < h->ncl; i++) {
    if (r[i] > mx) mx = r[i];
    if (s[i] > mx) mx = s[i];
  }
  free(r); free(s);
  return mx;
}

/* Far-block entry callbacks: local row 3p+a <-> triangle order[t.off+p], component a. */
typedef struct { const or_hmat* h; int t, s; } blk_src;
static void blk_row(void* u, int i, double* out) {
  blk_src* b = (blk_src*)u;
  const or_cluster* T = &b->h->cl[b->t];
  const or_cluster* S = &b->h->cl[b->s];
  int ti = b->h->order[T->off + i / 3], a = i % 3;
  for (int q = 0; q < S->len; q++) {
    double e[9];
    or_entry_block(b->h->c, ti, b->h->order[S->off + q], e);
    for (int d = 0; d < 3; d++) out[3 * q + d] = e[3 * a + d];
  }
}
static void blk_col(void* u, int j, double* out) {
  blk_src* b = (blk_src*)u;
  const or_cluster* T = &b->h->cl[b->t];
  const or_cluster* S = &b->h->cl[b->s];
  int tj = b->h->order[S->off + j / 3], d = j % 3;
  for (int p = 0; p < T->len; p++) {
    double e[9];
    or_entry_block(b->h->c, b->h->order[T->off + p], tj, e);
    for (int a = 0; a < 3; a++) out[3 * p + a] = e[3 * a + d];
  }
}

static const or_hmat* g_cost_h;
static int* g_cost_idx;
static int cmp_cost(const void* a, const void* b) {
  int x = *(const int*)a, y = *(const int*)b;
  const or_block* X = &g_cost_h->blk[x];
  const or_block* Y = &g_cost_h->blk[y];
  long cx = (long)g_cost_h->cl[X->t].len + g_cost_h->cl[X->s].len;
  long cy = (long)g_cost_h->cl[Y->t].len + g_cost_h->cl[Y->s].len;
  if (cx != cy) return cx > cy ? -1 : 1;
  return x < y ? -1 : (x > y ? 1 : 0);
}

static int h_fill(or_hmat* h, double eps, int kcap);

/* Dense blocks entry by entry (Sec. 2.2) and ACA on every admissible block. */
int or_h_fill(or_hmat* h, double eps) {
  if (!(eps > 0.0 && eps < 1.0)) return 1;
  return h_fill(h, eps, 0);
}

/* The same with ACA run for a fixed number of steps: no accuracy test
 * (eps = 0) and the class-cycling row rule (cycle_next), stopping at k = kcap
 * (stop code 4) unless a block is exhausted first (k = min(m,n), or every
 * row used). ACA is sequential, so the first r crosses of such a run are
 * those of any run that takes r steps: the adaptive multiplication
 * (Algorithm 2) uses prefixes of these crosses. */
int or_h_fill_steps(or_hmat* h, int kcap) {
  if (kcap < 1) return 1;
  return h_fill(h, 0.0, kcap);
}

static int h_fill(or_hmat* h, double eps, int kcap) {
  h->eps = eps;
  int nb = h->nb;
  h->rank = (int*)calloc(nb, sizeof(int));
  h->U = (double**)calloc(nb, sizeof(double*));
  h->Vf = (double**)calloc(nb, sizeof(double*));
  h->D = (double**)calloc(nb, sizeof(double*));
  h->prow = (int**)calloc(nb, sizeof(int*));
  h->pcol = (int**)calloc(nb, sizeof(int*));
  h->stop = (int*)calloc(nb, sizeof(int));
  h->ratio = (double*)calloc(nb, sizeof(double));
  double t0 = now_s();
#pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < nb; b++) {
    const or_block* B = &h->blk[b];
    if (B->far) continue;
    const or_cluster* T = &h->cl[B->t];
    const or_cluster* S = &h->cl[B->s];
    int m = 3 * T->len, n = 3 * S->len;
    double* D = (double*)malloc(sizeof(double) * (size_t)m * n);
    for (int q = 0; q < S->len; q++)
      for (int p = 0; p < T->len; p++) {
        double e[9];
        or_entry_block(h->c, h->order[T->off + p], h->order[S->off + q], e);
        for (int a = 0; a < 3; a++)
          for (int d = 0; d < 3; d++) D[(size_t)(3 * q + d) * m + 3 * p + a] = e[3 * a + d];
      }
    h->D[b] = D;
  }
  double t1 = now_s();
  int* idx = (int*)malloc(sizeof(int) * nb);
  int nf = 0;
  for (int b = 0; b < nb; b++)
    if (h->blk[b].far) idx[nf++] = b;
  g_cost_h = h;
  g_cost_idx = idx;
  qsort(idx, nf, sizeof(int), cmp_cost);
#pragma omp parallel for schedule(dynamic, 1)
  for (int f = 0; f < nf; f++) {
    int b = idx[f];
    const or_block* B = &h->blk[b];
    int m = 3 * h->cl[B->t].len, n = 3 * h->cl[B->s].len;
    int kmax = m < n ? m : n;
    blk_src src = {h, B->t, B->s};
    h->prow[b] = (int*)malloc(sizeof(int) * kmax);
    h->pcol[b] = (int*)malloc(sizeof(int) * kmax);
    h->rank[b] = aca_core(m, n, blk_row, blk_col, &src, eps, kcap, 3, eps == 0.0, &h->U[b], &h->Vf[b], h->prow[b],
                          h->pcol[b], &h->stop[b], &h->ratio[b]);
    /* A block whose accuracy-controlled ACA reaches full rank is stored
     * exactly: a cross approximation is kept only as a compression (Sec. 2
     * stores a block low-rank only if k(M+N) < MN, which full rank never
     * meets), and a full-rank run can end inexact when a remainder at
     * rounding level is taken as a cross. U = B, V = I for n <= m, else
     * U = I, V = B^T; the rank stays min(m, n). */
    if (eps > 0.0 && h->rank[b] == kmax) {
      double* U = h->U[b];
      double* V = h->Vf[b];
      memset(U, 0, sizeof(double) * (size_t)m * kmax);
      memset(V, 0, sizeof(double) * (size_t)n * kmax);
      if (n <= m) {
        for (int c = 0; c < n; c++) {
          blk_col(&src, c, U + (size_t)c * m);
          V[(size_t)c * n + c] = 1.0;
        }
      } else {
        for (int r = 0; r < m; r++) {
          blk_row(&src, r, V + (size_t)r * n);
          U[(size_t)r * m + r] = 1.0;
        }
      }
    }
  }
  free(idx);
  h->t_near = t1 - t0;
  h->t_aca = now_s() - t1;
  h->filled = 1;
  return 0;
}

void or_h_times(const or_hmat* h, double t[3]) {
  t[0] = h->t_plan; t[1] = h->t_near; t[2] = h->t_aca;
}

/* Factor export: U m x k, V n x k (column-major), pivots (k each). */
void or_h_factors(const or_hmat* h, int b, double* U, double* V, int* prow, int* pcol) {
  const or_block* B = &h->blk[b];
  int m = 3 * h->cl[B->t].len, n = 3 * h->cl[B->s].len, k = h->rank[b];
  if (U) memcpy(U, h->U[b], sizeof(double) * (size_t)m * k);
  if (V) memcpy(V, h->Vf[b], sizeof(double) * (size_t)n * k);
  if (prow) memcpy(prow, h->prow[b], sizeof(int) * k);
  if (pcol) memcpy(pcol, h->pcol[b], sizeof(int) * k);
}

void or_h_dense_block(const or_hmat* h, int b, double* D) {
  const or_block* B = &h->blk[b];
  int m = 3 * h->cl[B->t].len, n = 3 * h->cl[B->s].len;
  memcpy(D, h->D[b], sizeof(double) * (size_t)m * n);
}

/* Stored scalars: sum_far k(m+n) + sum_near m n. */
int64_t or_h_stored(const or_hmat* h) {
  int64_t s = 0;
  for (int b = 0; b < h->nb; b++) {
    const or_block* B = &h->blk[b];
    int64_t m = 3 * h->cl[B->t].len, n = 3 * h->cl[B->s].len;
    s += B->far ? (int64_t)h->rank[b] * (m + n) : m * n;
  }
  return s;
}

/* y = A_H x in the caller's DOF order for nrhs vectors (leading dimension 3nt). */
void or_h_matvec(const or_hmat* h, int nrhs, const double* x, double* y) {
  int nt = h->c->nt;
  int64_t N = 3 * (int64_t)nt;
  double* xp = (double*)malloc(sizeof(double) * N * nrhs);
  for (int r = 0; r < nrhs; r++)
    for (int p = 0; p < nt; p++)
      for (int a = 0; a < 3; a++) xp[r * N + 3 * p + a] = x[r * N + 3 * (int64_t)h->order[p] + a];
  int nth = or_num_threads();
  double* yp = (double*)calloc((size_t)nth * N * nrhs, sizeof(double));
#pragma omp parallel
  {
#ifdef _OPENMP
    int tid = omp_get_thread_num();
#else
    int tid = 0;
#endif
    double* yl = yp + (size_t)tid * N * nrhs;
#pragma omp for schedule(dynamic, 1)
    for (int b = 0; b < h->nb; b++) {
      const or_block* B = &h->blk[b];
      int m = 3 * h->cl[B->t].len, n = 3 * h->cl[B->s].len;
      int r0 = 3 * h->cl[B->t].off, c0 = 3 * h->cl[B->s].off;
      for (int r = 0; r < nrhs; r++) {
        const double* xs = xp + r * N + c0;
        double* yt = yl + r * N + r0;
        if (B->far) {
          int k = h->rank[b];
          for (int l = 0; l < k; l++) {
            const double* v = h->Vf[b] + (size_t)l * n;
            const double* u = h->U[b] + (size_t)l * m;
            double z = 0.0;
            for (int c = 0; c < n; c++) z += v[c] * xs[c];
            for (int i = 0; i < m; i++) yt[i] += u[i] * z;
          }
        } else {
          const double* D = h->D[b];
          for (int c = 0; c < n; c++) {
            double xc = xs[c];
            for (int i = 0; i < m; i++) yt[i] += D[(size_t)c * m + i] * xc;
          }
        }
      }
    }
  }
  for (int r = 0; r < nrhs; r++)
    for (int p = 0; p < nt; p++)
      for (int a = 0; a < 3; a++) {
        double s = 0.0;
        for (int t = 0; t < nth; t++) s += yp[(size_t)t * N * nrhs + r * N + 3 * p + a];
        y[r * N + 3 * (int64_t)h->order[p] + a] = s;
      }
  free(xp);
  free(yp);
}

void or_h_free(or_hmat* h) {
  if (!h) return;
  if (h->filled)
    for (int b = 0; b < h->nb; b++) {
      free(h->U[b]); free(h->Vf[b]); free(h->D[b]); free(h->prow[b]); free(h->pcol[b]);
    }
  free(h->rank); free(h->U); free(h->Vf); free(h->D); free(h->prow); free(h->pcol);
  free(h->stop); free(h->ratio);
  free(h->cl); free(h->order); free(h->blk);
  free(h);
}

/* ------------------------------------------------------------------------ */
/* GMRES(m) (Saad & Schultz 1986): x0 = 0, Arnoldi with modified Gram-Schmidt,
 * Givens rotations on the Hessenberg matrix, restart after m steps.
 * Converged iff the explicit residual ||b - A x|| <= tol ||b||; an inner
 * cycle ends early when the recurrence residual |g_{j+1}| reaches tol ||b||.
 * At most maxit matrix-vector products (Arnoldi steps). Returns 0 when
 * converged, 4 otherwise; x, *iters and *relres are always written. */
typedef void (*or_matvecfn)(void* u, const double* x, double* y);

static double dot(int64_t n, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

int or_gmres(int64_t n, or_matvecfn A, void* user, const double* b, double* x, double tol,
             int restart, int maxit, int* iters, double* relres) {
  int m = restart;
  double* Vb = (double*)malloc(sizeof(double) * (size_t)n * (m + 1));
  double* H = (double*)calloc((size_t)(m + 1) * m, sizeof(double)); /* H[i*m + j] */
  double* cs = (double*)malloc(sizeof(double) * m);
  double* sn = (double*)malloc(sizeof(double) * m);
  double* g = (double*)malloc(sizeof(double) * (m + 1));
  double* yv = (double*)malloc(sizeof(double) * m);
  double* r = (double*)malloc(sizeof(double) * n);
  double* w = (double*)malloc(sizeof(double) * n);
  for (int64_t i = 0; i < n; i++) x[i] = 0.0;
  double bn = sqrt(dot(n, b, b));
  int total = 0, status = 4;
  double rel = 1.0;
  if (bn == 0.0) {
    *iters = 0;
    *relres = 0.0;
    status = 0;
    goto done;
  }
  for (;;) {
    A(user, x, r);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - r[i];
    double beta = sqrt(dot(n, r, r));
    rel = beta / bn;
    if (beta <= tol * bn) { status = 0; break; }
    if (total >= maxit) break;
    for (int64_t i = 0; i < n; i++) Vb[i] = r[i] / beta;
    for (int i = 0; i <= m; i++) g[i] = 0.0;
    g[0] = beta;
    int j;
    for (j = 0; j < m && total < maxit; j++) {
      A(user, Vb + (size_t)j * n, w);
      total++;
      for (int i = 0; i <= j; i++) {
        double hij = dot(n, w, Vb + (size_t)i * n);
        H[i * m + j] = hij;
        for (int64_t q = 0; q < n; q++) w[q] -= hij * Vb[(size_t)i * n + q];
      }
      double hn = sqrt(dot(n, w, w));
      H[(j + 1) * m + j] = hn;
      if (hn != 0.0)
        for (int64_t q = 0; q < n; q++) Vb[(size_t)(j + 1) * n + q] = w[q] / hn;
      for (int i = 0; i < j; i++) {
        double a = H[i * m + j], c2 = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * c2;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c2;
      }
      double a = H[j * m + j], c2 = H[(j + 1) * m + j];
      double den = sqrt(a * a + c2 * c2);
      cs[j] = den == 0.0 ? 1.0 : a / den;
      sn[j] = den == 0.0 ? 0.0 : c2 / den;
      H[j * m + j] = cs[j] * a + sn[j] * c2;
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      if (fabs(g[j + 1]) <= tol * bn || hn == 0.0) { j++; break; }
    }
    for (int i = j - 1; i >= 0; i--) {
      double s = g[i];
      for (int q = i + 1; q < j; q++) s -= H[i * m + q] * yv[q];
      yv[i] = s / H[i * m + i];
    }
    for (int i = 0; i < j; i++)
      for (int64_t q = 0; q < n; q++) x[q] += yv[i] * Vb[(size_t)i * n + q];
  }
  *iters = total;
  *relres = rel;
done:
  free(Vb); free(H); free(cs); free(sn); free(g); free(yv); free(r); free(w);
  return status;
}

static void h_mv(void* u, const double* x, double* y) { or_h_matvec((const or_hmat*)u, 1, x, y); }
int or_h_gmres(const or_hmat* h, const double* b, double* x, double tol, int restart, int maxit,
               int* iters, double* relres) {
  return or_gmres(3 * (int64_t)h->c->nt, h_mv, (void*)h, b, x, tol, restart, maxit, iters, relres);
}

typedef struct { int64_t n; const double* A; } dense_op;
static void dense_mv(void* u, const double* x, double* y) {
  dense_op* d = (dense_op*)u;
  for (int64_t i = 0; i < d->n; i++) y[i] = dot(d->n, d->A + i * d->n, x);
}
int or_dense_gmres(int64_t n, const double* A, const double* b, double* x, double tol, int restart,
                   int maxit, int* iters, double* relres) {
  dense_op d = {n, A};
  return or_gmres(n, dense_mv, &d, b, x, tol, restart, maxit, iters, relres);
}
