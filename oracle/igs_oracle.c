/*
 * Plain FP64 CPU oracle for the surrogate-matrix IGA assembly path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) may include, link or call this file.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark use it.  It shares
 * no code, header, table or constant with the GPU path.
 *
 * What it computes (Drzisga, Keith & Wohlmuth, "The surrogate matrix
 * methodology: Low-cost assembly for isogeometric analysis"):
 *   - open uniform knot vectors and the tensor-product B-spline basis
 *     (Sec. 2.2, eq. NURBS with all weights 1);
 *   - the stiffness entries A_ij = a(B_j, B_i) through the pull-back tensor
 *     K = kappa |det J| J^{-1} J^{-T} (Sec. 3.2, eq. BilinearFormPoissonTensor)
 *     and the mass entries M_ij = int B_i B_j |det J| (Sec. 8, membrane
 *     problem), each row computed by element-wise Gauss quadrature over the
 *     support of B_i, entry (i, i+delta) stored at stencil slot delta;
 *   - the load vector F(B_i) = int f B_i (Sec. 7, eq. PoissonWeakForm);
 *   - the derivative of the stiffness entries with respect to one B-spline
 *     control coefficient of the diffusion coefficient (adjoint checks).
 *
 * Every entry (i, j) is computed from row i's own quadrature, so A_ij and A_ji
 * come out of independent arithmetic and symmetry is something tests check.
 * There is no sum factorisation, no blocking and no reuse across rows: each
 * row loops over its (p+1)^n support elements, each element over its
 * quadrature points, each point over the (p+1)^n basis functions alive there.
 *
 * Integer parameter block ip[]:
 *   ip[0]=n (2|3) ip[1]=p ip[2..4]=nelem per direction ip[5]=quadrature points
 *   per direction per element ip[6]=geometry kind ip[7]=coefficient kind
 *   ip[8]=coefficient spline degree ip[9..11]=coefficient spline functions per
 *   direction.
 * Double parameter block dp[]: dp[0]=map amplitude a, dp[1]=c0, dp[2]=amp.
 * Geometry kinds: 0 identity, 1 sine map, 2 quadratic bubble map.
 * Coefficient kinds: 0 constant c0, 1 c0 + amp*sin(2 pi x1)cos(2 pi x2)
 *   [*sin(2 pi x3)] at x = F(xi), 2 spline g(xi), 3 exp(g(xi)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

typedef struct {
  int n, p, nq;
  int nelem[3], m[3];
  int geom, coef, cdeg, cn[3];
  double ga, c0, camp;
  const double* cc;          /* coefficient spline control values, colex */
  double* knots[3];          /* open uniform knots, m+p+1 each */
  double* gx;                /* Gauss nodes on [-1,1] */
  double* gw;                /* Gauss weights */
  double* ck[3];             /* coefficient spline knots */
  double* tv[3];             /* tv[d][(e*nq + k)*(p+1) + a] = b_{e+a}(xi_{e,k}) */
  double* td[3];             /* same for the derivative */
} oprob;

/* ---------------------------------------------------------------- Gauss -- */
/* Gauss-Legendre rule on [-1,1]: nodes are the roots of P_nq, found by Newton
 * iteration on the three-term Legendre recurrence; w = 2/((1-x^2) P'(x)^2). */
static void legendre(int nq, double z, double* pn, double* pnm1) {
  double p0 = 1.0, p1 = z;           /* P_0, P_1 */
  for (int j = 2; j <= nq; ++j) {
    double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
    p0 = p1; p1 = p2;
  }
  *pn = p1; *pnm1 = p0;              /* P_nq, P_{nq-1} */
}

int or_gauss(int nq, double* x, double* w) {
  if (nq < 1 || nq > 32) return -1;
  for (int k = 0; k < nq; ++k) {
    double z = cos(OR_PI * (k + 0.75) / (nq + 0.5)), pn, pm, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(nq, z, &pn, &pm);
      dp = nq * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    legendre(nq, z, &pn, &pm);
    dp = nq * (z * pn - pm) / (z * z - 1.0);
    x[nq - 1 - k] = z;                /* roots come out descending */
    w[nq - 1 - k] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  return 0;
}

/* --------------------------------------------------------- B-splines ----- */
/* Cox-de Boor recursion written as its definition (Sec. 2.2): degree-0
 * functions are indicators of half-open knot spans, degree r is the convex
 * blend of two degree r-1 functions; 0/0 is taken as 0. */
static double cdb(const double* t, int k, int r, double x) {
  if (r == 0) return (t[k] <= x && x < t[k + 1]) ? 1.0 : 0.0;
  double a = 0.0, b = 0.0;
  double d1 = t[k + r] - t[k], d2 = t[k + r + 1] - t[k + 1];
  if (d1 > 0.0) a = (x - t[k]) / d1 * cdb(t, k, r - 1, x);
  if (d2 > 0.0) b = (t[k + r + 1] - x) / d2 * cdb(t, k + 1, r - 1, x);
  return a + b;
}

/* derivative of a degree-r B-spline: r/(t_{k+r}-t_k) b_{k,r-1} - r/(...) b_{k+1,r-1} */
static double cdb_d(const double* t, int k, int r, double x) {
  if (r == 0) return 0.0;
  double a = 0.0, b = 0.0;
  double d1 = t[k + r] - t[k], d2 = t[k + r + 1] - t[k + 1];
  if (d1 > 0.0) a = r / d1 * cdb(t, k, r - 1, x);
  if (d2 > 0.0) b = r / d2 * cdb(t, k + 1, r - 1, x);
  return a - b;
}

/* Open uniform knot vector with nel elements, degree p on [0,1] (Sec. 2.2). */
static double* open_knots(int nel, int p) {
  int m = nel + p;
  double* t = (double*)malloc(sizeof(double) * (m + p + 1));
  for (int k = 0; k < m + p + 1; ++k) {
    if (k <= p) t[k] = 0.0;
    else if (k >= m) t[k] = 1.0;
    else t[k] = (double)(k - p) / nel;
  }
  return t;
}

/* Expose basis evaluation for pinning against an independent library. */
int or_basis(int nel, int p, int k, double x, double* val, double* der) {
  double* t = open_knots(nel, p);
  *val = cdb(t, k, p, x);
  *der = cdb_d(t, k, p, x);
  free(t);
  return 0;
}

/* ------------------------------------------------------------ problem ---- */
static int setup(oprob* P, const int32_t* ip, const double* dp, const double* cc) {
  memset(P, 0, sizeof(*P));
  P->n = ip[0]; P->p = ip[1];
  if (P->n < 2 || P->n > 3 || P->p < 1 || P->p > 8) return -1;
  for (int d = 0; d < 3; ++d) P->nelem[d] = (d < P->n) ? ip[2 + d] : 1;
  for (int d = 0; d < P->n; ++d) {
    if (P->nelem[d] < 1) return -1;
    P->m[d] = P->nelem[d] + P->p;
    P->knots[d] = open_knots(P->nelem[d], P->p);
  }
  for (int d = P->n; d < 3; ++d) P->m[d] = 1;
  P->nq = ip[5] > 0 ? ip[5] : P->p + 1;
  P->geom = ip[6]; P->coef = ip[7]; P->cdeg = ip[8];
  for (int d = 0; d < 3; ++d) P->cn[d] = (d < P->n) ? ip[9 + d] : 1;
  P->ga = dp[0]; P->c0 = dp[1]; P->camp = dp[2];
  P->cc = cc;
  for (int d = 0; d < P->n; ++d) if (P->cn[d] > 64) return -1;
  P->gx = (double*)malloc(sizeof(double) * P->nq);
  P->gw = (double*)malloc(sizeof(double) * P->nq);
  if (or_gauss(P->nq, P->gx, P->gw)) return -1;
  /* tabulate the p+1 functions alive on each element at its Gauss points */
  for (int d = 0; d < P->n; ++d) {
    int ne = P->nelem[d], np1 = P->p + 1;
    P->tv[d] = (double*)malloc(sizeof(double) * ne * P->nq * np1);
    P->td[d] = (double*)malloc(sizeof(double) * ne * P->nq * np1);
    for (int e = 0; e < ne; ++e)
      for (int k = 0; k < P->nq; ++k) {
        double x = (e + 0.5 * (P->gx[k] + 1.0)) / ne;
        for (int a = 0; a < np1; ++a) {
          P->tv[d][(e * P->nq + k) * np1 + a] = cdb(P->knots[d], e + a, P->p, x);
          P->td[d][(e * P->nq + k) * np1 + a] = cdb_d(P->knots[d], e + a, P->p, x);
        }
      }
  }
  if (P->coef == 2 || P->coef == 3) {
    for (int d = 0; d < P->n; ++d) {
      if (P->cn[d] <= P->cdeg) return -1;
      P->ck[d] = open_knots(P->cn[d] - P->cdeg, P->cdeg);
    }
  }
  return 0;
}

static void teardown(oprob* P) {
  for (int d = 0; d < 3; ++d) { free(P->knots[d]); free(P->ck[d]); free(P->tv[d]); free(P->td[d]); }
  free(P->gx); free(P->gw);
}

/* Geometry map F and its Jacobian J[a][b] = dF_a/dxi_b. */
static void geometry(const oprob* P, const double* xi, double* F, double J[3][3]) {
  int n = P->n;
  double a = P->ga;
  for (int r = 0; r < 3; ++r) { F[r] = (r < n) ? xi[r] : 0.0; for (int c = 0; c < 3; ++c) J[r][c] = (r == c) ? 1.0 : 0.0; }
  if (P->geom == 0) return;
  if (P->geom == 1) {
    double s1[3], c1[3], s2[3], c2[3];
    for (int d = 0; d < n; ++d) {
      s1[d] = sin(OR_PI * xi[d]); c1[d] = OR_PI * cos(OR_PI * xi[d]);
      s2[d] = sin(2.0 * OR_PI * xi[d]); c2[d] = 2.0 * OR_PI * cos(2.0 * OR_PI * xi[d]);
    }
    if (n == 2) {
      /* F1 = x1 + a sin(pi x1) sin(2 pi x2), F2 = x2 + a sin(2 pi x1) sin(pi x2) */
      F[0] += a * s1[0] * s2[1];
      F[1] += a * s2[0] * s1[1];
      J[0][0] += a * c1[0] * s2[1]; J[0][1] += a * s1[0] * c2[1];
      J[1][0] += a * c2[0] * s1[1]; J[1][1] += a * s2[0] * c1[1];
    } else {
      /* F1 += a s(pi x1) s(2pi x2) s(pi x3); F2 += a s(2pi x1) s(pi x2) s(pi x3);
         F3 += a s(pi x1) s(pi x2) s(2pi x3) */
      F[0] += a * s1[0] * s2[1] * s1[2];
      F[1] += a * s2[0] * s1[1] * s1[2];
      F[2] += a * s1[0] * s1[1] * s2[2];
      J[0][0] += a * c1[0] * s2[1] * s1[2]; J[0][1] += a * s1[0] * c2[1] * s1[2]; J[0][2] += a * s1[0] * s2[1] * c1[2];
      J[1][0] += a * c2[0] * s1[1] * s1[2]; J[1][1] += a * s2[0] * c1[1] * s1[2]; J[1][2] += a * s2[0] * s1[1] * c1[2];
      J[2][0] += a * c1[0] * s1[1] * s2[2]; J[2][1] += a * s1[0] * c1[1] * s2[2]; J[2][2] += a * s1[0] * s1[1] * c2[2];
    }
    return;
  }
  if (P->geom == 2) {
    /* F_r = xi_r + a (r+1) prod_d xi_d (1 - xi_d): every component in Q_2 */
    double g[3], dg[3];
    for (int d = 0; d < n; ++d) { g[d] = xi[d] * (1.0 - xi[d]); dg[d] = 1.0 - 2.0 * xi[d]; }
    for (int r = 0; r < n; ++r) {
      double prod = 1.0;
      for (int d = 0; d < n; ++d) prod *= g[d];
      F[r] += a * (r + 1) * prod;
      for (int c = 0; c < n; ++c) {
        double dprod = dg[c];
        for (int d = 0; d < n; ++d) if (d != c) dprod *= g[d];
        J[r][c] += a * (r + 1) * dprod;
      }
    }
  }
}

static double det_inv(int n, double J[3][3], double Ji[3][3]) {
  if (n == 2) {
    double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    Ji[0][0] = J[1][1] / det; Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
    return det;
  }
  double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  Ji[0][0] = c00 / det;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  Ji[1][0] = c01 / det;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  Ji[2][0] = c02 / det;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  return det;
}

/* Coefficient spline g(xi) = sum_k c_k N_k(xi), and N_kk(xi) for one k. */
static double spline_g(const oprob* P, const double* xi, int kk, double* Nkk) {
  int n = P->n, deg = P->cdeg;
  double g = 0.0;
  *Nkk = 0.0;
  int kk_d[3] = {0, 0, 0};
  if (kk >= 0) { int r = kk; for (int d = 0; d < n; ++d) { kk_d[d] = r % P->cn[d]; r /= P->cn[d]; } }
  double vals[3][64];
  for (int d = 0; d < n; ++d)
    for (int k = 0; k < P->cn[d]; ++k) vals[d][k] = cdb(P->ck[d], k, deg, xi[d]);
  if (n == 2) {
    for (int k2 = 0; k2 < P->cn[1]; ++k2)
      for (int k1 = 0; k1 < P->cn[0]; ++k1)
        g += P->cc[k1 + P->cn[0] * k2] * vals[0][k1] * vals[1][k2];
    if (kk >= 0) *Nkk = vals[0][kk_d[0]] * vals[1][kk_d[1]];
  } else {
    for (int k3 = 0; k3 < P->cn[2]; ++k3)
      for (int k2 = 0; k2 < P->cn[1]; ++k2)
        for (int k1 = 0; k1 < P->cn[0]; ++k1)
          g += P->cc[k1 + P->cn[0] * (k2 + P->cn[1] * k3)] * vals[0][k1] * vals[1][k2] * vals[2][k3];
    if (kk >= 0) *Nkk = vals[0][kk_d[0]] * vals[1][kk_d[1]] * vals[2][kk_d[2]];
  }
  return g;
}

/* kappa at parametric point xi with physical image F; with dcoef >= 0 returns
 * d kappa / d c_dcoef instead. */
static double kappa(const oprob* P, const double* xi, const double* F, int dcoef) {
  if (P->coef == 0) return dcoef >= 0 ? 0.0 : P->c0;
  if (P->coef == 1) {
    if (dcoef >= 0) return 0.0;
    double v = sin(2.0 * OR_PI * F[0]) * cos(2.0 * OR_PI * F[1]);
    if (P->n == 3) v *= sin(2.0 * OR_PI * F[2]);
    return P->c0 + P->camp * v;
  }
  double Nk;
  double g = spline_g(P, xi, dcoef, &Nk);
  if (P->coef == 2) return dcoef >= 0 ? Nk : g;
  return dcoef >= 0 ? exp(g) * Nk : exp(g);
}

static int slot_of(const oprob* P, const int* delta) {
  int s = 0, stride = 1, w = 2 * P->p + 1;
  for (int d = 0; d < P->n; ++d) { s += (delta[d] + P->p) * stride; stride *= w; }
  return s;
}

/* One exact row: stiffness (form 0) or mass (form 1); dcoef >= 0 gives the
 * derivative of the stiffness row with respect to coefficient dcoef. */
static int exact_row(const oprob* P, int form, int dcoef, int64_t row, double* out) {
  int n = P->n, p = P->p, nq = P->nq;
  int S = 1;
  for (int d = 0; d < n; ++d) S *= 2 * p + 1;
  for (int s = 0; s < S; ++s) out[s] = 0.0;
  int i[3] = {0, 0, 0};
  int64_t r = row;
  for (int d = 0; d < n; ++d) { i[d] = (int)(r % P->m[d]); r /= P->m[d]; }
  int elo[3] = {0, 0, 0}, ehi[3] = {0, 0, 0};
  for (int d = 0; d < n; ++d) {
    elo[d] = i[d] - p < 0 ? 0 : i[d] - p;
    ehi[d] = i[d] > P->nelem[d] - 1 ? P->nelem[d] - 1 : i[d];
  }
  int bad = 0;
  int e[3] = {0, 0, 0};
  for (e[2] = elo[2]; e[2] <= ehi[2]; ++e[2])
  for (e[1] = elo[1]; e[1] <= ehi[1]; ++e[1])
  for (e[0] = elo[0]; e[0] <= ehi[0]; ++e[0]) {
    int k[3] = {0, 0, 0};
    int kmax3 = (n == 3) ? nq : 1;
    for (k[2] = 0; k[2] < kmax3; ++k[2])
    for (k[1] = 0; k[1] < nq; ++k[1])
    for (k[0] = 0; k[0] < nq; ++k[0]) {
      double xi[3] = {0, 0, 0}, wt = 1.0;
      for (int d = 0; d < n; ++d) {
        double h = 1.0 / P->nelem[d];
        xi[d] = (e[d] + 0.5 * (P->gx[k[d]] + 1.0)) * h;
        wt *= 0.5 * h * P->gw[k[d]];
      }
      double F[3], J[3][3], Ji[3][3];
      geometry(P, xi, F, J);
      double det = det_inv(n, J, Ji);
      if (!(det > 0.0)) bad = 1;
      /* basis values of the row function and of every function alive on e */
      double bv[3][16], bd[3][16];
      for (int d = 0; d < n; ++d)
        for (int a = 0; a <= p; ++a) {
          bv[d][a] = P->tv[d][(e[d] * nq + k[d]) * (p + 1) + a];
          bd[d][a] = P->td[d][(e[d] * nq + k[d]) * (p + 1) + a];
        }
      double Bi = 1.0, gi[3];
      for (int d = 0; d < n; ++d) Bi *= bv[d][i[d] - e[d]];
      for (int a = 0; a < n; ++a) {
        gi[a] = 1.0;
        for (int d = 0; d < n; ++d) gi[a] *= (d == a) ? bd[d][i[d] - e[d]] : bv[d][i[d] - e[d]];
      }
      double K[3][3];
      if (form == 0) {
        double kap = kappa(P, xi, F, dcoef);
        for (int a = 0; a < n; ++a)
          for (int b = 0; b < n; ++b) {
            double s = 0.0;
            for (int c = 0; c < n; ++c) s += Ji[a][c] * Ji[b][c];
            K[a][b] = kap * fabs(det) * s;
          }
      }
      int j[3] = {0, 0, 0};
      int jhi2 = (n == 3) ? e[2] + p : 0, jlo2 = (n == 3) ? e[2] : 0;
      for (j[2] = jlo2; j[2] <= jhi2; ++j[2])
      for (j[1] = e[1]; j[1] <= e[1] + p; ++j[1])
      for (j[0] = e[0]; j[0] <= e[0] + p; ++j[0]) {
        int delta[3] = {0, 0, 0};
        for (int d = 0; d < n; ++d) delta[d] = j[d] - i[d];
        double val;
        if (form == 0) {
          double gj[3];
          for (int a = 0; a < n; ++a) {
            gj[a] = 1.0;
            for (int d = 0; d < n; ++d) gj[a] *= (d == a) ? bd[d][j[d] - e[d]] : bv[d][j[d] - e[d]];
          }
          val = 0.0;
          for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) val += gi[a] * K[a][b] * gj[b];
        } else {
          double Bj = 1.0;
          for (int d = 0; d < n; ++d) Bj *= bv[d][j[d] - e[d]];
          val = fabs(det) * Bi * Bj;
        }
        out[slot_of(P, delta)] += wt * val;
      }
    }
  }
  return bad ? -2 : 0;
}

int or_rows(const int32_t* ip, const double* dp, const double* cc, int form, int dcoef,
            const int64_t* rows, int64_t nrows, double* out) {
  oprob P;
  if (setup(&P, ip, dp, cc)) { teardown(&P); return -1; }
  int S = 1;
  for (int d = 0; d < P.n; ++d) S *= 2 * P.p + 1;
  int64_t N = (int64_t)P.m[0] * P.m[1] * P.m[2];
  int status = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(min : status)
  for (int64_t r = 0; r < nrows; ++r) {
    if (rows[r] < 0 || rows[r] >= N) { status = -1; continue; }
    int st = exact_row(&P, form, dcoef, rows[r], out + r * S);
    if (st < status) status = st;
  }
  teardown(&P);
  return status;
}

/* Load vector F(B_i) = int f(x) B_i(x) dx with f = c (src 0) or
 * f = c prod_d sin(pi x_d) (src 1), x = F(xi) (Sec. 7, eq. PoissonWeakForm). */
int or_rhs(const int32_t* ip, const double* dp, const double* cc, int src, double c,
           const int64_t* rows, int64_t nrows, double* out) {
  oprob P;
  if (setup(&P, ip, dp, cc)) { teardown(&P); return -1; }
  int n = P.n, p = P.p, nq = P.nq;
  int64_t N = (int64_t)P.m[0] * P.m[1] * P.m[2];
  int status = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(min : status)
  for (int64_t r = 0; r < nrows; ++r) {
    if (rows[r] < 0 || rows[r] >= N) { status = -1; continue; }
    int i[3] = {0, 0, 0};
    int64_t rr = rows[r];
    for (int d = 0; d < n; ++d) { i[d] = (int)(rr % P.m[d]); rr /= P.m[d]; }
    int elo[3] = {0, 0, 0}, ehi[3] = {0, 0, 0};
    for (int d = 0; d < n; ++d) {
      elo[d] = i[d] - p < 0 ? 0 : i[d] - p;
      ehi[d] = i[d] > P.nelem[d] - 1 ? P.nelem[d] - 1 : i[d];
    }
    double acc = 0.0;
    int e[3] = {0, 0, 0};
    for (e[2] = elo[2]; e[2] <= ehi[2]; ++e[2])
    for (e[1] = elo[1]; e[1] <= ehi[1]; ++e[1])
    for (e[0] = elo[0]; e[0] <= ehi[0]; ++e[0]) {
      int k[3] = {0, 0, 0};
      int kmax3 = (n == 3) ? nq : 1;
      for (k[2] = 0; k[2] < kmax3; ++k[2])
      for (k[1] = 0; k[1] < nq; ++k[1])
      for (k[0] = 0; k[0] < nq; ++k[0]) {
        double xi[3] = {0, 0, 0}, wt = 1.0;
        for (int d = 0; d < n; ++d) {
          double h = 1.0 / P.nelem[d];
          xi[d] = (e[d] + 0.5 * (P.gx[k[d]] + 1.0)) * h;
          wt *= 0.5 * h * P.gw[k[d]];
        }
        double F[3], J[3][3], Ji[3][3];
        geometry(&P, xi, F, J);
        double det = det_inv(n, J, Ji);
        double Bi = 1.0;
        for (int d = 0; d < n; ++d) Bi *= P.tv[d][(e[d] * nq + k[d]) * (p + 1) + i[d] - e[d]];
        double f = c;
        if (src == 1)
          for (int d = 0; d < n; ++d) f *= sin(OR_PI * F[d]);
        acc += wt * f * Bi * fabs(det);
      }
    }
    out[r] = acc;
  }
  teardown(&P);
  return status;
}

/* Physical image and |det J| at given parametric points (used by the tests to
 * form L2 errors of discrete solutions). */
int or_map(const int32_t* ip, const double* dp, const double* xi, int64_t npts, double* F, double* det) {
  oprob P;
  if (setup(&P, ip, dp, NULL)) { teardown(&P); return -1; }
  for (int64_t t = 0; t < npts; ++t) {
    double J[3][3], Ji[3][3], f[3];
    geometry(&P, xi + t * P.n, f, J);
    det[t] = det_inv(P.n, J, Ji);
    for (int d = 0; d < P.n; ++d) F[t * P.n + d] = f[d];
  }
  teardown(&P);
  return 0;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int or_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
