/* Run of the oracle's C part under the address and undefined-behaviour
 * sanitizers: every entry point on small 2D and 3D problems (all maps and
 * coefficient kinds, both forms, coefficient derivatives), with the invariants
 * that need no reference: Gauss weights sum to 2, B-splines sum to 1,
 * stiffness rows sum to 0, invalid input is rejected. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int or_gauss(int nq, double* x, double* w);
int or_basis(int nel, int p, int k, double x, double* val, double* der);
int or_rows(const int32_t* ip, const double* dp, const double* cc, int form, int dcoef, const int64_t* rows,
            int64_t nrows, double* out);
int or_rhs(const int32_t* ip, const double* dp, const double* cc, int src, double c, const int64_t* rows,
           int64_t nrows, double* out);
int or_map(const int32_t* ip, const double* dp, const double* xi, int64_t npts, double* F, double* det);

static int fails = 0;
#define CHECK(c, msg)                              \
  do {                                             \
    if (!(c)) {                                    \
      printf("FAIL %s: %s\n", #c, msg);            \
      ++fails;                                     \
    }                                              \
  } while (0)

int main(void) {
  for (int nq = 1; nq <= 10; ++nq) {
    double x[10], w[10], s = 0.0;
    CHECK(or_gauss(nq, x, w) == 0, "gauss");
    for (int k = 0; k < nq; ++k) s += w[k];
    CHECK(fabs(s - 2.0) < 1e-13, "gauss weights");
  }
  /* half-open spans: at x = 1 every function is 0 (only interior points are used) */
  for (int p = 1; p <= 4; ++p)
    for (int t = 0; t < 20; ++t) {
      double x = t / 20.0, s = 0.0, v, dv;
      for (int k = 0; k < 9 + p; ++k) {
        or_basis(9, p, k, x, &v, &dv);
        s += v;
      }
      CHECK(fabs(s - 1.0) < 1e-13, "partition of unity");
    }
  /* n, p, nelem x3, nq, geom, coef, cdeg, cn x3 */
  const int32_t cases[][12] = {{2, 2, 9, 7, 1, 0, 1, 0, 0, 1, 1, 1},  {3, 3, 6, 5, 7, 0, 1, 1, 0, 1, 1, 1},
                               {2, 3, 8, 8, 1, 0, 2, 3, 2, 4, 4, 1},  {3, 1, 5, 4, 6, 0, 0, 2, 3, 5, 5, 5},
                               {3, 2, 4, 5, 4, 0, 2, 0, 0, 1, 1, 1},  {2, 4, 11, 9, 1, 0, 1, 1, 0, 1, 1, 1}};
  const double dp[3] = {0.05, 1.0, 0.5};
  double cc[125];
  for (int k = 0; k < 125; ++k) cc[k] = 0.3 * sin(0.7 * k);
  for (size_t c = 0; c < sizeof(cases) / sizeof(cases[0]); ++c) {
    const int32_t* ip = cases[c];
    const int n = ip[0], p = ip[1];
    int64_t N = 1;
    int S = 1;
    for (int d = 0; d < n; ++d) {
      N *= ip[2 + d] + p;
      S *= 2 * p + 1;
    }
    int64_t* rows = malloc(sizeof(int64_t) * N);
    double* out = malloc(sizeof(double) * N * S);
    for (int64_t r = 0; r < N; ++r) rows[r] = r;
    for (int form = 0; form <= 1; ++form) {
      CHECK(or_rows(ip, dp, cc, form, -1, rows, N, out) == 0, "rows");
      if (form == 0) {
        double mx = 0.0, worst = 0.0;
        for (int64_t r = 0; r < N * S; ++r) mx = fmax(mx, fabs(out[r]));
        for (int64_t r = 0; r < N; ++r) {
          double s = 0.0;
          for (int k = 0; k < S; ++k) s += out[r * S + k];
          worst = fmax(worst, fabs(s));
        }
        CHECK(worst < 1e-12 * mx, "stiffness row sums");
      }
    }
    if (ip[7] >= 2) CHECK(or_rows(ip, dp, cc, 0, 1, rows, N, out) == 0, "coefficient derivative rows");
    CHECK(or_rhs(ip, dp, cc, 1, 2.0, rows, N, out) == 0, "rhs");
    double xi[6] = {0.1, 0.2, 0.3, 0.9, 0.5, 0.7}, F[6], det[2];
    CHECK(or_map(ip, dp, xi, 2, F, det) == 0, "map");
    CHECK(det[0] > 0.0 && det[1] > 0.0, "map Jacobian");
    int64_t badrow = N;
    CHECK(or_rows(ip, dp, cc, 0, -1, &badrow, 1, out) != 0, "out-of-range row rejected");
    free(rows);
    free(out);
  }
  const int32_t bad[12] = {4, 2, 5, 5, 5, 0, 0, 0, 0, 1, 1, 1};
  int64_t r0 = 0;
  double o[1000];
  CHECK(or_rows(bad, dp, cc, 0, -1, &r0, 1, o) != 0, "n = 4 rejected");
  printf("oracle driver: %d failures\n", fails);
  return fails ? 1 : 0;
}
