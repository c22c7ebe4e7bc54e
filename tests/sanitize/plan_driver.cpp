// Host-only run of the assembly planner (csrc/plan.cpp) under the address and
// undefined-behaviour sanitizers: problem validation, the 1-D tables, the
// interpolation set-ups of the three surrogate variants, and the tile lists,
// checked for the rows they must cover.  No HIP call is made.
#include <cmath>
#include <cstdio>
#include <vector>

#include "igs_internal.h"

using namespace igs;

static int fails = 0;
#define CHECK(c, ...)                      \
  do {                                     \
    if (!(c)) {                            \
      std::printf("FAIL %s: ", #c);        \
      std::printf(__VA_ARGS__);            \
      std::printf("\n");                   \
      ++fails;                             \
    }                                      \
  } while (0)

static igs_problem problem(int n, int p, int e1, int e2, int e3, int geom = IGS_GEOM_SINE) {
  igs_problem pb{};
  pb.n = n;
  pb.p = p;
  pb.nelem[0] = e1;
  pb.nelem[1] = e2;
  pb.nelem[2] = e3;
  pb.batch = 1;
  pb.geom.kind = geom;
  pb.geom.a = 0.05;
  pb.coef.kind = IGS_COEF_CONST;
  pb.coef.c0 = 1.0;
  return pb;
}

// rows covered by a tile list, counted per flat row index
static std::vector<int> cover(const Dims& d, const std::vector<QTile>& t, size_t from, size_t to) {
  std::vector<int> c(d.N, 0);
  for (size_t k = from; k < to; ++k) {
    const QTile& q = t[k];
    for (int z = q.z0; z < q.z1; ++z)
      for (int y = 0; y < (d.n == 3 ? q.ny : 1); ++y)
        for (int x = 0; x < q.nx; ++x) {
          const int64_t r = d.n == 3 ? (q.i1 + x) + int64_t(d.m[0]) * ((q.i2 + y) + int64_t(d.m[1]) * z)
                                     : (q.i1 + x) + int64_t(d.m[0]) * z;
          if (r >= 0 && r < d.N) ++c[r];
          else ++fails;
        }
  }
  return c;
}

static void index_of(const Dims& d, int64_t r, int* i) {
  i[0] = int(r % d.m[0]);
  i[1] = int((r / d.m[0]) % d.m[1]);
  i[2] = d.n == 3 ? int(r / (int64_t(d.m[0]) * d.m[1])) : 0;
}

static bool in_set(const std::vector<int>& s, int v) {
  for (int x : s)
    if (x == v) return true;
  return false;
}

// spline values of every evaluated index sum to 1 (partition of unity)
static void check_unity(const std::vector<double>& eb, int q, int lo, int hi, const char* what) {
  for (int i = lo; i <= hi; ++i) {
    double s = 0.0;
    for (int c = 0; c <= q; ++c) s += eb[size_t(i) * (q + 1) + c];
    CHECK(std::fabs(s - 1.0) < 1e-12, "%s index %d sum %.17g", what, i, s);
  }
}

int main() {
  setvbuf(stdout, nullptr, _IONBF, 0);
  // validation
  {
    Dims d;
    igs_problem bad = problem(4, 2, 10, 10, 10);
    CHECK(make_dims(&bad, &d) != IGS_OK, "n = 4 accepted");
    bad = problem(3, 0, 10, 10, 10);
    CHECK(make_dims(&bad, &d) != IGS_OK, "p = 0 accepted");
    bad = problem(2, 2, 0, 10, 1);
    CHECK(make_dims(&bad, &d) != IGS_OK, "nelem = 0 accepted");
  }
  const int cases[][6] = {{2, 2, 30, 27, 1, 4}, {2, 3, 41, 33, 1, 5}, {3, 2, 16, 14, 15, 3}, {3, 3, 18, 17, 19, 2},
                          {3, 1, 17, 13, 15, 3}, {3, 4, 21, 20, 21, 3}};
  for (const auto& cs : cases) {
    igs_problem pb = problem(cs[0], cs[1], cs[2], cs[3], cs[4]);
    Dims d;
    if (make_dims(&pb, &d) != IGS_OK) {
      CHECK(false, "valid problem rejected");
      continue;
    }
    const int M = cs[5], q = 3, p = d.p;
    std::printf("n=%d p=%d nelem=%d,%d,%d M=%d\n", d.n, p, cs[2], cs[3], cs[4], M);
    HostTables ht;
    build_tables(&pb, d, &ht);
    const int tx = d.n == 3 ? 7 : 64, ty = d.n == 3 ? 2 : 1, zc = 5;
    // full assembly tiles: every row once
    {
      std::vector<QTile> t = tiles_all(d, tx, ty, zc);
      std::vector<int> c = cover(d, t, 0, t.size());
      for (int64_t r = 0; r < d.N; ++r) CHECK(c[r] == 1, "tiles_all row %lld covered %d times", (long long)r, c[r]);
    }
    // analysis-domain surrogate
    {
      HostInterp hi;
      int box[3] = {1, 1, 1};
      const igs_status st = build_interp(d, IGS_STIFFNESS, M, q, box, &hi);
      CHECK(st == IGS_OK, "build_interp status %d", int(st));
      if (st != IGS_OK) continue;
      for (int k = 0; k < d.n; ++k) check_unity(hi.eb[k], q, hi.samp[k].front(), hi.samp[k].back(), "lattice");
      int groups[3];
      std::vector<QTile> t = tiles_surrogate(d, hi.samp, tx, ty, zc, groups);
      std::vector<int> c = cover(d, t, 0, size_t(groups[0] + groups[1]));
      std::vector<int> cs2 = cover(d, t, size_t(groups[0] + groups[1]), t.size());
      for (int64_t r = 0; r < d.N; ++r) {
        int i[3];
        index_of(d, r, i);
        bool inner = true, samp = true;
        for (int k = 0; k < d.n; ++k) {
          inner = inner && i[k] >= 2 * p && i[k] <= d.m[k] - 2 * p - 1;
          samp = samp && in_set(hi.samp[k], i[k]);
        }
        CHECK(c[r] == (inner ? 0 : 1), "surrogate boundary row %lld covered %d times", (long long)r, c[r]);
        if (samp) CHECK(cs2[r] >= 1, "sample row %lld not covered", (long long)r);
      }
    }
    // face/edge
    {
      HostInterp hi;
      int box[3] = {1, 1, 1};
      CHECK(build_interp_fe(d, IGS_STIFFNESS, M, q, box, &hi) == IGS_OK, "build_interp_fe");
      int groups[3];
      std::vector<QTile> t = tiles_fe(d, hi.samp, tx, ty, zc, groups);
      std::vector<int> c = cover(d, t, 0, t.size());
      for (int64_t r = 0; r < d.N && d.n == 3; ++r) {
        int i[3];
        index_of(d, r, i);
        bool samp = true;
        for (int k = 0; k < d.n; ++k) samp = samp && in_set(hi.samp[k], i[k]);
        CHECK(c[r] == (samp ? 1 : 0), "face/edge row %lld covered %d times", (long long)r, c[r]);
      }
    }
    // per-delta domains
    {
      HostInterpPD hi;
      CHECK(build_interp_pd(d, IGS_STIFFNESS, M, q, &hi) == IGS_OK, "build_interp_pd");
      for (int k = 0; k < d.n; ++k)
        for (int e = 0; e < d.W; ++e) {
          CHECK(hi.lo[k][e] == p + std::max(0, p - e) && hi.hi[k][e] == d.m[k] - p - 1 - std::max(0, e - p),
                "per-delta range d=%d e=%d", k, e);
          for (int i = hi.lo[k][e]; i <= hi.hi[k][e]; ++i) {
            double s = 0.0;
            for (int c = 0; c <= q; ++c) s += hi.eb[k][(size_t(e) * (q + 1) + c) * d.m[k] + i];
            CHECK(std::fabs(s - 1.0) < 1e-12, "per-delta unity d=%d e=%d i=%d", k, e, i);
            const int f = hi.ef[k][size_t(e) * d.m[k] + i];
            CHECK(f >= 0 && f + q < hi.S[k][e], "per-delta span d=%d e=%d i=%d", k, e, i);
          }
          for (int r = 0; r < hi.S[k][e]; ++r) {
            const int u = hi.pos[k][size_t(e) * hi.smax + r];
            CHECK(u >= 0 && u < int(hi.U[k].size()), "per-delta position");
          }
        }
      int sg[2];
      std::vector<QTile> t = tiles_shell(d, p, tx, ty, zc, sg);
      std::vector<int> c = cover(d, t, 0, t.size());
      for (int64_t r = 0; r < d.N; ++r) {
        int i[3];
        index_of(d, r, i);
        bool card = true;
        for (int k = 0; k < d.n; ++k) card = card && i[k] >= p && i[k] <= d.m[k] - p - 1;
        CHECK(c[r] == (card ? 0 : 1), "shell row %lld covered %d times", (long long)r, c[r]);
      }
    }
  }
  std::printf("plan driver: %d failures\n", fails);
  return fails ? 1 : 0;
}
