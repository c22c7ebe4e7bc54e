// Host-side planning for libigs: problem validation, 1-D quadrature and
// B-spline tables, the surrogate's sample lattice and interpolation matrices,
// and the tile lists that drive the quadrature kernels.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "igs_internal.h"

namespace igs {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// Gauss-Legendre rule on [-1,1] (ascending nodes): Newton's method on
// P_n(x) = 0 from Tricomi's asymptotic first guess, with P_n and P_{n-1} from
// Bonnet's recurrence; w_k = 2 / ((1 - x_k^2) P_n'(x_k)^2).
void gauss_rule(int n, std::vector<double>* x, std::vector<double>* w) {
  x->assign(n, 0.0);
  w->assign(n, 0.0);
  for (int k = 1; k <= n; ++k) {
    double theta = kPi * (4.0 * k - 1.0) / (4.0 * n + 2.0);
    double z = (1.0 - (n - 1.0) / (8.0 * n * n * n)) * std::cos(theta);
    double dpn = 1.0;
    for (int it = 0; it < 64; ++it) {
      double pm = 1.0, pn = z;
      for (int j = 1; j < n; ++j) {
        double pk = ((2.0 * j + 1.0) * z * pn - j * pm) / (j + 1.0);
        pm = pn;
        pn = pk;
      }
      if (n == 1) { pn = z; pm = 1.0; }
      dpn = n * (pm - z * pn) / (1.0 - z * z);
      double step = pn / dpn;
      z -= step;
      if (std::fabs(step) <= 4e-17) break;
    }
    double pm = 1.0, pn = z;
    for (int j = 1; j < n; ++j) {
      double pk = ((2.0 * j + 1.0) * z * pn - j * pm) / (j + 1.0);
      pm = pn;
      pn = pk;
    }
    if (n == 1) { pn = z; pm = 1.0; }
    dpn = n * (pm - z * pn) / (1.0 - z * z);
    (*x)[n - k] = z;  // cos-ordered guesses descend
    (*w)[n - k] = 2.0 / ((1.0 - z * z) * dpn * dpn);
  }
}

// The deg+1 B-splines alive on knot span `span` (t[span] <= x < t[span+1]) by
// the triangular (de Boor) scheme: out[r] = N_{span-deg+r, deg}(x).
void span_basis(const std::vector<double>& t, int span, int deg, double x, double* out) {
  double left[16], right[16];
  out[0] = 1.0;
  for (int j = 1; j <= deg; ++j) {
    left[j] = x - t[span + 1 - j];
    right[j] = t[span + j] - x;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      double tmp = out[r] / (right[r + 1] + left[j - r]);
      out[r] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    out[j] = saved;
  }
}

// Values and first derivatives of the deg+1 B-splines alive on `span`.
void span_basis_d(const std::vector<double>& t, int span, int deg, double x, double* val, double* der) {
  span_basis(t, span, deg, x, val);
  if (deg == 0) {
    der[0] = 0.0;
    return;
  }
  double low[16];
  span_basis(t, span, deg - 1, x, low);  // functions span-deg+1 .. span
  for (int r = 0; r <= deg; ++r) {
    int i = span - deg + r;  // function index
    double a = 0.0, b = 0.0;
    if (r >= 1) {
      double den = t[i + deg] - t[i];
      if (den > 0.0) a = deg * low[r - 1] / den;
    }
    if (r <= deg - 1) {
      double den = t[i + deg + 1] - t[i + 1];
      if (den > 0.0) b = deg * low[r] / den;
    }
    der[r] = a - b;
  }
}

std::vector<double> open_uniform(int nel, int deg) {
  int m = nel + deg;
  std::vector<double> t(m + deg + 1);
  for (int k = 0; k <= m + deg; ++k) t[k] = (k <= deg) ? 0.0 : (k >= m ? 1.0 : double(k - deg) / nel);
  return t;
}

// LU with partial pivoting and explicit inverse of a dense n x n matrix.
bool invert(std::vector<double> a, int n, std::vector<double>* inv) {
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int pr = k;
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(a[r * n + k]) > std::fabs(a[pr * n + k])) pr = r;
    if (a[pr * n + k] == 0.0) return false;
    piv[k] = pr;
    if (pr != k)
      for (int c = 0; c < n; ++c) std::swap(a[k * n + c], a[pr * n + c]);
    for (int r = k + 1; r < n; ++r) {
      double f = a[r * n + k] / a[k * n + k];
      a[r * n + k] = f;
      for (int c = k + 1; c < n; ++c) a[r * n + c] -= f * a[k * n + c];
    }
  }
  inv->assign(size_t(n) * n, 0.0);
  std::vector<double> col(n);
  for (int j = 0; j < n; ++j) {
    std::fill(col.begin(), col.end(), 0.0);
    col[j] = 1.0;
    for (int k = 0; k < n; ++k) std::swap(col[k], col[piv[k]]);
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < r; ++c) col[r] -= a[r * n + c] * col[c];
    for (int r = n - 1; r >= 0; --r) {
      for (int c = r + 1; c < n; ++c) col[r] -= a[r * n + c] * col[c];
      col[r] /= a[r * n + r];
    }
    for (int r = 0; r < n; ++r) (*inv)[size_t(r) * n + j] = col[r];
  }
  return true;
}

}  // namespace

igs_status make_dims(const igs_problem* pb, Dims* d) {
  if (!pb || !d) return IGS_ERR_ARG;
  if (pb->n < 2 || pb->n > 3) return IGS_ERR_ARG;
  if (pb->p < 1) return IGS_ERR_ARG;
  if (pb->p > kMaxP) return IGS_ERR_UNSUPPORTED;
  if (pb->batch < 1) return IGS_ERR_ARG;
  if (pb->nquad != 0 && pb->nquad != pb->p + 1) return pb->nquad < 0 ? IGS_ERR_ARG : IGS_ERR_UNSUPPORTED;
  std::memset(d, 0, sizeof(*d));
  d->n = pb->n;
  d->p = pb->p;
  d->nq = pb->p + 1;
  d->W = 2 * pb->p + 1;
  d->S = 1;
  d->N = 1;
  d->batch = pb->batch;
  for (int k = 0; k < 3; ++k) {
    if (k < pb->n) {
      if (pb->nelem[k] < 1 || pb->nelem[k] > (1 << 20)) return IGS_ERR_ARG;
      d->nelem[k] = pb->nelem[k];
      d->m[k] = pb->nelem[k] + pb->p;
      d->S *= d->W;
      d->N *= d->m[k];
    } else {
      d->nelem[k] = 1;
      d->m[k] = 1;
    }
  }
  if (d->N > (int64_t(1) << 31)) return IGS_ERR_UNSUPPORTED;
  d->ld = (d->N + 64) / 64 * 64;  // strictly greater than N: the fill parks dead lanes in the padding
  // optional knot vectors must be the open uniform ones (Sec. 2.2)
  for (int k = 0; k < pb->n; ++k) {
    if (!pb->knots[k]) continue;
    std::vector<double> t = open_uniform(d->nelem[k], d->p);
    for (size_t r = 0; r < t.size(); ++r)
      if (std::fabs(pb->knots[k][r] - t[r]) > 1e-12) return IGS_ERR_KNOTS;
  }
  // geometry and coefficient
  if (pb->geom.kind < IGS_GEOM_IDENTITY || pb->geom.kind > IGS_GEOM_POLY2) return IGS_ERR_ARG;
  if (!std::isfinite(pb->geom.a)) return IGS_ERR_ARG;
  const igs_coef& c = pb->coef;
  if (c.kind < IGS_COEF_CONST || c.kind > IGS_COEF_EXP_SPLINE) return IGS_ERR_ARG;
  if (c.kind == IGS_COEF_SPLINE || c.kind == IGS_COEF_EXP_SPLINE) {
    if (!c.coef) return IGS_ERR_ARG;
    if (c.degree < 1 || c.degree > 5) return IGS_ERR_UNSUPPORTED;
    for (int k = 0; k < pb->n; ++k)
      if (c.ncoef[k] <= c.degree || c.ncoef[k] > 64) return IGS_ERR_ARG;
  }
  return IGS_OK;
}

void build_tables(const igs_problem* pb, const Dims& d, HostTables* t) {
  std::vector<double> gx, gw;
  gauss_rule(d.nq, &gx, &gw);
  const int np1 = d.p + 1;
  const bool spline = pb->coef.kind == IGS_COEF_SPLINE || pb->coef.kind == IGS_COEF_EXP_SPLINE;
  const int cdeg = spline ? pb->coef.degree : 0;
  for (int k = 0; k < d.n; ++k) {
    const int ne = d.nelem[k];
    const int Q = ne * d.nq;
    const double h = 1.0 / ne;
    std::vector<double> knots = open_uniform(ne, d.p);
    t->x[k].resize(Q);
    t->w[k].resize(Q);
    t->bv[k].resize(size_t(Q) * np1);
    t->bd[k].resize(size_t(Q) * np1);
    t->bpr[k].resize(size_t(Q) * np1 * np1 * 4);
    t->trig[k].resize(size_t(Q) * 4);
    std::vector<double> ck;
    int cne = 0;
    if (spline) {
      cne = pb->coef.ncoef[k] - cdeg;
      ck = open_uniform(cne, cdeg);
      t->cb[k].resize(size_t(Q) * (cdeg + 1));
      t->cf[k].resize(Q);
    } else {
      t->cb[k].assign(1, 0.0);
      t->cf[k].assign(1, 0);
    }
    for (int e = 0; e < ne; ++e)
      for (int g = 0; g < d.nq; ++g) {
        const int qi = e * d.nq + g;
        const double x = (e + 0.5 * (gx[g] + 1.0)) * h;
        t->x[k][qi] = x;
        t->w[k][qi] = 0.5 * h * gw[g];
        span_basis_d(knots, e + d.p, d.p, x, &t->bv[k][size_t(qi) * np1], &t->bd[k][size_t(qi) * np1]);
        {
          const double* v = &t->bv[k][size_t(qi) * np1];
          const double* dv = &t->bd[k][size_t(qi) * np1];
          for (int a = 0; a < np1; ++a)
            for (int c = 0; c < np1; ++c) {
              double* o = &t->bpr[k][((size_t(qi) * np1 + a) * np1 + c) * 4];
              o[0] = v[a] * v[c];
              o[1] = v[a] * dv[c];
              o[2] = dv[a] * v[c];
              o[3] = dv[a] * dv[c];
            }
        }
        t->trig[k][qi * 4 + 0] = std::sin(kPi * x);
        t->trig[k][qi * 4 + 1] = kPi * std::cos(kPi * x);
        t->trig[k][qi * 4 + 2] = std::sin(2.0 * kPi * x);
        t->trig[k][qi * 4 + 3] = 2.0 * kPi * std::cos(2.0 * kPi * x);
        if (spline) {
          int sp = cdeg + std::min(cne - 1, int(std::floor(x * cne)));
          while (sp > cdeg && x < ck[sp]) --sp;
          while (sp < cne + cdeg - 1 && x >= ck[sp + 1]) ++sp;
          span_basis(ck, sp, cdeg, x, &t->cb[k][size_t(qi) * (cdeg + 1)]);
          t->cf[k][qi] = sp - cdeg;
        }
      }
  }
}

igs_status sample_lattice(int m, int p, int M, std::vector<int>* s) {
  const int lo = 2 * p, hi = m - 2 * p - 1;
  if (hi < lo) return IGS_ERR_SAMPLES;
  s->clear();
  for (int v = lo; v <= hi; v += M) s->push_back(v);
  if (s->back() != hi) s->push_back(hi);
  return IGS_OK;
}

// Degree-q interpolation on the sample indices s (increasing): the inverse
// collocation matrix (row-major S x S) and, for every index i in [s_0,
// s_{S-1}], the first spline coefficient alive at i and the q+1 values there
// (ef[i], eb[i (q+1) + c]; ef and eb span m indices).
static igs_status spline_1d(const std::vector<int>& s, int q, int m, std::vector<double>* ginv, std::vector<int>* ef,
                            std::vector<double>* eb) {
  const int S = int(s.size());
  if (S < q + 1) return IGS_ERR_SAMPLES;
  // knots: end samples repeated q+1 times; interior = samples (odd q,
  // not-a-knot) or midpoints of consecutive samples (even q)
  std::vector<double> t;
  for (int r = 0; r <= q; ++r) t.push_back(s[0]);
  if (q % 2 == 1) {
    for (int r = (q + 1) / 2; r <= S - 1 - (q + 1) / 2; ++r) t.push_back(s[r]);
  } else {
    for (int r = q / 2; r <= S - 2 - q / 2; ++r) t.push_back(0.5 * (s[r] + s[r + 1]));
  }
  for (int r = 0; r <= q; ++r) t.push_back(s[S - 1]);
  // span of a point: last span with t[k] <= x, capped at the last nonempty one
  auto span_of = [&](double x) {
    int sp = q;
    while (sp + 1 < S && t[sp + 1] <= x) ++sp;
    return sp;
  };
  std::vector<double> G(size_t(S) * S, 0.0);
  double vals[16];
  for (int r = 0; r < S; ++r) {
    int sp = span_of(s[r]);
    span_basis(t, sp, q, s[r], vals);
    for (int c = 0; c <= q; ++c) G[size_t(r) * S + sp - q + c] = vals[c];
  }
  if (!invert(G, S, ginv)) return IGS_ERR_SAMPLES;
  ef->assign(m, 0);
  eb->assign(size_t(m) * (q + 1), 0.0);
  for (int i = s[0]; i <= s[S - 1]; ++i) {
    int sp = span_of(i);
    span_basis(t, sp, q, i, vals);
    (*ef)[i] = sp - q;
    for (int c = 0; c <= q; ++c) (*eb)[size_t(i) * (q + 1) + c] = vals[c];
  }
  return IGS_OK;
}

igs_status build_interp(const Dims& d, int form, int M, int q, int boxlen[3], HostInterp* hi) {
  hi->q = q;
  for (int k = 0; k < d.n; ++k) {
    igs_status st = sample_lattice(d.m[k], d.p, M, &hi->samp[k]);
    if (st != IGS_OK) return st;
    const int S = int(hi->samp[k].size());
    const std::vector<int>& s = hi->samp[k];
    st = spline_1d(s, q, d.m[k], &hi->ginv[k], &hi->ef[k], &hi->eb[k]);
    if (st != IGS_OK) return st;
    // widest coefficient span of any window of boxlen[k] consecutive indices
    int nc = 0;
    for (int i = s[0]; i <= s[S - 1]; ++i) {
      int j = std::min(s[S - 1], i + boxlen[k] - 1);
      nc = std::max(nc, hi->ef[k][j] - hi->ef[k][i] + q + 1);
    }
    hi->nc[k] = std::min(nc, S);
  }
  for (int k = d.n; k < 3; ++k) hi->nc[k] = 1;
  for (int k = 0; k < 3; ++k) {
    hi->lo[k] = k < d.n ? 2 * d.p : 0;
    hi->hi[k] = k < d.n ? d.m[k] - 2 * d.p - 1 : 0;
    hi->flo[k] = 0;
    hi->fhi[k] = k < d.n ? int(hi->samp[k].size()) : 1;
  }
  hi->upslot.clear();
  const int sc = (d.S - 1) / 2;
  for (int s = 0; s < d.S; ++s)
    if (s > sc || (form == IGS_MASS && s == sc)) hi->upslot.push_back(s);
  return IGS_OK;
}

igs_status build_interp_fe(const Dims& d, int form, int M, int q, int boxlen[3], HostInterp* hi) {
  // the lattice spline of each direction, as for the analysis-domain surrogate
  int one[3] = {1, 1, 1};
  HostInterp base;
  igs_status st = build_interp(d, form, M, q, one, &base);
  if (st != IGS_OK) return st;
  const int p = d.p;
  hi->q = q;
  hi->upslot = base.upslot;
  for (int k = 0; k < d.n; ++k) {
    const int m = d.m[k], S = int(base.samp[k].size()), Sx = S + 4 * p;
    // augmented coefficient index: low layers 0..2p-1, lattice 2p..2p+S-1,
    // high layers after; increasing with the fine index
    hi->samp[k].clear();
    for (int i = 0; i < 2 * p; ++i) hi->samp[k].push_back(i);
    for (int v : base.samp[k]) hi->samp[k].push_back(v);
    for (int i = m - 2 * p; i < m; ++i) hi->samp[k].push_back(i);
    hi->ginv[k].assign(size_t(Sx) * Sx, 0.0);
    for (int r = 0; r < Sx; ++r) {
      if (r < 2 * p || r >= 2 * p + S) {
        hi->ginv[k][size_t(r) * Sx + r] = 1.0;
      } else {
        for (int c = 0; c < S; ++c)
          hi->ginv[k][size_t(r) * Sx + 2 * p + c] = base.ginv[k][size_t(r - 2 * p) * S + c];
      }
    }
    hi->ef[k].assign(m, 0);
    hi->eb[k].assign(size_t(m) * (q + 1), 0.0);
    for (int i = 0; i < m; ++i) {
      if (i >= 2 * p && i <= m - 2 * p - 1) {
        hi->ef[k][i] = 2 * p + base.ef[k][i];
        for (int c = 0; c <= q; ++c) hi->eb[k][size_t(i) * (q + 1) + c] = base.eb[k][size_t(i) * (q + 1) + c];
      } else {
        // a layer: weight 1 at its own coefficient, inside a window of q+1
        const int pos = i < 2 * p ? i : 2 * p + S + (i - (m - 2 * p));
        const int f = std::min(pos, Sx - q - 1);
        hi->ef[k][i] = f;
        hi->eb[k][size_t(i) * (q + 1) + (pos - f)] = 1.0;
      }
    }
    int nc = 0;
    for (int i = 0; i < m; ++i) {
      const int j = std::min(m - 1, i + boxlen[k] - 1);
      nc = std::max(nc, hi->ef[k][j] - hi->ef[k][i] + q + 1);
    }
    hi->nc[k] = std::min(nc, Sx);
    hi->lo[k] = 0;
    hi->hi[k] = m - 1;
    hi->flo[k] = 2 * p;
    hi->fhi[k] = 2 * p + S;
  }
  for (int k = d.n; k < 3; ++k) {
    hi->nc[k] = 1;
    hi->lo[k] = hi->hi[k] = 0;
    hi->flo[k] = 0;
    hi->fhi[k] = 1;
  }
  return IGS_OK;
}

igs_status build_interp_pd(const Dims& d, int form, int M, int q, HostInterpPD* hi) {
  const int p = d.p, W = 2 * p + 1;
  if (W > kMaxW) return IGS_ERR_UNSUPPORTED;
  hi->q = q;
  hi->p = p;
  hi->W = W;
  hi->smax = 1;
  std::vector<int> samp[3][kMaxW];
  for (int k = 0; k < d.n; ++k) {
    std::vector<int> base;
    igs_status st = sample_lattice(d.m[k], p, M, &base);
    if (st != IGS_OK) return st;
    const int m = d.m[k];
    // common set: band [p, 2p), the lattice, band [m - 2p, m - p)
    hi->U[k].clear();
    for (int i = p; i < 2 * p; ++i) hi->U[k].push_back(i);
    for (int v : base) hi->U[k].push_back(v);
    for (int i = m - 2 * p; i < m - p; ++i) hi->U[k].push_back(i);
    for (int e = 0; e < W; ++e) {
      const int dd = e - p;
      const int lo = p + std::max(0, -dd), hi_ = m - p - 1 - std::max(0, dd);
      for (int v : hi->U[k])
        if (v >= lo && v <= hi_) samp[k][e].push_back(v);
      hi->S[k][e] = int(samp[k][e].size());
      hi->lo[k][e] = lo;
      hi->hi[k][e] = hi_;
      if (hi->S[k][e] < q + 1) return IGS_ERR_SAMPLES;
      hi->smax = std::max(hi->smax, hi->S[k][e]);
    }
  }
  const int sm = hi->smax;
  for (int k = 0; k < 3; ++k) {
    hi->pos[k].clear();
    hi->ginv[k].clear();
    hi->ef[k].clear();
    hi->eb[k].clear();
    if (k >= d.n) {
      for (int e = 0; e < W; ++e) hi->S[k][e] = 1, hi->lo[k][e] = hi->hi[k][e] = 0;
      continue;
    }
    const int m = d.m[k];
    hi->pos[k].assign(size_t(W) * sm, 0);
    hi->ginv[k].assign(size_t(W) * sm * sm, 0.0);
    hi->ef[k].assign(size_t(W) * m, 0);
    hi->eb[k].assign(size_t(W) * (q + 1) * m, 0.0);
    for (int e = 0; e < W; ++e) {
      const std::vector<int>& s = samp[k][e];
      const int S = int(s.size());
      for (int r = 0; r < S; ++r)
        hi->pos[k][size_t(e) * sm + r] =
            int(std::lower_bound(hi->U[k].begin(), hi->U[k].end(), s[r]) - hi->U[k].begin());
      std::vector<double> gi, eb;
      std::vector<int> ef;
      igs_status st = spline_1d(s, q, m, &gi, &ef, &eb);
      if (st != IGS_OK) return st;
      for (int r = 0; r < S; ++r)
        for (int c = 0; c < S; ++c) hi->ginv[k][(size_t(e) * sm + r) * sm + c] = gi[size_t(r) * S + c];
      for (int i = 0; i < m; ++i) {
        hi->ef[k][size_t(e) * m + i] = ef[i];
        for (int c = 0; c <= q; ++c) hi->eb[k][(size_t(e) * (q + 1) + c) * m + i] = eb[size_t(i) * (q + 1) + c];
      }
    }
  }
  hi->upslot.clear();
  const int sc = (d.S - 1) / 2;
  for (int s = 0; s < d.S; ++s)
    if (s > sc || (form == IGS_MASS && s == sc)) hi->upslot.push_back(s);
  return IGS_OK;
}

std::vector<QTile> tiles_all(const Dims& d, int tx, int ty, int zchunk) {
  std::vector<QTile> out;
  const int mz = (d.n == 3) ? d.m[2] : d.m[1];
  const int my = (d.n == 3) ? d.m[1] : 1;
  for (int z0 = 0; z0 < mz; z0 += zchunk)
    for (int i2 = 0; i2 < my; i2 += (d.n == 3 ? ty : 1))
      for (int i1 = 0; i1 < d.m[0]; i1 += tx) {
        QTile t;
        t.i1 = i1;
        t.nx = std::min(tx, d.m[0] - i1);
        t.i2 = i2;
        t.ny = (d.n == 3) ? std::min(ty, d.m[1] - i2) : 1;
        t.z0 = z0;
        t.z1 = std::min(mz, z0 + zchunk);
        out.push_back(t);
      }
  return out;
}

namespace {
void tile_rect(std::vector<QTile>* out, int x0, int x1, int y0, int y1, int tx, int ty, int z0, int z1, int zchunk) {
  if (x1 <= x0 || y1 <= y0 || z1 <= z0) return;
  for (int za = z0; za < z1; za += zchunk)
    for (int y = y0; y < y1; y += ty)
      for (int x = x0; x < x1; x += tx) {
        QTile t;
        t.i1 = x;
        t.nx = std::min(tx, x1 - x);
        t.i2 = y;
        t.ny = std::min(ty, y1 - y);
        t.z0 = za;
        t.z1 = std::min(z1, za + zchunk);
        out->push_back(t);
      }
}
}  // namespace

// Rows assembled by quadrature in the surrogate: every row outside the
// analysis domain [2p, m-2p-1]^n plus the sample lattice, in three groups.
// Group 0: rows of the analysis-domain pencils (pencils along i1, the flat
// index's fastest direction) outside the domain in i1.  Group 1: rows of the
// pencils outside the analysis domain in (i2, i3).  Group 2: the sample rows
// (single-row tiles in 3-D, line tiles in 2-D).  Groups 0 and 1 run as one
// launch; the list puts the long tiles (whole columns, chunked along the
// streamed direction) before the short end slabs so that the short ones fill
// the launch's tail.
std::vector<QTile> tiles_surrogate(const Dims& d, const std::vector<int> samp[3], int tx, int ty, int zchunk,
                                   int groups[3]) {
  std::vector<QTile> out;
  const int p = d.p;
  const int lo1 = 2 * p, hi1 = d.m[0] - 2 * p, lo2 = 2 * p, hi2 = d.m[1] - 2 * p;
  if (d.n == 3) {
    const int lo3 = 2 * p, hi3 = d.m[2] - 2 * p;
    // tiles are (i1, i2) rectangles streamed along i3
    tile_rect(&out, 0, lo1, lo2, hi2, tx, ty, lo3, hi3, zchunk);
    tile_rect(&out, hi1, d.m[0], lo2, hi2, tx, ty, lo3, hi3, zchunk);
    groups[0] = int(out.size());
    tile_rect(&out, 0, d.m[0], 0, lo2, tx, ty, 0, d.m[2], zchunk);
    tile_rect(&out, 0, d.m[0], hi2, d.m[1], tx, ty, 0, d.m[2], zchunk);
    tile_rect(&out, 0, d.m[0], lo2, hi2, tx, ty, 0, lo3, zchunk);
    tile_rect(&out, 0, d.m[0], lo2, hi2, tx, ty, hi3, d.m[2], zchunk);
    groups[1] = int(out.size()) - groups[0];
    for (int s3 : samp[2])
      for (int s2 : samp[1])
        for (int s1 : samp[0]) out.push_back(QTile{s1, s2, 1, 1, s3, s3 + 1});
  } else {
    // tiles are i1 ranges streamed along i2
    tile_rect(&out, 0, lo1, 0, 1, tx, 1, lo2, hi2, zchunk);
    tile_rect(&out, hi1, d.m[0], 0, 1, tx, 1, lo2, hi2, zchunk);
    groups[0] = int(out.size());
    tile_rect(&out, 0, d.m[0], 0, 1, tx, 1, 0, lo2, zchunk);
    tile_rect(&out, 0, d.m[0], 0, 1, tx, 1, hi2, d.m[1], zchunk);
    groups[1] = int(out.size()) - groups[0];
    // a 2-D tile computes tx consecutive i1 for every i2 it streams: the
    // sample rows of a lattice line i2 = s2 come from tiles over the line's
    // analysis range (its other rows are domain rows that the fill, which runs
    // later, overwrites), not from single-row tiles that would leave all but
    // one of a tile's tx lanes idle
    for (int s2 : samp[1]) tile_rect(&out, samp[0].front(), samp[0].back() + 1, 0, 1, tx, 1, s2, s2 + 1, 1);
  }
  groups[2] = int(out.size()) - groups[0] - groups[1];
  return out;
}

std::vector<QTile> tiles_shell(const Dims& d, int c, int tx, int ty, int zchunk, int groups[2]) {
  std::vector<QTile> out;
  const int lo1 = c, hi1 = d.m[0] - c, lo2 = c, hi2 = d.m[1] - c;
  if (d.n == 3) {
    const int lo3 = c, hi3 = d.m[2] - c;
    tile_rect(&out, 0, lo1, lo2, hi2, tx, ty, lo3, hi3, zchunk);
    tile_rect(&out, hi1, d.m[0], lo2, hi2, tx, ty, lo3, hi3, zchunk);
    groups[0] = int(out.size());
    tile_rect(&out, 0, d.m[0], 0, lo2, tx, ty, 0, d.m[2], zchunk);
    tile_rect(&out, 0, d.m[0], hi2, d.m[1], tx, ty, 0, d.m[2], zchunk);
    tile_rect(&out, 0, d.m[0], lo2, hi2, tx, ty, 0, lo3, zchunk);
    tile_rect(&out, 0, d.m[0], lo2, hi2, tx, ty, hi3, d.m[2], zchunk);
  } else {
    tile_rect(&out, 0, lo1, 0, 1, tx, 1, lo2, hi2, zchunk);
    tile_rect(&out, hi1, d.m[0], 0, 1, tx, 1, lo2, hi2, zchunk);
    groups[0] = int(out.size());
    tile_rect(&out, 0, d.m[0], 0, 1, tx, 1, 0, lo2, zchunk);
    tile_rect(&out, 0, d.m[0], 0, 1, tx, 1, hi2, d.m[1], zchunk);
  }
  groups[1] = int(out.size()) - groups[0];
  return out;
}

namespace {
// maximal runs [first, first + len) of consecutive values in a sorted set
std::vector<std::pair<int, int>> index_runs(const std::vector<int>& t) {
  std::vector<std::pair<int, int>> out;
  for (size_t a = 0; a < t.size();) {
    size_t b = a + 1;
    while (b < t.size() && t[b] == t[b - 1] + 1) ++b;
    out.push_back({t[a], int(b - a)});
    a = b;
  }
  return out;
}
}  // namespace

// Rows the face/edge surrogate assembles by quadrature: the tensor product of
// the per-direction sample sets (layers and lattice; samp from
// build_interp_fe).  3-D: the rows whose i1 lies in a run of the set (the 2p+1
// indices at each end) as tiles over (i1 run) x (i2 run or single index),
// streamed over each i3 run or single index -> groups[0]; the rows with an
// isolated i1 (a lattice index) as single-row tiles -> groups[2].  2-D: whole
// i1 lines over each run of consecutive i2 in the set (the extra rows are
// evaluated again by the fill) -> groups[0].
std::vector<QTile> tiles_fe(const Dims& d, const std::vector<int> samp[3], int tx, int ty, int zchunk,
                            int groups[3]) {
  std::vector<QTile> out;
  groups[0] = groups[1] = groups[2] = 0;
  if (d.n == 3) {
    const auto r1 = index_runs(samp[0]), r2 = index_runs(samp[1]), r3 = index_runs(samp[2]);
    for (const auto& z : r3)
      for (const auto& y : r2)
        for (const auto& x : r1)
          if (x.second > 1) tile_rect(&out, x.first, x.first + x.second, y.first, y.first + y.second, tx, ty, z.first,
                                      z.first + z.second, z.second);
    groups[0] = int(out.size());
    for (int s3 : samp[2])
      for (int s2 : samp[1])
        for (const auto& x : r1)
          if (x.second == 1) out.push_back(QTile{x.first, s2, 1, 1, s3, s3 + 1});
    groups[2] = int(out.size()) - groups[0];
    return out;
  }
  for (const auto& z : index_runs(samp[1])) tile_rect(&out, 0, d.m[0], 0, 1, tx, 1, z.first, z.first + z.second, zchunk);
  groups[0] = int(out.size());
  return out;
}

igs_status Arena::alloc(size_t bytes, hipStream_t s) {
  release();
  stream = s;
  size = bytes;
  used = 0;
  if (bytes == 0) return IGS_OK;
  if (pool) {
    const size_t off = padded(pool->used);
    if (off > pool->cap || bytes > pool->cap - off) return IGS_ERR_SCRATCH;
    base = pool->base + off;
    pool->used = off + bytes;
    return IGS_OK;
  }
  const hipError_t e = persistent ? hipMalloc(reinterpret_cast<void**>(&base), bytes)
                                  : hipMallocAsync(reinterpret_cast<void**>(&base), bytes, s);
  if (e != hipSuccess) {
    base = nullptr;
    return IGS_ERR_NOMEM;
  }
  return IGS_OK;
}

igs_status Arena::flush() {
  if (dhi <= dlo) return IGS_OK;
  const hipError_t e = hipMemcpyAsync(base + dlo, stage.data() + dlo, dhi - dlo, hipMemcpyHostToDevice, stream);
  dlo = ~size_t(0);
  dhi = 0;
  return e == hipSuccess ? IGS_OK : IGS_ERR_HIP;
}

void Arena::release() {
  if (base && !pool) (void)(persistent ? hipFree(base) : hipFreeAsync(base, stream));
  base = nullptr;
  size = used = 0;
  stage.clear();
  dlo = ~size_t(0);
  dhi = 0;
}

}  // namespace igs
