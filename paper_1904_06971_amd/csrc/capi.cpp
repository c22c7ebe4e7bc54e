// extern "C" entry points of libigs (declared in include/igs.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <vector>

#include "igs_internal.h"
#include "profile.h"

namespace igs {

// launchers defined in the kernel translation units
template <typename OutT>
hipError_t launch_quad(const KProblem& kp, int form, const QTile* tiles, int ntiles, bool rows, OutT* band,
                       hipStream_t s);
hipError_t launch_rhs(const KProblem& kp, const QTile* tiles, int ntiles, int src, double c, double* f, hipStream_t s);
void quad_tile_shape(int n, int p, int* tx, int* ty);
void rhs_tile_shape(int n, int* tx, int* ty);
template <typename BT>
hipError_t launch_fit(const KInterp<double>& ip, int n, int m1, int m2, int64_t ld, int S, int batch, const BT* band,
                      double* tmp0, double* tmp1, double* coef, const double* g0T, hipStream_t s);
template <typename T>
hipError_t launch_fill(const KInterp<T>& ip, int form, const Dims& d, const int* chunks, int nchunks, int chunk_rows,
                       int n2max, int n3max, const int4* dsl, const double* coef, T* band, hipStream_t s);
template <typename T>
size_t fill_lds_bytes(const KInterp<T>& ip, int npen, const Dims& d, int blk);
void fill_block_dims(const Dims& d, const std::vector<int> ef[3], int q, const std::vector<int>& chunks, int rows,
                     const int lo[3], const int hi[3], int* n2max, int* n3max);
std::vector<int> fill_chunks(const Dims& d, int rows, const int lo[3], const int hi[3]);
int fill_npen(const Dims& d, int rows);
bool fill_is_2d(const Dims& d);
bool fill2d_wide_fits(const Dims& d, int S1, size_t tsize);
bool fit_use_gemm(const KInterp<double>& ip, int n, int batch);
template <typename BT>
hipError_t launch_fit_gemm(const KInterp<double>& ip, int n, int m1, int m2, int64_t ld, int S, int batch,
                           const BT* band, double* tmp0, double* tmp1, double* coef, hipStream_t s);
int fill_chunk_rows(const Dims& d, int Sd1, int q, int nup);
template <typename T>
hipError_t launch_zero_pad(T* band, int64_t N, int64_t ld, int slots_total, hipStream_t s);
template <typename T>
hipError_t launch_copy(const KInterp<T>& ip, int form, const Dims& d, const int* rows, int nrows, T* band,
                       hipStream_t s);
// rows of the box [c, m_d - c - 1]^n within p of its edge (partners outside it)
std::vector<int> copy_rows(const Dims& d, int c);
template <typename BT>
hipError_t launch_fit_pd(const KInterpPD& ip, int n, int64_t ld, int S, int batch, const int* upslot, const BT* band,
                         double* tmp0, double* tmp1, double* coef, hipStream_t s);
template <typename T>
hipError_t launch_fill_pd(const KInterpPD& ip, int form, const Dims& d, const double* coef, T* band, hipStream_t s);
size_t fill_pd_lds_bytes(const KInterpPD& ip, int S);
igs_status launch_apply(const Dims& d, int dtype, const void* band, const void* x, void* y, int dirichlet,
                        hipStream_t s);
igs_status solve_cg(const Dims& d, const double* band64, const float* band32, const double* f, double* u, double rtol,
                    int maxit, igs_cg_info* info, hipStream_t s);
template <typename T>
hipError_t launch_apply_mf(const KInterp<T>& ip, int form, const Dims& d, const int* chunks, int nchunks,
                           int chunk_rows, int n2max, int n3max, const int4* dsl, const double* coef, const T* band,
                           const int* crow, int ncopy, const int* brow, int nbrow, const T* x, T* y, T* xm,
                           int dirichlet, bool x_masked, hipStream_t s);
std::vector<int> boundary_rows(const Dims& d);
igs_status solve_cg_op(const Dims& d, const std::function<igs_status(const double*, double*)>& A, const double* f,
                       double* u, double rtol, int maxit, igs_cg_info* info, hipStream_t s);
igs_status adjoint_weights_grad(const igs_problem* pb, const Dims& d, const KProblem& kp, int M, int q,
                                const double* x, const double* ybar, double* cbar, hipStream_t s);

#define HIP_TRY(x)                             \
  do {                                         \
    if ((x) != hipSuccess) return IGS_ERR_HIP; \
  } while (0)

// Device copy of the 1-D tables plus the error word.
struct Prepared {
  Dims d;
  HostTables ht;
  KProblem kp;
  Arena ar;
};

template <typename V>
static size_t vbytes(const V& v) {
  return padded(v.size() * sizeof(typename V::value_type));
}

// stages v in the arena; the copy happens at the arena's flush()
template <typename V>
static auto* upload(Arena& ar, const V& v, hipStream_t, igs_status*) {
  return ar.put(v.data(), v.size());
}

static igs_status prepare(const igs_problem* pb, hipStream_t s, Prepared* P) {
  igs_status st = make_dims(pb, &P->d);
  if (st != IGS_OK) return st;
  build_tables(pb, P->d, &P->ht);
  size_t bytes = padded(sizeof(int));
  for (int k = 0; k < P->d.n; ++k)
    bytes += vbytes(P->ht.x[k]) + vbytes(P->ht.w[k]) + vbytes(P->ht.bv[k]) + vbytes(P->ht.bd[k]) +
             vbytes(P->ht.bpr[k]) + vbytes(P->ht.trig[k]) + vbytes(P->ht.cb[k]) + vbytes(P->ht.cf[k]);
  st = P->ar.alloc(bytes, s);
  if (st != IGS_OK) return st;
  KProblem& kp = P->kp;
  std::memset(&kp, 0, sizeof(kp));
  kp.n = P->d.n;
  kp.p = P->d.p;
  kp.nq = P->d.nq;
  for (int k = 0; k < 3; ++k) {
    kp.nelem[k] = P->d.nelem[k];
    kp.m[k] = P->d.m[k];
  }
  kp.N = P->d.N;
  kp.ld = P->d.ld;
  kp.S = P->d.S;
  kp.batch = P->d.batch;
  kp.geom = pb->geom.kind;
  kp.ga = pb->geom.a;
  kp.coef = pb->coef.kind;
  kp.c0 = pb->coef.c0;
  kp.camp = pb->coef.amp;
  const bool spline = kp.coef == IGS_COEF_SPLINE || kp.coef == IGS_COEF_EXP_SPLINE;
  kp.cdeg = spline ? pb->coef.degree : 0;
  kp.cstride = 1;
  for (int k = 0; k < 3; ++k) {
    kp.cn[k] = (spline && k < kp.n) ? pb->coef.ncoef[k] : 1;
    kp.cstride *= kp.cn[k];
  }
  kp.cc = spline ? pb->coef.coef : nullptr;
  // the error word starts at 0: it is sent with the tables (no memset node)
  const int zero = 0;
  kp.flag = const_cast<int*>(P->ar.put(&zero, 1));
  for (int k = 0; k < kp.n; ++k) {
    kp.t[k].x = upload(P->ar, P->ht.x[k], s, &st);
    kp.t[k].w = upload(P->ar, P->ht.w[k], s, &st);
    kp.t[k].bv = upload(P->ar, P->ht.bv[k], s, &st);
    kp.t[k].bd = upload(P->ar, P->ht.bd[k], s, &st);
    kp.t[k].bpr = upload(P->ar, P->ht.bpr[k], s, &st);
    kp.t[k].trig = upload(P->ar, P->ht.trig[k], s, &st);
    kp.t[k].cb = upload(P->ar, P->ht.cb[k], s, &st);
    kp.t[k].cf = upload(P->ar, P->ht.cf[k], s, &st);
  }
  if (st == IGS_OK) st = P->ar.flush();
  return st;
}

static igs_status finish(const Prepared& P, hipStream_t s) {
  int flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, P.kp.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return (flag & 1) ? IGS_ERR_GEOMETRY : IGS_OK;
}

// used by the adjoint translation unit
igs_status prepare_problem(const igs_problem* pb, hipStream_t s, Dims* d, KProblem* kp, Arena* ar, HostTables* ht) {
  Prepared P;
  igs_status st = prepare(pb, s, &P);
  if (st != IGS_OK) return st;
  *d = P.d;
  *kp = P.kp;
  *ht = P.ht;
  std::swap(ar->base, P.ar.base);
  std::swap(ar->size, P.ar.size);
  std::swap(ar->used, P.ar.used);
  std::swap(ar->stream, P.ar.stream);
  return IGS_OK;
}

igs_status finish_problem(const KProblem& kp, hipStream_t s) {
  int flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, kp.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return (flag & 1) ? IGS_ERR_GEOMETRY : IGS_OK;
}

static int pick_zchunk(const Dims& d, int tx, int ty) {
  const int mz = d.n == 3 ? d.m[2] : d.m[1];
  int64_t base = int64_t((d.m[0] + tx - 1) / tx) * (d.n == 3 ? (d.m[1] + ty - 1) / ty : 1) * d.batch;
  int64_t chunks = std::max<int64_t>(1, (2048 + base - 1) / base);
  int zc = int((mz + chunks - 1) / chunks);
  return std::max(zc, std::min(mz, 4 * (d.p + 1)));
}

template <typename T>
static KInterp<T> interp_view(const HostInterp& hi, const Dims& d, Arena& ar, hipStream_t s, igs_status* st,
                              const std::vector<T> eb[3]) {
  KInterp<T> ip;
  std::memset(&ip, 0, sizeof(ip));
  ip.q = hi.q;
  for (int k = 0; k < 3; ++k) {
    ip.flo[k] = hi.flo[k];
    ip.fhi[k] = hi.fhi[k];
    if (k < d.n) {
      ip.Sd[k] = int(hi.samp[k].size());
      ip.lo[k] = hi.lo[k];
      ip.hi[k] = hi.hi[k];
      ip.samp[k] = upload(ar, hi.samp[k], s, st);
      ip.ginv[k] = upload(ar, hi.ginv[k], s, st);
      ip.ef[k] = upload(ar, hi.ef[k], s, st);
      ip.eb[k] = upload(ar, eb[k], s, st);
    } else {
      ip.Sd[k] = 1;
      ip.lo[k] = 0;
      ip.hi[k] = 0;
    }
    ip.nc[k] = hi.nc[k];
  }
  ip.nup = int(hi.upslot.size());
  ip.upslot = upload(ar, hi.upslot, s, st);
  return ip;
}

static igs_status check_sampling(const Dims& d, int M, int q) {
  if (M < 1) return IGS_ERR_ARG;
  if (q < 1 || q > kMaxQ) return q < 1 ? IGS_ERR_ARG : IGS_ERR_UNSUPPORTED;
  for (int k = 0; k < d.n; ++k) {
    std::vector<int> s;
    igs_status st = sample_lattice(d.m[k], d.p, M, &s);
    if (st != IGS_OK) return st;
    if (int(s.size()) < q + 1) return IGS_ERR_SAMPLES;
  }
  return IGS_OK;
}

// ------------------------------------------------------------------ plans
//
// A plan holds everything an assembly needs besides the band: the device 1-D
// tables, tile and chunk lists, interpolation tables and coefficient scratch.
// The one-shot entry points build a plan, run it, check the geometry flag and
// free it; igs_plan_* keep it for repeated runs.

struct Plan {
  int kind = 0;  // 0 exact, 1 surrogate, 2 face/edge, 3 matrix-free, 4 per-delta domains
  int form = 0, dtype = 0, M = 0, q = 0;
  Prepared P;
  Arena ta;
  const QTile* dt = nullptr;
  int ntiles = 0, groups[3] = {0, 0, 0};
  KInterp<double> ip64{}, ipd{};
  KInterp<float> ipf{};
  const int* dchunks = nullptr;
  int nchunks = 0, chunk_rows = 0, n2max = 1, n3max = 1;
  const int4* ddsl = nullptr;
  double *tmp0 = nullptr, *tmp1 = nullptr, *coef = nullptr;
  const double* g0T = nullptr;  // direction-1 inverse collocation matrix, transposed
  const int* dcopy = nullptr;  // analysis-domain rows whose stencil leaves the domain
  int ncopy = 0;
  const int* dbrow = nullptr;  // matrix-free: rows outside the analysis domain
  int nbrow = 0;
  double* xm = nullptr;        // matrix-free: Dirichlet-masked copy of x
  KInterpPD ippd{};            // per-delta: interpolation tables
  const int* dupslot = nullptr;
  int pdg[3] = {0, 0, 0};      // per-delta sample tiles: [0] tiles, [2] single rows
  int state = 0;  // geometry flag: 0 not read yet, 1 read and clear, 2 set
  Plan() = default;
  Plan(const Plan&) = delete;
  Plan& operator=(const Plan&) = delete;
};

static igs_status build_exact(const igs_problem* pb, hipStream_t s, Plan* pl) {
  igs_status st = prepare(pb, s, &pl->P);
  if (st != IGS_OK) return st;
  int tx, ty;
  quad_tile_shape(pl->P.d.n, pl->P.d.p, &tx, &ty);
  std::vector<QTile> tiles = tiles_all(pl->P.d, tx, ty, pick_zchunk(pl->P.d, tx, ty));
  st = pl->ta.alloc(padded(tiles.size() * sizeof(QTile)), s);
  if (st != IGS_OK) return st;
  pl->dt = upload(pl->ta, tiles, s, &st);
  pl->ntiles = int(tiles.size());
  if (st == IGS_OK) st = pl->ta.flush();
  return st;
}

static igs_status build_surrogate(const igs_problem* pb, hipStream_t s, Plan* pl) {
  igs_status st = prepare(pb, s, &pl->P);
  if (st != IGS_OK) return st;
  const Dims& d = pl->P.d;
  const int form = pl->form, M = pl->M, q = pl->q;
  st = check_sampling(d, M, q);
  if (st != IGS_OK) return st;
  const bool fe = pl->kind == 2;
  HostInterp hi;
  int box[3] = {1, 1, 1};
  st = fe ? build_interp_fe(d, form, M, q, box, &hi) : build_interp(d, form, M, q, box, &hi);
  if (st != IGS_OK) return st;
  std::vector<float> ebf[3];
  for (int k = 0; k < d.n; ++k) ebf[k].assign(hi.eb[k].begin(), hi.eb[k].end());
  int tx, ty;
  quad_tile_shape(d.n, d.p, &tx, &ty);
  int zchunk = pick_zchunk(d, tx, ty);
  if (d.n == 2) {
    // the 2-D boundary columns are 2p rows wide, so a launch holds only two
    // tiles per z-chunk: shorter chunks (about 1024 tiles in all, at least
    // p+1 long) trade p halo element rows per chunk for parallelism
    const int64_t want = (int64_t(2) * (d.m[1] - 4 * d.p) * d.batch + 1023) / 1024;
    zchunk = int(std::min<int64_t>(zchunk, std::max<int64_t>(d.p + 1, want)));
  }
  std::vector<QTile> tiles;
  if (fe) {
    tiles = tiles_fe(d, hi.samp, tx, ty, zchunk, pl->groups);
  } else {
    tiles = tiles_surrogate(d, hi.samp, tx, ty, zchunk, pl->groups);
  }
  size_t per = 1;
  for (int k = 0; k < d.n; ++k) per *= hi.samp[k].size();
  const size_t ncoef = per * hi.upslot.size() * d.batch;
  pl->chunk_rows = fill_chunk_rows(d, int(hi.samp[0].size()), q, int(hi.upslot.size()));
  std::vector<int> chunks = fill_chunks(d, pl->chunk_rows, hi.lo, hi.hi);
  // face/edge: every entry is interpolated or (corners) copied by the identity
  // part of the fit, so no entry is left for the copy kernel
  std::vector<int> crow = fe ? std::vector<int>() : copy_rows(d, 2 * d.p);
  std::vector<int> dsl;  // (slot, delta1, delta2, delta3) per interpolated slot
  for (int sl : hi.upslot) {
    const int W = d.W;
    dsl.push_back(sl);
    dsl.push_back(sl % W - d.p);
    dsl.push_back((sl / W) % W - d.p);
    dsl.push_back(d.n == 3 ? sl / (W * W) - d.p : 0);
  }
  const bool mf = pl->kind == 3;
  std::vector<int> brow = mf ? boundary_rows(d) : std::vector<int>();
  const size_t S1 = hi.samp[0].size();
  // 2-D pencils past the register-held fill's length take the 2-D fill with
  // reloaded weights when its LDS footprint fits, else the chunked fill
  pl->P.d.wide2d = fill2d_wide_fits(d, int(S1), pl->dtype == IGS_F64 ? sizeof(double) : sizeof(float)) ? 1 : 0;
  std::vector<double> g0t(S1 * S1);
  for (size_t r = 0; r < S1; ++r)
    for (size_t c = 0; c < S1; ++c) g0t[c * S1 + r] = hi.ginv[0][r * S1 + c];
  size_t bytes = padded(tiles.size() * sizeof(QTile)) + 3 * padded(ncoef * sizeof(double)) + vbytes(chunks) +
                 vbytes(crow) + vbytes(dsl) + padded(hi.upslot.size() * sizeof(int)) * 2 + vbytes(g0t);
  for (int k = 0; k < d.n; ++k)
    bytes += 2 * (vbytes(hi.samp[k]) + vbytes(hi.ginv[k]) + vbytes(hi.ef[k]) + vbytes(hi.eb[k]));
  if (mf) bytes += vbytes(brow) + padded(sizeof(double) * size_t(d.N) * d.batch);
  st = pl->ta.alloc(bytes, s);
  if (st != IGS_OK) return st;
  Arena& ta = pl->ta;
  pl->dt = upload(ta, tiles, s, &st);
  pl->ntiles = int(tiles.size());
  pl->ip64 = interp_view<double>(hi, d, ta, s, &st, hi.eb);
  if (pl->dtype == IGS_F64)
    pl->ipd = pl->ip64;
  else
    pl->ipf = interp_view<float>(hi, d, ta, s, &st, ebf);
  pl->dchunks = upload(ta, chunks, s, &st);
  pl->nchunks = int(chunks.size());
  pl->dcopy = upload(ta, crow, s, &st);
  pl->ncopy = int(crow.size());
  pl->ddsl = reinterpret_cast<const int4*>(upload(ta, dsl, s, &st));
  pl->g0T = upload(ta, g0t, s, &st);
  if (mf) {
    pl->dbrow = upload(ta, brow, s, &st);
    pl->nbrow = int(brow.size());
    pl->xm = ta.take<double>(size_t(d.N) * d.batch);
  }
  pl->tmp0 = ta.take<double>(ncoef);
  pl->tmp1 = ta.take<double>(ncoef);
  pl->coef = ta.take<double>(ncoef);
  if (st == IGS_OK) st = ta.flush();
  if (st != IGS_OK) return st;
  const size_t lds = pl->dtype == IGS_F64 ? fill_lds_bytes<double>(pl->ipd, fill_npen(d, pl->chunk_rows), d, 0)
                                          : fill_lds_bytes<float>(pl->ipf, fill_npen(d, pl->chunk_rows), d, 0);
  if (!fill_is_2d(d) && lds > 160 * 1024) return IGS_ERR_UNSUPPORTED;
  fill_block_dims(d, hi.ef, q, chunks, pl->chunk_rows, hi.lo, hi.hi, &pl->n2max, &pl->n3max);
  return IGS_OK;
}

// Per-delta domains (Sec. 4 remark): quadrature of the rows of non-cardinal
// functions (tiles over the shell outside [p, m_d - p - 1]) and of the common
// sample rows; one fit and one fill per stencil function on its own domain.
static igs_status build_surrogate_pd(const igs_problem* pb, hipStream_t s, Plan* pl) {
  igs_status st = prepare(pb, s, &pl->P);
  if (st != IGS_OK) return st;
  const Dims& d = pl->P.d;
  const int form = pl->form, M = pl->M, q = pl->q, p = d.p;
  st = check_sampling(d, M, q);
  if (st != IGS_OK) return st;
  HostInterpPD hi;
  st = build_interp_pd(d, form, M, q, &hi);
  if (st != IGS_OK) return st;
  int tx, ty;
  quad_tile_shape(d.n, d.p, &tx, &ty);
  const int zchunk = pick_zchunk(d, tx, ty);
  int sg[2];
  std::vector<QTile> tiles = tiles_shell(d, p, tx, ty, zchunk, sg);
  pl->groups[0] = sg[0];
  pl->groups[1] = sg[1];
  pl->groups[2] = 0;
  int g2[3];
  std::vector<QTile> st_tiles = tiles_fe(d, hi.U, tx, ty, zchunk, g2);
  pl->pdg[0] = g2[0];
  pl->pdg[1] = 0;
  pl->pdg[2] = g2[2];
  tiles.insert(tiles.end(), st_tiles.begin(), st_tiles.end());
  const int sm = hi.smax;
  const size_t per = d.n == 3 ? size_t(sm) * sm * sm : size_t(sm) * sm;
  const size_t ncoef = per * hi.upslot.size() * d.batch;
  std::vector<int> crow = copy_rows(d, p);
  size_t bytes = padded(tiles.size() * sizeof(QTile)) + 3 * padded(ncoef * sizeof(double)) + vbytes(crow) +
                 vbytes(hi.upslot);
  for (int k = 0; k < d.n; ++k)
    bytes += vbytes(hi.U[k]) + vbytes(hi.pos[k]) + vbytes(hi.ginv[k]) + vbytes(hi.ef[k]) + vbytes(hi.eb[k]);
  st = pl->ta.alloc(bytes, s);
  if (st != IGS_OK) return st;
  Arena& ta = pl->ta;
  pl->dt = upload(ta, tiles, s, &st);
  pl->ntiles = int(tiles.size());
  KInterpPD& ip = pl->ippd;
  std::memset(&ip, 0, sizeof(ip));
  ip.q = q;
  ip.p = p;
  ip.W = d.W;
  ip.smax = sm;
  ip.nup = int(hi.upslot.size());
  ip.form = form;
  for (int k = 0; k < 3; ++k) {
    ip.m[k] = k < d.n ? d.m[k] : 1;
    for (int e = 0; e < kMaxW; ++e) {
      ip.S[k][e] = e < d.W ? hi.S[k][e] : 1;
      ip.lo[k][e] = e < d.W ? hi.lo[k][e] : 0;
      ip.hi[k][e] = e < d.W ? hi.hi[k][e] : 0;
    }
    if (k < d.n) {
      ip.nu[k] = int(hi.U[k].size());
      ip.U[k] = upload(ta, hi.U[k], s, &st);
      ip.pos[k] = upload(ta, hi.pos[k], s, &st);
      ip.ginv[k] = upload(ta, hi.ginv[k], s, &st);
      ip.ef[k] = upload(ta, hi.ef[k], s, &st);
      ip.eb[k] = upload(ta, hi.eb[k], s, &st);
    }
  }
  pl->dupslot = upload(ta, hi.upslot, s, &st);
  pl->dcopy = upload(ta, crow, s, &st);
  pl->ncopy = int(crow.size());
  pl->tmp0 = ta.take<double>(ncoef);
  pl->tmp1 = ta.take<double>(ncoef);
  pl->coef = ta.take<double>(ncoef);
  if (st == IGS_OK) st = ta.flush();
  if (st != IGS_OK) return st;
  if (fill_pd_lds_bytes(ip, d.S) > (d.n == 3 ? 160 : 64) * 1024) return IGS_ERR_UNSUPPORTED;
  // the copy / diagonal fix-up kernels only test partners against the box of
  // cardinal rows
  pl->ipd = KInterp<double>{};
  pl->ipf = KInterp<float>{};
  for (int k = 0; k < 3; ++k) {
    pl->ipd.lo[k] = pl->ipf.lo[k] = k < d.n ? p : 0;
    pl->ipd.hi[k] = pl->ipf.hi[k] = k < d.n ? d.m[k] - p - 1 : 0;
  }
  return IGS_OK;
}

template <typename OutT>
static igs_status run_t(const Plan& pl, const KProblem& kp, const KInterp<OutT>& ipT, OutT* band, hipStream_t s) {
  const Dims& d = pl.P.d;
  if (pl.kind == 0) {
    {
      PhaseTimer t("quad_exact", s);
      HIP_TRY(launch_quad<OutT>(kp, pl.form, pl.dt, pl.ntiles, false, band, s));
    }
  } else if (pl.kind == 3) {
    // matrix-free: only what igs_apply_mf reads -- the sample rows, the
    // spline coefficients (kept in the plan) and the rows outside the analysis
    // domain; the band rows of the domain are neither written nor read
    const QTile* t2 = pl.dt + pl.groups[0] + pl.groups[1];
    {
      PhaseTimer t("quad_sample_rows", s);
      HIP_TRY(launch_quad<OutT>(kp, pl.form, t2, pl.groups[2], d.n == 3, band, s));
    }
    {
      PhaseTimer t("fit", s);
      if (fit_use_gemm(pl.ip64, d.n, d.batch))
        HIP_TRY(launch_fit_gemm<OutT>(pl.ip64, d.n, d.m[0], d.m[1], d.ld, d.S, d.batch, band, pl.tmp0, pl.tmp1,
                                      pl.coef, s));
      else
        HIP_TRY(launch_fit<OutT>(pl.ip64, d.n, d.m[0], d.m[1], d.ld, d.S, d.batch, band, pl.tmp0, pl.tmp1, pl.coef,
                                 pl.g0T, s));
    }
    {
      PhaseTimer t("quad_boundary_rows", s);
      HIP_TRY(launch_quad<OutT>(kp, pl.form, pl.dt, pl.groups[0] + pl.groups[1], false, band, s));
    }
    return IGS_OK;
  } else if (pl.kind == 4) {
    // per-delta domains: sample rows, fit, fill of the cardinal rows' entries
    // whose partner is cardinal, then the non-cardinal rows, which (3-D) also
    // store every entry of a cardinal partner there (transposed store), and the
    // copy (2-D) or diagonal fix-up (3-D stiffness) of those entries
    const QTile* ts = pl.dt + pl.groups[0] + pl.groups[1];
    {
      PhaseTimer t("quad_pd_sample_tiles", s);
      HIP_TRY(launch_quad<OutT>(kp, pl.form, ts, pl.pdg[0], false, band, s));
    }
    if (pl.pdg[2] > 0) {
      PhaseTimer t("quad_pd_sample_rows", s);
      HIP_TRY(launch_quad<OutT>(kp, pl.form, ts + pl.pdg[0], pl.pdg[2], true, band, s));
    }
    {
      PhaseTimer t("fit", s);
      HIP_TRY(launch_fit_pd<OutT>(pl.ippd, d.n, d.ld, d.S, d.batch, pl.dupslot, band, pl.tmp0, pl.tmp1, pl.coef, s));
    }
    {
      PhaseTimer t("fill", s);
      HIP_TRY(launch_fill_pd<OutT>(pl.ippd, pl.form, d, pl.coef, band, s));
    }
    {
      KProblem kt = kp;
      if (d.n == 3) {
        kt.transpose = 1;
        for (int k = 0; k < 3; ++k) {
          kt.tr_lo[k] = d.p;
          kt.tr_hi[k] = d.m[k] - d.p - 1;
        }
      }
      PhaseTimer t("quad_boundary_rows", s);
      HIP_TRY(launch_quad<OutT>(kt, pl.form, pl.dt, pl.groups[0] + pl.groups[1], false, band, s));
    }
    if (pl.ncopy > 0 && (d.n == 2 || pl.form == IGS_STIFFNESS)) {
      PhaseTimer t(d.n == 3 ? "diag_fixup" : "copy", s);
      HIP_TRY(launch_copy<OutT>(ipT, pl.form, d, pl.dcopy, pl.ncopy, band, s));
    }
  } else if (pl.kind == 2) {
    // face/edge: the quadrature rows (every sample row of every class, and the
    // corner rows), the fit over the augmented sample sets, and one fill over
    // every row of the band
    {
      PhaseTimer t("quad_fe_tiles", s);
      HIP_TRY(launch_quad<OutT>(kp, pl.form, pl.dt, pl.groups[0], false, band, s));
    }
    if (pl.groups[2] > 0) {
      PhaseTimer t("quad_fe_rows", s);
      HIP_TRY(launch_quad<OutT>(kp, pl.form, pl.dt + pl.groups[0], pl.groups[2], true, band, s));
    }
    {
      PhaseTimer t("fit", s);
      if (fit_use_gemm(pl.ip64, d.n, d.batch))
        HIP_TRY(launch_fit_gemm<OutT>(pl.ip64, d.n, d.m[0], d.m[1], d.ld, d.S, d.batch, band, pl.tmp0, pl.tmp1,
                                      pl.coef, s));
      else
        HIP_TRY(launch_fit<OutT>(pl.ip64, d.n, d.m[0], d.m[1], d.ld, d.S, d.batch, band, pl.tmp0, pl.tmp1, pl.coef,
                                 pl.g0T, s));
    }
    {
      PhaseTimer t("fill", s);
      HIP_TRY(launch_fill<OutT>(ipT, pl.form, d, pl.dchunks, pl.nchunks, pl.chunk_rows, pl.n2max, pl.n3max, pl.ddsl,
                                pl.coef, band, s));
    }
  } else if (d.n == 2 && fill_is_2d(d)) {
    // 2-D, pencils short enough for fill2d, which stores only the
    // analysis-domain rows: the rows outside the domain and the lattice lines
    // in one quadrature launch (their tiles do not overlap), then the fit, the
    // fill, and the copy kernel, which reads the exact entries of the rows
    // outside the domain.  Four launches where the order below takes five;
    // on small meshes each costs latency, not bandwidth.
    {
      PhaseTimer t("quad_rows", s);
      HIP_TRY(launch_quad<OutT>(kp, pl.form, pl.dt, pl.groups[0] + pl.groups[1] + pl.groups[2], false, band, s));
    }
    {
      PhaseTimer t("fit", s);
      if (fit_use_gemm(pl.ip64, d.n, d.batch))
        HIP_TRY(launch_fit_gemm<OutT>(pl.ip64, d.n, d.m[0], d.m[1], d.ld, d.S, d.batch, band, pl.tmp0, pl.tmp1,
                                      pl.coef, s));
      else
        HIP_TRY(launch_fit<OutT>(pl.ip64, d.n, d.m[0], d.m[1], d.ld, d.S, d.batch, band, pl.tmp0, pl.tmp1, pl.coef,
                                 pl.g0T, s));
    }
    {
      PhaseTimer t("fill", s);
      HIP_TRY(launch_fill<OutT>(ipT, pl.form, d, pl.dchunks, pl.nchunks, pl.chunk_rows, pl.n2max, pl.n3max, pl.ddsl,
                                pl.coef, band, s));
    }
    if (pl.ncopy > 0) {
      PhaseTimer t("copy", s);
      HIP_TRY(launch_copy<OutT>(ipT, pl.form, d, pl.dcopy, pl.ncopy, band, s));
    }
  } else {
    // Order: sample rows, fit and fill first; the fill writes whole lines of
    // the analysis-domain pencils, placeholders included, and reads nothing of
    // the band.  Then the quadrature of every row outside the analysis domain
    // (overwriting the placeholders) and the copy kernel, which reads the
    // exact entries of those rows.
    const QTile* t2 = pl.dt + pl.groups[0] + pl.groups[1];
    {
      // the sample rows: isolated, one workgroup each in 3-D (single-row
      // tiles); whole lattice lines in 2-D
      PhaseTimer t("quad_sample_rows", s);
      HIP_TRY(launch_quad<OutT>(kp, pl.form, t2, pl.groups[2], d.n == 3, band, s));
    }
    {
      PhaseTimer t("fit", s);
      if (fit_use_gemm(pl.ip64, d.n, d.batch))
        HIP_TRY(launch_fit_gemm<OutT>(pl.ip64, d.n, d.m[0], d.m[1], d.ld, d.S, d.batch, band, pl.tmp0, pl.tmp1,
                                      pl.coef, s));
      else
        HIP_TRY(launch_fit<OutT>(pl.ip64, d.n, d.m[0], d.m[1], d.ld, d.S, d.batch, band, pl.tmp0, pl.tmp1, pl.coef,
                                 pl.g0T, s));
    }
    {
      PhaseTimer t("fill", s);
      HIP_TRY(launch_fill<OutT>(ipT, pl.form, d, pl.dchunks, pl.nchunks, pl.chunk_rows, pl.n2max, pl.n3max, pl.ddsl,
                                pl.coef, band, s));
    }
    {
      // 3-D: the boundary rows also store each entry whose partner is an
      // analysis-domain row into that row (its copied exact entry)
      KProblem kt = kp;
      if (d.n == 3) {
        kt.transpose = 1;
        for (int k = 0; k < 3; ++k) {
          kt.tr_lo[k] = 2 * d.p;
          kt.tr_hi[k] = d.m[k] - 2 * d.p - 1;
        }
      }
      PhaseTimer t("quad_boundary_rows", s);
      HIP_TRY(launch_quad<OutT>(kt, pl.form, pl.dt, pl.groups[0] + pl.groups[1], false, band, s));
    }
    if (pl.ncopy > 0 && (d.n == 2 || pl.form == IGS_STIFFNESS)) {
      // 2-D: copies of the exact partner entries; 3-D stiffness: their sum
      // leaves the diagonal of the rows next to the domain's edge
      PhaseTimer t(d.n == 3 ? "diag_fixup" : "copy", s);
      HIP_TRY(launch_copy<OutT>(ipT, pl.form, d, pl.dcopy, pl.ncopy, band, s));
    }
  }
  // the 2-D fill zeroes the padding columns itself
  const bool fill_pads = fill_is_2d(d) && (pl.kind == 1 || pl.kind == 2);
  if (!fill_pads) {
    PhaseTimer t("zero_pad", s);
    HIP_TRY(launch_zero_pad<OutT>(band, d.N, d.ld, d.S * d.batch, s));
  }
  return IGS_OK;
}

// Queue the plan's kernels; coef (device, optional) replaces the spline
// control values of the problem it was built for.
static igs_status run_plan(const Plan& pl, const double* coef, void* band, hipStream_t s) {
  KProblem kp = pl.P.kp;
  if (coef && kp.cc) kp.cc = coef;
  if (pl.dtype == IGS_F64) return run_t<double>(pl, kp, pl.ipd, static_cast<double*>(band), s);
  return run_t<float>(pl, kp, pl.ipf, static_cast<float*>(band), s);
}

// Reads the geometry flag the first time (synchronising s), or every time if
// always is set.
static igs_status check_plan(Plan* pl, hipStream_t s, bool always) {
  if (pl->state == 2) return IGS_ERR_GEOMETRY;
  if (pl->state == 1 && !always) return IGS_OK;
  const igs_status st = finish(pl->P, s);
  if (st == IGS_OK) pl->state = 1;
  if (st == IGS_ERR_GEOMETRY) pl->state = 2;
  return st;
}

// ---------------------------------------------------- asynchronous calls
//
// A status word per (device, stream), made on the first asynchronous call on
// that stream: each such call queues fold_status_kernel after its kernels,
// which sets the word when the call's own geometry flag is set; igs_check
// reads and clears it.  Words live until the process ends.
__global__ void fold_status_kernel(const int* flag, int* word) {
  if (threadIdx.x == 0 && (*flag & 1)) *word = 1;
}

static std::mutex g_status_mu;
static std::vector<std::pair<std::pair<int, hipStream_t>, int*>> g_status;

// The word of (current device, s); made when create is set (zeroed by a copy
// ordered on s, ahead of the kernel that may set it), else null if no
// asynchronous call has used the stream yet.
static igs_status status_word(hipStream_t s, bool create, int** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_status_mu);
  for (auto& e : g_status)
    if (e.first.first == dev && e.first.second == s) {
      *out = e.second;
      return IGS_OK;
    }
  *out = nullptr;
  if (!create) return IGS_OK;
  void* w = nullptr;
  HIP_TRY(hipMalloc(&w, 256));
  static const int kZero = 0;  // static storage: valid whenever the copy reads it
  hipError_t e = hipMemcpyAsync(w, &kZero, sizeof(int), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    (void)hipFree(w);
    return IGS_ERR_HIP;
  }
  g_status.push_back({{dev, s}, static_cast<int*>(w)});
  *out = static_cast<int*>(w);
  return IGS_OK;
}

static igs_status fold_status(const int* flag, hipStream_t s) {
  int* w = nullptr;
  igs_status st = status_word(s, true, &w);
  if (st != IGS_OK) return st;
  hipLaunchKernelGGL(fold_status_kernel, dim3(1), dim3(64), 0, s, flag, w);
  HIP_TRY(hipGetLastError());
  return IGS_OK;
}

// async: queue the work and fold the geometry flag into the stream's status
// word instead of reading it; the plan's device memory is released in stream
// order (hipFreeAsync on s), its host staging was consumed by the time the
// upload call returned (pageable-memory copies are staged before return).
static igs_status one_shot(const igs_problem* pb, int kind, int form, int M, int q, int dtype, void* band,
                           hipStream_t s, ScratchPool* pool = nullptr, bool async = false) {
  Plan pl;
  pl.P.ar.pool = pool;
  pl.ta.pool = pool;
  pl.kind = kind;
  pl.form = form;
  pl.dtype = dtype;
  pl.M = M;
  pl.q = q;
  igs_status st = kind == 0 ? build_exact(pb, s, &pl)
                  : kind == 4 ? build_surrogate_pd(pb, s, &pl)
                              : build_surrogate(pb, s, &pl);
  if (st != IGS_OK) return st;
  st = run_plan(pl, nullptr, band, s);
  if (st != IGS_OK) return st;
  if (async) return fold_status(pl.P.kp.flag, s);
  return check_plan(&pl, s, true);
}

// ------------------------------------------------------ allocation-free path
//
// The scratch of igs_assemble_noalloc: one array per GPU for the life of the
// process.  Its name is a host-side stand-in, not a device address: host code
// uses only the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) char scratch[IGS_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::vector<char*> g_scratch_ptr;  // per device ordinal; null until looked up

static igs_status scratch_address(char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0) return IGS_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (size_t(dev) >= g_scratch_ptr.size()) g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return IGS_ERR_HIP;
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return IGS_OK;
}

}  // namespace igs

using namespace igs;

extern "C" {

igs_status igs_band_layout(const igs_problem* pb, igs_layout* out) {
  if (!out) return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  for (int k = 0; k < 3; ++k) out->m[k] = d.m[k];
  out->slots = d.S;
  out->upper = (d.S - 1) / 2;
  out->N = d.N;
  out->ld = d.ld;
  out->band_elems = int64_t(d.batch) * d.S * d.ld;
  return IGS_OK;
}

igs_status igs_validate(const igs_problem* pb, int32_t M, int32_t q) {
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  if (M >= 1 || q != 0) return check_sampling(d, M, q);
  return IGS_OK;
}

igs_status igs_surrogate_layout(const igs_problem* pb, int32_t M, int32_t q, igs_surrogate_info* out, int32_t* indices,
                                int32_t capacity) {
  if (!out) return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  st = check_sampling(d, M, q);
  if (st != IGS_OK) return st;
  std::memset(out, 0, sizeof(*out));
  int64_t interior = 1;
  int64_t samples = 1;
  int pos = 0;
  for (int k = 0; k < 3; ++k) {
    if (k >= d.n) {
      out->samples[k] = 1;
      out->interior[k] = 1;
      continue;
    }
    std::vector<int> s;
    sample_lattice(d.m[k], d.p, M, &s);
    out->samples[k] = int(s.size());
    out->interior[k] = d.m[k] - 4 * d.p;
    interior *= out->interior[k];
    samples *= int64_t(s.size());
    if (indices) {
      if (pos + int(s.size()) > capacity) return IGS_ERR_ARG;
      for (int v : s) indices[pos++] = v;
    }
  }
  out->sample_rows = samples;
  out->boundary_rows = d.N - interior;
  out->quadrature_rows = out->boundary_rows + samples;
  return IGS_OK;
}

int32_t igs_sampling_length(int32_t nelem, int32_t p, int32_t q, double c, double beta) {
  if (nelem < 1 || p < 1 || q < 1 || !std::isfinite(c) || !std::isfinite(beta) || c < 0.0 || beta < 0.0)
    return IGS_ERR_ARG;
  // h^((p - q + beta) / (q + 1)) with h = 1/nelem, written as a power of nelem.
  const double v = c * std::pow(double(nelem), (double(q) - double(p) - beta) / double(q + 1));
  // A value that is an integer in exact arithmetic may come out a few ulps
  // below it; the relative nudge keeps floor() on that integer.
  const double f = std::floor(v * (1.0 + 1e-12));
  if (!(f >= 1.0)) return 1;
  return f >= double(1 << 30) ? int32_t(1 << 30) : int32_t(f);
}

const char* igs_status_string(int32_t status) {
  switch (status) {
    case IGS_OK: return "ok";
    case IGS_ERR_ARG: return "invalid argument";
    case IGS_ERR_UNSUPPORTED: return "unsupported by the library";
    case IGS_ERR_KNOTS: return "knot vector is not open uniform";
    case IGS_ERR_SAMPLES: return "too few samples for the interpolation degree";
    case IGS_ERR_GEOMETRY: return "geometry map folds (det J <= 0 at a quadrature point)";
    case IGS_ERR_HIP: return "HIP runtime error";
    case IGS_ERR_NOMEM: return "out of device memory";
    case IGS_ERR_SCRATCH: return "problem needs more scratch than the allocation-free entry point holds";
    case IGS_NOT_CONVERGED: return "not converged within maxit";
    case IGS_BREAKDOWN: return "CG breakdown";
    default: return "unknown status";
  }
}

const char* igs_version(void) { return "igs 0.1.0 (gfx950)"; }

igs_status igs_assemble_exact(const igs_problem* pb, int32_t form, int32_t dtype, void* band, void* stream) {
  if (!pb || !band) return IGS_ERR_ARG;
  if (form != IGS_STIFFNESS && form != IGS_MASS) return IGS_ERR_ARG;
  if (dtype != IGS_F64 && dtype != IGS_F32) return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  return one_shot(pb, 0, form, 0, 0, dtype, band, static_cast<hipStream_t>(stream));
}

igs_status igs_assemble_surrogate(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype, void* band,
                                  void* stream) {
  if (!pb || !band) return IGS_ERR_ARG;
  if (form != IGS_STIFFNESS && form != IGS_MASS) return IGS_ERR_ARG;
  if (dtype != IGS_F64 && dtype != IGS_F32) return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  st = check_sampling(d, M, q);
  if (st != IGS_OK) return st;
  return one_shot(pb, 1, form, M, q, dtype, band, static_cast<hipStream_t>(stream));
}

igs_status igs_assemble_noalloc(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype, void* band,
                                void* stream) {
  if (!pb || !band) return IGS_ERR_ARG;
  if (form != IGS_STIFFNESS && form != IGS_MASS) return IGS_ERR_ARG;
  if (dtype != IGS_F64 && dtype != IGS_F32) return IGS_ERR_ARG;
  if (M < 0) return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  if (M >= 1) {
    st = check_sampling(d, M, q);
    if (st != IGS_OK) return st;
  }
  ScratchPool pool;
  st = scratch_address(&pool.base);
  if (st != IGS_OK) return st;
  pool.cap = IGS_NOALLOC_SCRATCH_BYTES;
  return one_shot(pb, M == 0 ? 0 : 1, form, M, q, dtype, band, static_cast<hipStream_t>(stream), &pool);
}

igs_status igs_assemble_surrogate_fe(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype,
                                     void* band, void* stream) {
  if (!pb || !band) return IGS_ERR_ARG;
  if (form != IGS_STIFFNESS && form != IGS_MASS) return IGS_ERR_ARG;
  if (dtype != IGS_F64 && dtype != IGS_F32) return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  st = check_sampling(d, M, q);
  if (st != IGS_OK) return st;
  return one_shot(pb, 2, form, M, q, dtype, band, static_cast<hipStream_t>(stream));
}

igs_status igs_surrogate_fe_layout(const igs_problem* pb, int32_t M, int32_t q, igs_fe_info* out) {
  if (!out) return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  st = check_sampling(d, M, q);
  if (st != IGS_OK) return st;
  std::memset(out, 0, sizeof(*out));
  int64_t all = 1, layers = 1, free_or_layer = 1;
  for (int k = 0; k < 3; ++k) {
    if (k >= d.n) {
      out->samples[k] = 1;
      continue;
    }
    std::vector<int> s;
    sample_lattice(d.m[k], d.p, M, &s);
    out->samples[k] = int(s.size()) + 4 * d.p;
    all *= out->samples[k];
    layers *= 4 * d.p;
    free_or_layer *= 4 * d.p + 1;
  }
  out->classes = free_or_layer - layers;
  out->corner_rows = layers;
  out->quadrature_rows = all;
  return IGS_OK;
}

igs_status igs_assemble_surrogate_pd(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype,
                                     void* band, void* stream) {
  if (!pb || !band) return IGS_ERR_ARG;
  if (form != IGS_STIFFNESS && form != IGS_MASS) return IGS_ERR_ARG;
  if (dtype != IGS_F64 && dtype != IGS_F32) return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  st = check_sampling(d, M, q);
  if (st != IGS_OK) return st;
  return one_shot(pb, 4, form, M, q, dtype, band, static_cast<hipStream_t>(stream));
}

igs_status igs_surrogate_pd_layout(const igs_problem* pb, int32_t M, int32_t q, igs_pd_info* out) {
  if (!out) return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  st = check_sampling(d, M, q);
  if (st != IGS_OK) return st;
  HostInterpPD hi;
  st = build_interp_pd(d, IGS_STIFFNESS, M, q, &hi);
  if (st != IGS_OK) return st;
  std::memset(out, 0, sizeof(*out));
  int64_t card = 1, samp = 1;
  for (int k = 0; k < 3; ++k) {
    out->samples[k] = k < d.n ? int32_t(hi.U[k].size()) : 1;
    out->max_samples[k] = 1;
    for (int e = 0; k < d.n && e < d.W; ++e) out->max_samples[k] = std::max(out->max_samples[k], hi.S[k][e]);
    if (k < d.n) card *= d.m[k] - 2 * d.p;
    samp *= out->samples[k];
  }
  out->noncardinal_rows = d.N - card;
  out->quadrature_rows = out->noncardinal_rows + samp;
  return IGS_OK;
}

struct igs_plan_s {
  igs::Plan pl;
  hipStream_t last = nullptr;
};

static igs_status plan_create(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype, void* stream,
                              igs_plan* out, int variant) {
  if (!pb || !out) return IGS_ERR_ARG;
  *out = nullptr;
  if (variant != 0 && M < 1) return IGS_ERR_ARG;
  if (variant == 3 && pb->n != 3) return IGS_ERR_UNSUPPORTED;
  *out = nullptr;
  if (form != IGS_STIFFNESS && form != IGS_MASS) return IGS_ERR_ARG;
  if (dtype != IGS_F64 && dtype != IGS_F32) return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  if (M != 0) {
    st = check_sampling(d, M, q);
    if (st != IGS_OK) return st;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  igs_plan_s* h = new igs_plan_s;
  h->pl.P.ar.persistent = true;
  h->pl.ta.persistent = true;
  h->pl.kind = M == 0 ? 0 : (variant != 0 ? variant : 1);
  h->pl.form = form;
  h->pl.dtype = dtype;
  h->pl.M = M;
  h->pl.q = q;
  st = h->pl.kind == 0   ? build_exact(pb, s, &h->pl)
       : h->pl.kind == 4 ? build_surrogate_pd(pb, s, &h->pl)
                         : build_surrogate(pb, s, &h->pl);
  // the plan's memory and tables are complete before any other stream uses them
  if (st == IGS_OK && hipStreamSynchronize(s) != hipSuccess) st = IGS_ERR_HIP;
  if (st != IGS_OK) {
    delete h;
    return st;
  }
  h->last = s;
  *out = h;
  return IGS_OK;
}

igs_status igs_plan_create(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype, void* stream,
                           igs_plan* out) {
  return plan_create(pb, form, M, q, dtype, stream, out, 0);
}

igs_status igs_plan_create_fe(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype, void* stream,
                              igs_plan* out) {
  return plan_create(pb, form, M, q, dtype, stream, out, 2);
}

igs_status igs_plan_create_pd(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype, void* stream,
                              igs_plan* out) {
  return plan_create(pb, form, M, q, dtype, stream, out, 4);
}

igs_status igs_plan_create_mf(const igs_problem* pb, int32_t form, int32_t M, int32_t q, void* stream, igs_plan* out) {
  return plan_create(pb, form, M, q, IGS_F64, stream, out, 3);
}

static igs_status mf_apply(const Plan& pl, const double* band, const double* x, double* y, int dirichlet,
                           bool x_masked, hipStream_t s) {
  const Dims& d = pl.P.d;
  const hipError_t e = launch_apply_mf<double>(pl.ipd, pl.form, d, pl.dchunks, pl.nchunks, pl.chunk_rows, pl.n2max,
                                               pl.n3max, pl.ddsl, pl.coef, band, pl.dcopy, pl.ncopy, pl.dbrow,
                                               pl.nbrow, x, y, pl.xm, dirichlet, x_masked, s);
  if (e == hipErrorInvalidValue) return IGS_ERR_UNSUPPORTED;
  return e == hipSuccess ? IGS_OK : IGS_ERR_HIP;
}

igs_status igs_apply_mf(igs_plan plan, const double* band, const double* x, double* y, int32_t dirichlet,
                        void* stream) {
  if (!plan || !band || !x || !y) return IGS_ERR_ARG;
  if (plan->pl.kind != 3) return IGS_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  plan->last = s;
  return mf_apply(plan->pl, band, x, y, dirichlet, false, s);
}

igs_status igs_solve_cg_mf(igs_plan plan, const double* band, const double* f, double* u, double rtol, int32_t maxit,
                           igs_cg_info* info, void* stream) {
  if (!plan || !band || !f || !u || !info) return IGS_ERR_ARG;
  if (plan->pl.kind != 3 || !(rtol > 0.0) || maxit < 1) return IGS_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  plan->last = s;
  std::memset(info, 0, sizeof(*info));
  const Plan& pl = plan->pl;
  // CG keeps its vectors zero on the Dirichlet dofs: no masking copy
  auto A = [&](const double* x, double* y) { return mf_apply(pl, band, x, y, 1, true, s); };
  return solve_cg_op(pl.P.d, A, f, u, rtol, maxit, info, s);
}

igs_status igs_plan_execute(igs_plan plan, const double* coef, void* band, void* stream) {
  if (!plan || !band) return IGS_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  plan->last = s;
  igs_status st = run_plan(plan->pl, coef, band, s);
  if (st != IGS_OK) return st;
  return check_plan(&plan->pl, s, false);
}

igs_status igs_plan_destroy(igs_plan plan) {
  if (!plan) return IGS_OK;
  const bool ok = hipStreamSynchronize(plan->last) == hipSuccess;
  delete plan;
  return ok ? IGS_OK : IGS_ERR_HIP;
}

static igs_status assemble_rhs(const igs_problem* pb, int32_t source, double c, double* f, void* stream,
                               bool async) {
  if (!pb || !f) return IGS_ERR_ARG;
  if (source != 0 && source != 1) return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Prepared P;
  st = prepare(pb, s, &P);
  if (st != IGS_OK) return st;
  int tx, ty;
  rhs_tile_shape(P.d.n, &tx, &ty);
  std::vector<QTile> tiles = tiles_all(P.d, tx, ty, pick_zchunk(P.d, tx, ty));
  Arena ta;
  st = ta.alloc(padded(tiles.size() * sizeof(QTile)), s);
  if (st != IGS_OK) return st;
  const QTile* dt = upload(ta, tiles, s, &st);
  if (st == IGS_OK) st = ta.flush();
  if (st != IGS_OK) return st;
  {
    PhaseTimer t("rhs", s);
    HIP_TRY(launch_rhs(P.kp, dt, int(tiles.size()), source, c, f, s));
  }
  if (async) return fold_status(P.kp.flag, s);
  return finish(P, s);
}

igs_status igs_assemble_rhs(const igs_problem* pb, int32_t source, double c, double* f, void* stream) {
  return assemble_rhs(pb, source, c, f, stream, false);
}

igs_status igs_assemble_rhs_async(const igs_problem* pb, int32_t source, double c, double* f, void* stream) {
  return assemble_rhs(pb, source, c, f, stream, true);
}

igs_status igs_assemble_async(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype, void* band,
                              void* stream) {
  if (!pb || !band) return IGS_ERR_ARG;
  if (form != IGS_STIFFNESS && form != IGS_MASS) return IGS_ERR_ARG;
  if (dtype != IGS_F64 && dtype != IGS_F32) return IGS_ERR_ARG;
  if (M < 0) return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  if (M >= 1) {
    st = check_sampling(d, M, q);
    if (st != IGS_OK) return st;
  }
  return one_shot(pb, M == 0 ? 0 : 1, form, M, q, dtype, band, static_cast<hipStream_t>(stream), nullptr, true);
}

igs_status igs_check(void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  int* w = nullptr;
  igs_status st = status_word(s, false, &w);
  if (st != IGS_OK) return st;
  HIP_TRY(hipStreamSynchronize(s));
  if (!w) return IGS_OK;
  int v = 0;
  HIP_TRY(hipMemcpyAsync(&v, w, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (!v) return IGS_OK;
  const int zero = 0;
  HIP_TRY(hipMemcpyAsync(w, &zero, sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return IGS_ERR_GEOMETRY;
}

igs_status igs_apply(const igs_problem* pb, int32_t dtype, const void* band, const void* x, void* y, int32_t dirichlet,
                     void* stream) {
  if (!pb || !band || !x || !y) return IGS_ERR_ARG;
  if (dtype != IGS_F64 && dtype != IGS_F32) return IGS_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(band) % (dtype == IGS_F64 ? 16 : 8) != 0) return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  return launch_apply(d, dtype, band, x, y, dirichlet, static_cast<hipStream_t>(stream));
}

igs_status igs_solve_cg(const igs_problem* pb, const double* band64, const float* band32, const double* f, double* u,
                        double rtol, int32_t maxit, igs_cg_info* info, void* stream) {
  if (!pb || !band64 || !f || !u || !info) return IGS_ERR_ARG;
  if (!(rtol > 0.0) || maxit < 1) return IGS_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(band64) % 16 != 0 || reinterpret_cast<uintptr_t>(band32) % 8 != 0)
    return IGS_ERR_ARG;
  Dims d;
  igs_status st = make_dims(pb, &d);
  if (st != IGS_OK) return st;
  std::memset(info, 0, sizeof(*info));
  return solve_cg(d, band64, band32, f, u, rtol, maxit, info, static_cast<hipStream_t>(stream));
}

}  // extern "C"
