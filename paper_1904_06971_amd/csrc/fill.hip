// Surrogate interpolation: fit, fill and copy kernels (Secs. 4.1, 5, 6).
//
// fit:  for every interpolated ("upper") stencil delta, the sample values
//       V_delta[k] = A_{s(k), s(k)+delta} (read from the band rows that the
//       quadrature kernel wrote) become tensor spline coefficients
//       c_delta = (G_n^-1 x ... x G_1^-1) V_delta, one direction per pass.
// fill: every analysis-domain row gets, for each upper delta, Phi~_delta at
//       its own index (upper entry) and at the index of its lower partner
//       (lower entry, eq. 5.1b/5.1c copy rule).  A workgroup evaluates the
//       interpolant separably on its chunk of rows through two LDS stages and
//       writes every slot of every row of the analysis-domain pencils (rows
//       with (i2, i3) inside the analysis domain), whole 128-byte lines, with
//       no reads of the band.  Slots it cannot know yet hold placeholders:
//       the rows of those pencils outside the domain in i1 (their quadrature
//       runs afterwards and overwrites them) and the entries whose partner
//       leaves the domain.  The stiffness diagonal holds minus the sum of the
//       interpolated entries.
// copy: afterwards, the domain rows whose stencil leaves the domain take the
//       exact entries of their partners (A_ij = A_ji, row j from quadrature)
//       and subtract them from the diagonal, which then closes the row sum
//       over every off-diagonal entry (eq. 5.1c).
#include <algorithm>

#include "igs_internal.h"
#include "profile.h"

namespace igs {

// ------------------------------------------------------------------ fit ----

// out[b][u][..k_d..] = sum_j ginv_d[k_d][j] in[b][u][..j..]; pass 0 gathers
// `in` from the band at the sample rows.  gT (optional) is ginv_d transposed:
// in direction 1 consecutive threads have consecutive k_d, so reading
// gT[j][k_d] is one coalesced load per j where ginv_d[k_d][j] would touch a
// separate cache line per lane.
template <typename BT, bool GATHER>
__global__ void fit_pass_kernel(KInterp<double> ip, int d, int n, int m1, int m2, int64_t ld, int S, int batch,
                                const BT* __restrict__ band, const double* __restrict__ in, double* __restrict__ out,
                                const double* __restrict__ gT) {
  const int S1 = ip.Sd[0], S2 = ip.Sd[1], S3 = (n == 3) ? ip.Sd[2] : 1;
  const int64_t per = int64_t(S1) * S2 * S3;
  const int64_t total = per * ip.nup * batch;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    int64_t r = t;
    const int k1 = r % S1; r /= S1;
    const int k2 = r % S2; r /= S2;
    const int k3 = r % S3; r /= S3;
    const int u = r % ip.nup;
    const int b = r / ip.nup;
    const int kd = (d == 0) ? k1 : (d == 1 ? k2 : k3);
    const int Sd = ip.Sd[d];
    const double* g = gT ? gT + kd : ip.ginv[d] + size_t(kd) * Sd;
    const size_t gs = gT ? size_t(Sd) : 1;
    // the spline block [flo, fhi) of the matrix; outside it the matrix is
    // the identity (face/edge layers) and the value is copied
    const int flo = ip.flo[d], fhi = ip.fhi[d];
    const bool copy = kd < flo || kd >= fhi;
    const int ja = copy ? kd : flo, jb = copy ? kd + 1 : fhi;
    // four independent partial sums over j = ja + 4l + e keep several loads in
    // flight per thread (a single chain waits on each load in turn)
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    const int J4 = copy ? ja : ja + ((jb - ja) & ~3);
    if constexpr (GATHER) {
      const BT* bs = band + (size_t(b) * S + ip.upslot[u]) * ld;
      const size_t rowbase = size_t(m1) * (ip.samp[1][k2] + size_t(m2) * (n == 3 ? ip.samp[2][k3] : 0));
      const int* s1 = ip.samp[0];
      if (copy) {
        out[t] = double(bs[rowbase + s1[kd]]);
        continue;
      }
      for (int j = ja; j < J4; j += 4) {
        a0 += g[j * gs] * double(bs[rowbase + s1[j]]);
        a1 += g[(j + 1) * gs] * double(bs[rowbase + s1[j + 1]]);
        a2 += g[(j + 2) * gs] * double(bs[rowbase + s1[j + 2]]);
        a3 += g[(j + 3) * gs] * double(bs[rowbase + s1[j + 3]]);
      }
      for (int j = J4; j < jb; ++j) a0 += g[j * gs] * double(bs[rowbase + s1[j]]);
    } else {
      const double* src = in + (size_t(b) * ip.nup + u) * per;
      const size_t stride = d == 0 ? 1 : (d == 1 ? size_t(S1) : size_t(S1) * S2);
      const double* sp = src + (size_t(d == 2 ? 0 : k3) * S2 + (d == 1 ? 0 : k2)) * S1 + (d == 0 ? 0 : k1);
      if (copy) {
        out[t] = sp[kd * stride];
        continue;
      }
      for (int j = ja; j < J4; j += 4) {
        a0 += g[j * gs] * sp[j * stride];
        a1 += g[(j + 1) * gs] * sp[(j + 1) * stride];
        a2 += g[(j + 2) * gs] * sp[(j + 2) * stride];
        a3 += g[(j + 3) * gs] * sp[(j + 3) * stride];
      }
      for (int j = J4; j < jb; ++j) a0 += g[j * gs] * sp[j * stride];
    }
    out[t] = (a0 + a1) + (a2 + a3);
  }
}

// ----------------------------------------------------------------- fill ----
//
// A workgroup owns an aligned chunk of kChunk consecutive rows of the flat
// (colex) index, one row per thread, and writes every slot of every row of the
// chunk that lies in an analysis-domain pencil, so each store instruction of
// a wave covers whole 128-byte lines (the HBM write path streams those at full
// rate).  Per interpolated delta the chunk's pencils (rows with the same
// (i2, i3)) get the partial contraction T[c1] = sum_{c2,c3} beta2 beta3
// c_delta[c3][c2][c1] in LDS (for the pencil itself and for the pencil of the
// lower partners); each row then finishes with its q+1 direction-1 weights.
// LDS is double-buffered so one barrier per delta suffices.

bool fill_is_2d(const Dims& d);
template <typename T>
hipError_t launch_fill2d(const KInterp<T>& ip, int form, const Dims& d, const int4* dsl, const double* coef, T* band,
                         hipStream_t s);

constexpr int kChunk = 256;

struct FillGeom {
  int n, P, m1, m2, m3;
  int64_t N, ld;
  int S;
  int npen;           // max pencils a chunk can touch
  int nchunks;
  const int* chunks;  // chunk ids that contain analysis-domain rows
  int n2max, n3max;   // largest coefficient block (directions 2, 3) a chunk's tasks use
  // matrix-free apply (fill_fast_kernel with APPLY): y_i for the evaluated
  // rows from their interpolated entries and x, instead of band stores
  const void* ax;
  void* ay;
};

// host-side per-delta table (slot, delta1, delta2, delta3)
struct DeltaRec {
  int s, d1, d2, d3;
};

template <typename T>
__device__ __forceinline__ bool in_dom(const KInterp<T>& ip, int d, int i) {
  return i >= ip.lo[d] && i <= ip.hi[d];
}

// MULTI = false: every pencil task fits one thread (npen*2*S1 <= kChunk) and
// its operands for the next delta are prefetched into registers; MULTI = true
// (tiny sampling steps, many coefficients per line) loops over the tasks.
template <int ND, int FORM, int Q, typename T, bool MULTI>
__global__ void __launch_bounds__(kChunk)
    fill_kernel(KInterp<T> ip, FillGeom g, const double* __restrict__ coef, T* __restrict__ band) {
  extern __shared__ char smem_raw[];
  constexpr int NC = (ND == 3) ? (Q + 1) * (Q + 1) : (Q + 1);  // coefficients per pencil task
  const int W = 2 * g.P + 1;
  const int S1 = ip.Sd[0], S2 = ip.Sd[1], S3 = (ND == 3) ? ip.Sd[2] : 1;
  const int m3 = (ND == 3) ? g.m3 : 1;
  // LDS layout (see fill_lds_bytes): T [2][npen][2][S1]; spline weights
  // b1[m1], b2[m2], b3[m3] (Q+1 each); first functions f1, f2, f3; per-delta
  // (slot, delta1, delta2, delta3)
  T* Tbuf = reinterpret_cast<T*>(smem_raw);
  T* tb1 = Tbuf + size_t(2) * g.npen * 2 * S1;
  T* tb2 = tb1 + size_t(g.m1) * (Q + 1);
  T* tb3 = tb2 + size_t(g.m2) * (Q + 1);
  int* tf1 = reinterpret_cast<int*>(tb3 + size_t(m3) * (Q + 1));
  int* tf2 = tf1 + g.m1;
  int* tf3 = tf2 + g.m2;
  int4* dsl = reinterpret_cast<int4*>(tf3 + m3 + ((4 - ((g.m1 + g.m2 + m3) & 3)) & 3));
  const int b = blockIdx.y;
  const int64_t c0 = int64_t(g.chunks[blockIdx.x]) * kChunk;
  const int tid = threadIdx.x;
  for (int d = 0; d < ND; ++d) {
    const int md = d == 0 ? g.m1 : (d == 1 ? g.m2 : m3);
    T* tb = d == 0 ? tb1 : (d == 1 ? tb2 : tb3);
    int* tf = d == 0 ? tf1 : (d == 1 ? tf2 : tf3);
    for (int t = tid; t < md * (Q + 1); t += kChunk) {
      const int ii = t / (Q + 1);
      const bool ok = in_dom(ip, d, ii);
      tb[t] = ok ? ip.eb[d][t] : T(0);
      if (t % (Q + 1) == 0) tf[ii] = ok ? ip.ef[d][ii] : 0;
    }
  }
  for (int u = tid; u < ip.nup; u += kChunk) {
    const int s = ip.upslot[u];
    dsl[u] = make_int4(s, s % W - g.P, (s / W) % W - g.P, (ND == 3) ? s / (W * W) - g.P : 0);
  }
  const int64_t i = c0 + tid;
  const int64_t pen0 = c0 / g.m1;
  int i1 = 0, i2 = 0, i3 = 0;
  int64_t pen = pen0;
  if (i < g.N) {
    pen = i / g.m1;
    i1 = int(i - pen * g.m1);
    i2 = int(pen % g.m2);
    i3 = int(pen / g.m2);
  }
  const int k = int(pen - pen0);  // this row's pencil slot in the chunk
  // rows of pencils outside the analysis domain in (i2, i3) are left to the
  // quadrature (their lines are not shared with domain rows except at the two
  // ends of a run of domain pencils)
  const bool live = i < g.N && in_dom(ip, 1, i2) && (ND == 2 || in_dom(ip, 2, i3));
  const bool inner = live && in_dom(ip, 0, i1);
  T* bnd = band + size_t(b) * g.S * g.ld;
  const size_t per = size_t(S1) * S2 * S3;
  const int sc = (g.S - 1) / 2;
  const int ntask = g.npen * 2 * S1;
  __syncthreads();  // tables staged

  // pencil-task operands: spline weights of the pencil and its coefficients.
  // Loads are issued for every lane (invalid tasks read coefficient 0 and get
  // zero weights) so the wait counters stay exact across iterations.
  auto task_load = [&](int u, int t, T* wgt, double* cv) {
    const int4 dd = dsl[u];
    const int c1 = t % S1;
    const int side = (t / S1) & 1;
    const int64_t pp = pen0 + t / (2 * S1);
    int j2 = int(pp % g.m2), j3 = int(pp / g.m2);
    if (side) {
      j2 -= dd.z;
      j3 -= dd.w;
    }
    const bool ok = in_dom(ip, 1, j2) && (ND == 2 || in_dom(ip, 2, j3)) && pp * g.m1 < g.N;
    if (!ok) {
      j2 = ip.lo[1];
      j3 = ND == 3 ? ip.lo[2] : 0;
    }
    const double* cu = coef + (size_t(b) * ip.nup + u) * per;
    const int f2 = tf2[j2];
    const T* b2 = tb2 + j2 * (Q + 1);
    const T z = ok ? T(1) : T(0);
    if constexpr (ND == 3) {
      const int f3 = tf3[j3];
      const T* b3 = tb3 + j3 * (Q + 1);
#pragma unroll
      for (int a3 = 0; a3 <= Q; ++a3)
#pragma unroll
        for (int a2 = 0; a2 <= Q; ++a2) {
          wgt[a3 * (Q + 1) + a2] = z * b3[a3] * b2[a2];
          cv[a3 * (Q + 1) + a2] = cu[(size_t(f3 + a3) * S2 + f2 + a2) * S1 + c1];
        }
    } else {
#pragma unroll
      for (int a2 = 0; a2 <= Q; ++a2) {
        wgt[a2] = z * b2[a2];
        cv[a2] = cu[size_t(f2 + a2) * S1 + c1];
      }
    }
  };
  T wgt[MULTI ? 1 : NC];
  double cv[MULTI ? 1 : NC];
  // The steady-state loop issues the same global loads and stores on every
  // thread and iteration (surplus threads reload a valid task, the last
  // iteration reloads the last delta, dead rows store into the zeroed
  // padding), so the compiler's memory-wait counters stay exact and the
  // operands prefetched one delta ahead are not drained early.
  const int tt = MULTI ? 0 : tid % ntask;
  if constexpr (!MULTI) task_load(0, tt, wgt, cv);
  T dsum = T(0);
  // dead rows (beyond N in the last chunk) write into the padding of slot 0,
  // which zero_pad clears afterwards
  const size_t irow = live ? size_t(i) : size_t(g.ld - 1);

  for (int u = 0; u < ip.nup; ++u) {
    const int4 dd = dsl[u];
    const int s = dd.x, dl1 = dd.y, dl2 = dd.z, dl3 = dd.w;
    T* Tu = Tbuf + size_t(u & 1) * ntask;
    // pencil contractions T[c1] = sum beta2 beta3 c[c3][c2][c1]
    if constexpr (!MULTI) {
      T v = T(0);
#pragma unroll
      for (int c = 0; c < NC; ++c) v += wgt[c] * T(cv[c]);
      if (tid < ntask) Tu[tid] = v;
      task_load(u + 1 < ip.nup ? u + 1 : u, tt, wgt, cv);
    } else {
      for (int t = tid; t < ntask; t += kChunk) {
        T w2[NC];
        double c2v[NC];
        T v = T(0);
        task_load(u, t, w2, c2v);
#pragma unroll
        for (int c = 0; c < NC; ++c) v += w2[c] * T(c2v[c]);
        Tu[t] = v;
      }
    }
    __syncthreads();
    const bool has_lo = FORM == IGS_STIFFNESS || s != sc;
    // placeholders (0) where the entry is not interpolated: the quadrature of
    // boundary rows and the copy kernel overwrite them
    T vu = T(0), vl = T(0);
    if (inner) {
      const T* Tk = Tu + size_t(k) * 2 * S1;
      const bool up = in_dom(ip, 0, i1 + dl1) && in_dom(ip, 1, i2 + dl2) && (ND == 2 || in_dom(ip, 2, i3 + dl3));
      if (up) {
        const int f1 = tf1[i1];
        const T* bb = tb1 + i1 * (Q + 1);
#pragma unroll
        for (int a = 0; a <= Q; ++a) vu += bb[a] * Tk[f1 + a];
      }
      if (has_lo) {
        const int j1 = i1 - dl1;
        const bool lo = in_dom(ip, 0, j1) && in_dom(ip, 1, i2 - dl2) && (ND == 2 || in_dom(ip, 2, i3 - dl3));
        if (lo) {
          const int f1 = tf1[j1];
          const T* bb = tb1 + j1 * (Q + 1);
#pragma unroll
          for (int a = 0; a <= Q; ++a) vl += bb[a] * Tk[S1 + f1 + a];
        }
      }
      if (FORM == IGS_STIFFNESS) dsum += vu + vl;
    }
    bnd[live ? size_t(s) * g.ld + irow : irow] = vu;
    if (has_lo) bnd[live ? size_t(g.S - 1 - s) * g.ld + irow : irow] = vl;
  }
  // diagonal of the interpolated part (the copy kernel subtracts the copies)
  if (FORM == IGS_STIFFNESS) bnd[live ? size_t(sc) * g.ld + irow : irow] = inner ? -dsum : T(0);
}

// Fast path: R rows per thread (chunks of R*kChunk rows), per-delta metadata
// read from a host-built table through the scalar cache, per-row domain tests
// as bitmasks.  The direction-1 weights are read from LDS for every delta:
// keeping a row's q+1 weights in registers costs the VGPRs that separate 4
// from 5 waves per SIMD, and the extra wave hides more of the stores.
// A thread carries NT pencil tasks: npen*2*S1 <= NT*kChunk (NT = 2 for the
// face/edge surrogate, whose lines carry the 4p layer coefficients too).
constexpr int kRows = 3;

// STAGE = true: the coefficient block that the chunk's pencil tasks read for a
// delta ((directions 2, 3) ranges of the chunk's pencils and their lower
// partners, all c1) is copied into LDS by coalesced loads two deltas ahead,
// instead of every task gathering its (q+1)^2 coefficients from memory.
// Chunks whose block exceeds kStage*kChunk values (face/edge chunks next to
// the boundary layers, where every layer has a coefficient of its own) gather
// instead; the choice is uniform per workgroup.
constexpr int kStage = 4;  // staged coefficients per thread (block <= kStage * kChunk)

// APPLY = true: the matrix-free surrogate apply (Sec. 1; remark after eq.
// 5.1c): the same evaluation, but each evaluated row accumulates
// sum_j A~_ij x_j over its interpolated entries (the diagonal as minus their
// sum for stiffness) into g.ay instead of writing the band; the band is not
// touched.
template <int ND, int FORM, int Q, typename T, bool STAGE, int NT, bool APPLY = false>
__global__ void __launch_bounds__(kChunk)
    fill_fast_kernel(KInterp<T> ip, FillGeom g, const int4* __restrict__ dsl, const double* __restrict__ coef,
                     T* __restrict__ band) {
  extern __shared__ char smem_raw[];
  constexpr int NC = (ND == 3) ? (Q + 1) * (Q + 1) : (Q + 1);
  constexpr int R = kRows;
  const int S1 = ip.Sd[0], S2 = ip.Sd[1], S3 = (ND == 3) ? ip.Sd[2] : 1;
  const int m3 = (ND == 3) ? g.m3 : 1;
  const int P = g.P;
  static_assert(STAGE || NT == 1, "the prefetching path carries one task per thread");
  const int blk = STAGE ? min(g.n3max * g.n2max * S1, kStage * kChunk) : 0;
  double* Cb = reinterpret_cast<double*>(smem_raw);  // [2][blk]
  T* Tbuf = reinterpret_cast<T*>(Cb + 2 * blk);
  T* tb1 = Tbuf + size_t(2) * g.npen * 2 * S1;
  T* tb2 = tb1 + size_t(g.m1) * (Q + 1);
  T* tb3 = tb2 + size_t(g.m2) * (Q + 1);
  int* tf1 = reinterpret_cast<int*>(tb3 + size_t(m3) * (Q + 1));
  int* tf2 = tf1 + g.m1;
  int* tf3 = tf2 + g.m2;
  const int b = blockIdx.y;
  const int64_t c0 = int64_t(g.chunks[blockIdx.x]) * (kChunk * R);
  const int tid = threadIdx.x;
  // tb1 is stored [a][i1] so that neighbouring lanes (neighbouring i1) read
  // neighbouring words; tb2, tb3 are read per pencil and stay [i][a]
  for (int d = 0; d < ND; ++d) {
    const int md = d == 0 ? g.m1 : (d == 1 ? g.m2 : m3);
    T* tb = d == 0 ? tb1 : (d == 1 ? tb2 : tb3);
    int* tf = d == 0 ? tf1 : (d == 1 ? tf2 : tf3);
    for (int t = tid; t < md * (Q + 1); t += kChunk) {
      const int ii = t / (Q + 1), a = t - ii * (Q + 1);
      const bool ok = in_dom(ip, d, ii);
      tb[d == 0 ? a * md + ii : t] = ok ? ip.eb[d][t] : T(0);
      if (a == 0) tf[ii] = ok ? ip.ef[d][ii] : 0;
    }
  }
  const int64_t pen0 = c0 / g.m1;
  T* bnd = band + size_t(b) * g.S * g.ld;
  const size_t per = size_t(S1) * S2 * S3;
  const int sc = (g.S - 1) / 2;
  const int ntask = g.npen * 2 * S1;
  const size_t ld = size_t(g.ld);
  const size_t Sm1ld = size_t(g.S - 1) * ld;

  // per-row state
  bool live[R], inner[R];
  int i1r[R], kr[R], mask[R], f1u[R];
  size_t irow[R];
  T dsum[R], yacc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    yacc[r] = T(0);
    const int64_t i = c0 + tid + int64_t(r) * kChunk;
    const int64_t pen = i < g.N ? i / g.m1 : pen0;
    const int i1 = i < g.N ? int(i - pen * g.m1) : 0;
    const int i2 = int(pen % g.m2), i3 = int(pen / g.m2);
    // rows of pencils outside the analysis domain in (i2, i3) belong to the
    // quadrature alone (whole pencils: their lines are not shared with domain
    // rows except at the two ends of a run of domain pencils) and are not
    // written here; rows of domain pencils outside it in i1 share lines with
    // domain rows and get placeholders that their quadrature overwrites later
    live[r] = i < g.N && in_dom(ip, 1, i2) && (ND == 2 || in_dom(ip, 2, i3));
    inner[r] = live[r] && in_dom(ip, 0, i1);
    i1r[r] = i1;
    kr[r] = int(pen - pen0);
    irow[r] = live[r] ? size_t(i) : size_t(g.ld - 1);
    // bit (d*9 + t) set iff index i_d + t - P lies in the analysis range
    int mk = 0;
    for (int t = 0; t <= 2 * P; ++t) {
      mk |= (in_dom(ip, 0, i1 + t - P) ? 1 : 0) << t;
      mk |= (in_dom(ip, 1, i2 + t - P) ? 1 : 0) << (9 + t);
      if (ND == 3) mk |= (in_dom(ip, 2, i3 + t - P) ? 1 : 0) << (18 + t);
    }
    mask[r] = mk;
    dsum[r] = T(0);
  }
  __syncthreads();  // tables staged
#pragma unroll
  for (int r = 0; r < R; ++r) {
    f1u[r] = tf1[i1r[r]];
  }

  auto inside = [&](int mk, int d1, int d2, int d3) {
    int v = (mk >> (d1 + P)) & (mk >> (9 + d2 + P));
    if (ND == 3) v &= mk >> (18 + d3 + P);
    return (v & 1) != 0;
  };
  // coefficient block of the chunk: c2 in [c2lo, c2lo + n2), c3 in [c3lo, c3lo + n3)
  int c2lo = 0, c3lo = 0, n2 = 1, n3 = 1;
  if constexpr (STAGE) {
    int i2a = ip.hi[1], i2b = ip.lo[1], i3a = ND == 3 ? ip.hi[2] : 0, i3b = ND == 3 ? ip.lo[2] : 0;
    for (int k = 0; k < g.npen; ++k) {
      const int64_t pp = pen0 + k;
      if (pp * g.m1 >= g.N) break;
      const int j2 = int(pp % g.m2), j3 = int(pp / g.m2);
      if (!in_dom(ip, 1, j2) || (ND == 3 && !in_dom(ip, 2, j3))) continue;
      i2a = min(i2a, j2);
      i2b = max(i2b, j2);
      i3a = min(i3a, j3);
      i3b = max(i3b, j3);
    }
    const int j2lo = max(ip.lo[1], i2a - P), j2hi = min(ip.hi[1], i2b + P);
    c2lo = tf2[j2lo];
    n2 = tf2[j2hi] + Q + 1 - c2lo;
    if (ND == 3) {
      const int j3lo = max(ip.lo[2], i3a - P), j3hi = min(ip.hi[2], i3b + P);
      c3lo = tf3[j3lo];
      n3 = tf3[j3hi] + Q + 1 - c3lo;
    }
  }
  const int nblk = n3 * n2 * S1;
  // this chunk stages its blocks (uniform per workgroup); with one task per
  // thread the host has checked that every block fits
  constexpr bool MIXED = NT > 1;
  const bool stg = STAGE && (!MIXED || nblk <= kStage * kChunk);
  double cs[kStage];
  // this thread's staged block entries: offsets into a delta's coefficient
  // array (loop-invariant; -1 for entries beyond the block)
  int soff[kStage];
#pragma unroll
  for (int k = 0; k < kStage; ++k) {
    const int e = tid + k * kChunk;
    const int c1 = e % S1, r = e / S1;
    const int l2 = r % n2, l3 = r / n2;
    soff[k] = (stg && e < nblk) ? int((size_t(c3lo + l3) * S2 + c2lo + l2) * S1 + c1) : -1;
  }
  auto stage_load = [&](int u) {
    const double* cu = coef + (size_t(b) * ip.nup + u) * per;
#pragma unroll
    for (int k = 0; k < kStage; ++k)
      if (soff[k] >= 0) cs[k] = cu[soff[k]];
  };
  auto stage_store = [&](int u) {
    double* cb = Cb + (u & 1) * blk;
#pragma unroll
    for (int k = 0; k < kStage; ++k)
      if (soff[k] >= 0) cb[tid + k * kChunk] = cs[k];
  };
  if (stg) {
    stage_load(0);
    stage_store(0);
    if (ip.nup > 1) stage_load(1);
  }
  __syncthreads();  // block 0 visible
  // pencil task operands (loaded one delta ahead); every thread loads a valid task
  int tc1[NT], tside[NT], tj2[NT], tj3[NT];
  int64_t tpp[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const int tt = (tid + k * kChunk) % ntask;
    tc1[k] = tt % S1;
    tside[k] = (tt / S1) & 1;
    tpp[k] = pen0 + tt / (2 * S1);
    tj2[k] = int(tpp[k] % g.m2);
    tj3[k] = int(tpp[k] / g.m2);
  }
  double cv[STAGE ? 1 : NC];
  bool tok[NT];
  int tf2v[NT], tf3v[NT], tj2v[NT], tj3v[NT];
  auto task_load = [&](int u) {
    const int4 dd = dsl[u];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      int j2 = tj2[k], j3 = tj3[k];
      if (tside[k]) {
        j2 -= dd.z;
        j3 -= dd.w;
      }
      tok[k] = in_dom(ip, 1, j2) && (ND == 2 || in_dom(ip, 2, j3)) && tpp[k] * g.m1 < g.N;
      if (!tok[k]) {
        j2 = ip.lo[1];
        j3 = ND == 3 ? ip.lo[2] : 0;
      }
      tj2v[k] = j2;
      tj3v[k] = j3;
      tf2v[k] = tf2[j2];
      tf3v[k] = ND == 3 ? tf3[j3] : 0;
    }
    if constexpr (!STAGE) {
      const double* cu = coef + (size_t(b) * ip.nup + u) * per;
#pragma unroll
      for (int a3 = 0; a3 < (ND == 3 ? Q + 1 : 1); ++a3)
#pragma unroll
        for (int a2 = 0; a2 <= Q; ++a2)
          cv[a3 * (Q + 1) + a2] = cu[(size_t(tf3v[0] + a3) * S2 + tf2v[0] + a2) * S1 + tc1[0]];
    }
  };
  task_load(0);

  for (int u = 0; u < ip.nup; ++u) {
    const int4 dd = dsl[u];
    const int s = dd.x, dl1 = dd.y, dl2 = dd.z, dl3 = dd.w;
    T* Tu = Tbuf + size_t(u & 1) * ntask;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      const int task = tid + k * kChunk;
      if (NT > 1 && task >= ntask) break;
      const T* b2 = tb2 + tj2v[k] * (Q + 1);
      T v = T(0);
      if constexpr (STAGE) {
        if (!MIXED || stg) {
          // tasks outside the evaluated range read a clamped (valid) block
          // entry and are zeroed below
          const int l2 = min(max(tf2v[k] - c2lo, 0), n2 - Q - 1);
          const int l3 = ND == 3 ? min(max(tf3v[k] - c3lo, 0), n3 - Q - 1) : 0;
          const double* cb = Cb + (u & 1) * blk + (size_t(l3) * n2 + l2) * S1 + tc1[k];
#pragma unroll
          for (int a3 = 0; a3 < (ND == 3 ? Q + 1 : 1); ++a3) {
            T r2 = T(0);
#pragma unroll
            for (int a2 = 0; a2 <= Q; ++a2) r2 += b2[a2] * T(cb[(a3 * n2 + a2) * S1]);
            v += (ND == 3 ? tb3[tj3v[k] * (Q + 1) + a3] : T(1)) * r2;
          }
        } else if constexpr (MIXED) {
          // the same contraction from memory
          const double* cb = coef + (size_t(b) * ip.nup + u) * per + (size_t(tf3v[k]) * S2 + tf2v[k]) * S1 + tc1[k];
#pragma unroll
          for (int a3 = 0; a3 < (ND == 3 ? Q + 1 : 1); ++a3) {
            T r2 = T(0);
#pragma unroll
            for (int a2 = 0; a2 <= Q; ++a2) r2 += b2[a2] * T(cb[(size_t(a3) * S2 + a2) * S1]);
            v += (ND == 3 ? tb3[tj3v[k] * (Q + 1) + a3] : T(1)) * r2;
          }
        }
      } else {
#pragma unroll
        for (int a3 = 0; a3 < (ND == 3 ? Q + 1 : 1); ++a3) {
          T r2 = T(0);
#pragma unroll
          for (int a2 = 0; a2 <= Q; ++a2) r2 += b2[a2] * T(cv[a3 * (Q + 1) + a2]);
          v += (ND == 3 ? tb3[tj3v[k] * (Q + 1) + a3] : T(1)) * r2;
        }
      }
      if (task < ntask) Tu[task] = tok[k] ? v : T(0);
    }
    task_load(u + 1 < ip.nup ? u + 1 : u);
    if (stg) {
      // block u+1 (loaded during the previous delta) into the other buffer, whose
      // readers finished before the previous barrier; then fetch block u+2
      if (u + 1 < ip.nup) stage_store(u + 1);
      if (u + 2 < ip.nup) stage_load(u + 2);
    }
    __syncthreads();
    const bool has_lo = FORM == IGS_STIFFNESS || s != sc;
    const size_t su = size_t(s) * ld, sl = Sm1ld - size_t(s) * ld;
    const int64_t xoff = APPLY ? int64_t(dl1) + int64_t(g.m1) * (dl2 + int64_t(g.m2) * dl3) : 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      // placeholders (0) where the entry is not interpolated: the quadrature of
      // boundary rows and the copy kernel overwrite them
      // branch-free: every row evaluates both (its table reads stay in range:
      // rows outside the domain have zero weights and first function 0) and
      // the domain tests select
      const T* Tk = Tu + size_t(kr[r]) * 2 * S1;
      T vu = T(0), vl = T(0);
#pragma unroll
      for (int a = 0; a <= Q; ++a) vu += tb1[a * g.m1 + i1r[r]] * Tk[f1u[r] + a];
      vu = (inner[r] && inside(mask[r], dl1, dl2, dl3)) ? vu : T(0);
      if (has_lo) {
        const int j1 = min(max(i1r[r] - dl1, 0), g.m1 - 1);
        const int f1 = tf1[j1];
#pragma unroll
        for (int a = 0; a <= Q; ++a) vl += tb1[a * g.m1 + j1] * Tk[S1 + f1 + a];
        vl = (inner[r] && inside(mask[r], -dl1, -dl2, -dl3)) ? vl : T(0);
      }
      if (FORM == IGS_STIFFNESS) dsum[r] += vu + vl;
      if constexpr (APPLY) {
        // an evaluated row's partners stay within p of it, inside the box
        if (inner[r]) {
          const T* xb = static_cast<const T*>(g.ax) + size_t(b) * g.N + irow[r];
          yacc[r] += vu * xb[xoff];
          if (has_lo) yacc[r] += vl * xb[-xoff];
        }
      } else {
        bnd[live[r] ? su + irow[r] : irow[r]] = vu;
        if (has_lo) bnd[live[r] ? sl + irow[r] : irow[r]] = vl;
      }
    }
  }
  if constexpr (APPLY) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!inner[r]) continue;
      const size_t k = size_t(b) * g.N + irow[r];
      T v = yacc[r];
      if (FORM == IGS_STIFFNESS) v -= dsum[r] * static_cast<const T*>(g.ax)[k];
      static_cast<T*>(g.ay)[k] = v;
    }
    return;
  }
  // diagonal of the interpolated part (the copy kernel subtracts the copies)
  if (FORM == IGS_STIFFNESS) {
#pragma unroll
    for (int r = 0; r < R; ++r) bnd[live[r] ? size_t(sc) * ld + irow[r] : irow[r]] = inner[r] ? -dsum[r] : T(0);
  }
}

// Zero the padding k in [N, ld) of every slot.
template <typename T>
__global__ void zero_pad_kernel(T* band, int64_t N, int64_t ld, int slots_total) {
  const int64_t pad = ld - N;
  const int64_t total = pad * slots_total;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t s = t / pad;
    band[s * ld + N + (t - s * pad)] = T(0);
  }
}

// ------------------------------------------------------------------ copy ----
//
// Analysis-domain rows whose stencil leaves the analysis domain (listed on the
// host in flat order): every slot whose partner j = i + delta lies outside
// takes the exact entry A_ij, read as A_ji from slot -delta of row j (a row
// assembled by quadrature; the form is symmetric), and the stiffness
// diagonal, which the fill left at minus the sum of the interpolated entries,
// loses these entries too (eq. 5.1c).  Runs after the fill and every
// quadrature launch of the assembly.
//
// A workgroup takes 64 rows (one per lane); its four waves split the rows'
// (delta2, delta3) lines, so each wave waits on memory about a quarter as
// often, and the 2p+1 loads of a line are issued before any is used.  The
// waves' partial sums meet in LDS in a fixed order.
constexpr int kCopyWaves = 4;

// APPLY = true (matrix-free apply): the copied entries are not stored; the row
// adds sum_j A_ij (x_j - x_i) over them to y_i (stiffness: the diagonal loses
// them), or sum_j A_ij x_j (mass).  Runs after the evaluation of the domain
// rows (fill_fast_kernel with APPLY), which wrote y_i.
// FIXUP = true (3-D stiffness, after boundary quadrature with transposed
// stores): the copied entries are already in place in the row's own slots;
// the row only subtracts them from its diagonal, reading its own entries
// (consecutive rows, coalesced) instead of its partners'.
template <int ND, int FORM, int P, typename T, bool APPLY = false, bool FIXUP = false>
__global__ void __launch_bounds__(64 * kCopyWaves)
    copy_kernel(KInterp<T> ip, int m1, int m2, int64_t ld, int S, const int* __restrict__ rows, int nrows,
                T* __restrict__ band, const T* __restrict__ x = nullptr, T* __restrict__ y = nullptr, int64_t N = 0) {
  constexpr int W = 2 * P + 1, NL = ND == 3 ? W * W : W;
  __shared__ T part[kCopyWaves][64];
  __shared__ T xpart[kCopyWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + lane;
  const bool ok = t < nrows;
  const int64_t i = rows[ok ? t : 0];
  const int64_t pen = i / m1;
  const int i1 = int(i - pen * m1), i2 = int(pen % m2), i3 = ND == 3 ? int(pen / m2) : 0;
  T* bnd = band + size_t(blockIdx.y) * S * ld;
  const size_t Sm1ld = size_t(S - 1) * ld;
  int o1 = 0;  // bit d1 + P: i1 + d1 leaves the domain
#pragma unroll
  for (int d1 = -P; d1 <= P; ++d1) o1 |= in_dom(ip, 0, i1 + d1) ? 0 : 1 << (d1 + P);
  T csum = T(0), xsum = T(0);
  const T* xb = APPLY ? x + size_t(blockIdx.y) * N : nullptr;
  for (int L = w; L < NL; L += kCopyWaves) {
    const int d2 = L % W - P, d3 = ND == 3 ? L / W - P : 0;
    const bool out23 = !in_dom(ip, 1, i2 + d2) || (ND == 3 && !in_dom(ip, 2, i3 + d3));
    const int om = ok ? (out23 ? (1 << W) - 1 : o1) : 0;
    const int s0 = W * L;
    const int64_t off0 = int64_t(m1) * (d2 + int64_t(m2) * d3);
    T v[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
      v[k] = T(0);
      if (om >> k & 1)
        v[k] = FIXUP ? bnd[size_t(s0 + k) * ld + size_t(i)]
                     : bnd[Sm1ld - size_t(s0 + k) * ld + size_t(i + off0 + (k - P))];
    }
#pragma unroll
    for (int k = 0; k < W; ++k)
      if (om >> k & 1) {
        if constexpr (APPLY)
          xsum += v[k] * xb[i + off0 + (k - P)];
        else if constexpr (!FIXUP)
          bnd[size_t(s0 + k) * ld + size_t(i)] = v[k];
        csum += v[k];
      }
  }
  if constexpr (APPLY) {
    part[w][lane] = csum;
    xpart[w][lane] = xsum;
    __syncthreads();
    if (w == 0 && ok) {
      T c = part[0][lane], xs = xpart[0][lane];
#pragma unroll
      for (int k = 1; k < kCopyWaves; ++k) {
        c += part[k][lane];
        xs += xpart[k][lane];
      }
      T* yi = y + size_t(blockIdx.y) * N + size_t(i);
      *yi += FORM == IGS_STIFFNESS ? xs - c * xb[i] : xs;
    }
  } else if (FORM == IGS_STIFFNESS) {
    part[w][lane] = csum;
    __syncthreads();
    if (w == 0 && ok) {
      T c = part[0][lane];
#pragma unroll
      for (int k = 1; k < kCopyWaves; ++k) c += part[k][lane];
      const size_t ic = size_t((S - 1) / 2) * ld + size_t(i);
      bnd[ic] = bnd[ic] - c;
    }
  }
}

// Matrix-free apply, the rows assembled by quadrature (listed): y_i =
// sum_s band[s][i] x_{i+delta_s} from the stored rows; Dirichlet rows give 0
// when dirichlet is set (x is then already zero on the Dirichlet dofs).  One
// row per thread: consecutive threads read consecutive entries of a slot.
// Workgroups are dealt round-robin to the 8 XCDs; XCD x takes a contiguous
// range of the list, so the x planes its rows touch stay in its L2.
template <typename T>
__global__ void __launch_bounds__(256)
    rows_spmv_kernel(int n, int P, int m1, int m2, int m3, int64_t N, int64_t ld, int S, const int* __restrict__ rows,
                     int nrows, const T* __restrict__ band, const T* __restrict__ x, T* __restrict__ y, int dirichlet) {
  const int nb = gridDim.x, per = nb / 8;
  const int bid = (per == 0 || int(blockIdx.x) >= per * 8) ? int(blockIdx.x) : int(blockIdx.x % 8) * per + int(blockIdx.x / 8);
  const int t = bid * 256 + threadIdx.x;
  if (t >= nrows) return;
  const int b = blockIdx.y;
  const int64_t i = rows[t];
  const int i1 = int(i % m1), i2 = int((i / m1) % m2), i3 = n == 3 ? int(i / (int64_t(m1) * m2)) : 0;
  T* yb = y + size_t(b) * N;
  if (dirichlet) {
    const bool dr = i1 == 0 || i1 == m1 - 1 || i2 == 0 || i2 == m2 - 1 || (n == 3 && (i3 == 0 || i3 == m3 - 1));
    if (dr) {
      yb[i] = T(0);
      return;
    }
  }
  const T* bb = band + size_t(b) * S * ld + size_t(i);
  const T* xb = x + size_t(b) * N;
  const int W = 2 * P + 1;
  T acc = T(0);
  for (int s = 0; s < S; ++s) {
    const int d1 = s % W - P, d2 = (s / W) % W - P, d3 = n == 3 ? s / (W * W) - P : 0;
    // entries whose partner leaves the box are stored as 0: clamp the read
    int64_t j = i + d1 + int64_t(m1) * (d2 + int64_t(m2) * d3);
    j = j < 0 ? 0 : (j >= N ? N - 1 : j);
    acc += bb[size_t(s) * ld] * xb[j];
  }
  yb[i] = acc;
}

// 2-D fit in one launch, for small sample grids (S1 S2 <= kFit2dLds): one
// workgroup per (upper stencil function, problem) gathers its S1 x S2 sample
// values into LDS, applies ginv_1 along direction 1 into a second LDS grid and
// ginv_2 along direction 2 into the coefficients, with fit_pass_kernel's
// arithmetic (the identity outside [flo, fhi), four partial sums).  On small
// 2-D meshes the two passes are two latency-bound launches; here each
// workgroup does both.  Its work grows as S^3 on nup x batch workgroups, so
// larger grids keep the two passes (2D p=2 q=5: 64^2 and 128^2 elements,
// S <= 26, fit 13 -> 8 us; at S = 36 and 50 one workgroup per function was
// slower than the passes).
constexpr int kFit2dLds = 1024;  // values per grid (two grids: 16 KB)
template <typename BT>
__global__ void __launch_bounds__(256)
    fit2d_lds_kernel(KInterp<double> ip, int m1, int64_t ld, int S, const BT* __restrict__ band,
                     double* __restrict__ coef) {
  __shared__ double X[kFit2dLds], Y[kFit2dLds];
  const int S1 = ip.Sd[0], S2 = ip.Sd[1], n12 = S1 * S2;
  const int u = blockIdx.x, b = blockIdx.y;
  const BT* bs = band + (size_t(b) * S + ip.upslot[u]) * ld;
  for (int t = threadIdx.x; t < n12; t += blockDim.x) {
    const int k1 = t % S1, k2 = t / S1;
    X[t] = double(bs[size_t(m1) * ip.samp[1][k2] + ip.samp[0][k1]]);
  }
  __syncthreads();
  // one direction: out[k] = sum_j ginv_d[kd][j] in[k with kd -> j]
  auto pass = [&](int d, const double* in, double* out, bool global) {
    const int Sd = ip.Sd[d], flo = ip.flo[d], fhi = ip.fhi[d];
    const size_t stride = d == 0 ? 1 : size_t(S1);
    for (int t = threadIdx.x; t < n12; t += blockDim.x) {
      const int k1 = t % S1, k2 = t / S1;
      const int kd = d == 0 ? k1 : k2;
      const double* sp = in + (d == 0 ? size_t(k2) * S1 : size_t(k1));
      double v;
      if (kd < flo || kd >= fhi) {
        v = sp[kd * stride];
      } else {
        const double* g = ip.ginv[d] + size_t(kd) * Sd;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        const int J4 = flo + ((fhi - flo) & ~3);
        for (int j = flo; j < J4; j += 4) {
          a0 += g[j] * sp[j * stride];
          a1 += g[j + 1] * sp[(j + 1) * stride];
          a2 += g[j + 2] * sp[(j + 2) * stride];
          a3 += g[j + 3] * sp[(j + 3) * stride];
        }
        for (int j = J4; j < fhi; ++j) a0 += g[j] * sp[j * stride];
        v = (a0 + a1) + (a2 + a3);
      }
      if (global)
        out[(size_t(b) * ip.nup + u) * n12 + t] = v;
      else
        out[t] = v;
    }
  };
  pass(0, X, Y, false);
  __syncthreads();
  pass(1, Y, coef, true);
}

bool fit_2d_lds(const KInterp<double>& ip, int n) { return n == 2 && ip.Sd[0] * ip.Sd[1] <= kFit2dLds; }

// ------------------------------------------------------------ launchers ----

template <typename BT>
hipError_t launch_fit(const KInterp<double>& ip, int n, int m1, int m2, int64_t ld, int S, int batch, const BT* band,
                      double* tmp0, double* tmp1, double* coef, const double* g0T, hipStream_t s) {
  if (fit_2d_lds(ip, n)) {
    hipLaunchKernelGGL((fit2d_lds_kernel<BT>), dim3(ip.nup, batch), dim3(256), 0, s, ip, m1, ld, S, band, coef);
    return hipGetLastError();
  }
  int64_t total = int64_t(ip.Sd[0]) * ip.Sd[1] * (n == 3 ? ip.Sd[2] : 1) * ip.nup * batch;
  int blocks = int(std::min<int64_t>((total + 255) / 256, 65535));
  double* bufs[3];
  if (n == 3) {
    bufs[0] = tmp0; bufs[1] = tmp1; bufs[2] = coef;
  } else {
    bufs[0] = tmp0; bufs[1] = coef; bufs[2] = nullptr;
  }
  hipLaunchKernelGGL((fit_pass_kernel<BT, true>), dim3(blocks), dim3(256), 0, s, ip, 0, n, m1, m2, ld, S, batch, band,
                     nullptr, bufs[0], g0T);
  for (int d = 1; d < n; ++d)
    hipLaunchKernelGGL((fit_pass_kernel<BT, false>), dim3(blocks), dim3(256), 0, s, ip, d, n, m1, m2, ld, S, batch,
                       band, bufs[d - 1], bufs[d], static_cast<const double*>(nullptr));
  return hipGetLastError();
}

// one separable pass out = (ginv_d applied along direction d) in, no gather
template <typename T>
hipError_t launch_fit_pass_plain(const KInterp<double>& ip, int d, int n, int batch, const double* in, double* out,
                                 hipStream_t s) {
  int64_t total = int64_t(ip.Sd[0]) * ip.Sd[1] * (n == 3 ? ip.Sd[2] : 1) * ip.nup * batch;
  int blocks = int(std::min<int64_t>((total + 255) / 256, 65535));
  hipLaunchKernelGGL((fit_pass_kernel<T, false>), dim3(blocks), dim3(256), 0, s, ip, d, n, 0, 0, int64_t(0), 0, batch,
                     static_cast<const T*>(nullptr), in, out, static_cast<const double*>(nullptr));
  return hipGetLastError();
}
template hipError_t launch_fit_pass_plain<double>(const KInterp<double>&, int, int, int, const double*, double*,
                                                  hipStream_t);

template hipError_t launch_fit<double>(const KInterp<double>&, int, int, int, int64_t, int, int, const double*,
                                       double*, double*, double*, const double*, hipStream_t);
template hipError_t launch_fit<float>(const KInterp<double>&, int, int, int, int64_t, int, int, const float*,
                                      double*, double*, double*, const double*, hipStream_t);

// chunk ids (of `rows` rows) that contain at least one row the fill
// evaluates: rows with every i_d in [lo[d], hi[d]]
std::vector<int> fill_chunks(const Dims& d, int rows, const int lo[3], const int hi[3]) {
  std::vector<int> out;
  const int lo3 = (d.n == 3) ? lo[2] : 0, hi3 = (d.n == 3) ? hi[2] : 0;
  for (int i3 = lo3; i3 <= hi3; ++i3)
    for (int i2 = lo[1]; i2 <= hi[1]; ++i2) {
      const int64_t base = int64_t(d.m[0]) * (i2 + int64_t(d.m[1]) * i3);
      const int a = int((base + lo[0]) / rows), z = int((base + hi[0]) / rows);
      for (int c = a; c <= z; ++c)
        if (out.empty() || out.back() < c) out.push_back(c);
    }
  return out;
}

int fill_npen(const Dims& d, int rows) { return (rows - 1) / d.m[0] + 2; }

// rows per chunk of the fill launch: the fast kernel when its pencil tasks fit
// one per thread, or two per thread with a staged block of kStage*kChunk
// values that fits LDS with the tables; else the generic one
int fill_chunk_rows(const Dims& d, int Sd1, int q, int nup) {
  const int npen = fill_npen(d, kChunk * kRows), ntask = npen * 2 * Sd1;
  if (ntask <= kChunk) return kChunk * kRows;
  const size_t msum = size_t(d.m[0]) + d.m[1] + (d.n == 3 ? d.m[2] : 1);
  const size_t lds = size_t(2) * kStage * kChunk * sizeof(double) + size_t(2) * ntask * sizeof(double) +
                     msum * (q + 1) * sizeof(double) + (msum + 4) * 4 + size_t(nup) * 16;
  return ntask <= 2 * kChunk && lds <= 160 * 1024 ? kChunk * kRows : kChunk;
}

template <typename T>
size_t fill_lds_bytes(const KInterp<T>& ip, int npen, const Dims& d, int blk) {
  const size_t msum = size_t(d.m[0]) + d.m[1] + (d.n == 3 ? d.m[2] : 1);
  return size_t(2) * blk * sizeof(double) + size_t(2) * npen * 2 * ip.Sd[0] * sizeof(T) +
         msum * (ip.q + 1) * sizeof(T) + (msum + 4) * 4 + size_t(ip.nup) * 16;
}

// Largest coefficient block (extent in directions 2 and 3) that the pencil
// tasks of one fill chunk read; mirrors the bounds the fast kernel computes.
void fill_block_dims(const Dims& d, const std::vector<int> ef[3], int q, const std::vector<int>& chunks, int rows,
                     const int lo[3], const int hi[3], int* n2max, int* n3max) {
  const int p = d.p, npen = fill_npen(d, rows);
  const int lo2 = lo[1], hi2 = hi[1];
  const int lo3 = d.n == 3 ? lo[2] : 0, hi3 = d.n == 3 ? hi[2] : 0;
  *n2max = 1;
  *n3max = 1;
  for (int c : chunks) {
    const int64_t pen0 = int64_t(c) * rows / d.m[0];
    int i2a = hi2, i2b = lo2, i3a = hi3, i3b = lo3;
    for (int k = 0; k < npen; ++k) {
      const int64_t pp = pen0 + k;
      if (pp * d.m[0] >= d.N) break;
      const int j2 = int(pp % d.m[1]), j3 = int(pp / d.m[1]);
      if (j2 < lo2 || j2 > hi2 || j3 < lo3 || j3 > hi3) continue;
      i2a = std::min(i2a, j2);
      i2b = std::max(i2b, j2);
      i3a = std::min(i3a, j3);
      i3b = std::max(i3b, j3);
    }
    const int j2lo = std::max(lo2, i2a - p), j2hi = std::min(hi2, i2b + p);
    *n2max = std::max(*n2max, ef[1][j2hi] + q + 1 - ef[1][j2lo]);
    if (d.n == 3) {
      const int j3lo = std::max(lo3, i3a - p), j3hi = std::min(hi3, i3b + p);
      *n3max = std::max(*n3max, ef[2][j3hi] + q + 1 - ef[2][j3lo]);
    }
  }
}

template <int ND, int FORM, typename T, bool MULTI>
static void launch_fill_q(const KInterp<T>& ip, const FillGeom& g, dim3 grid, size_t lds, const double* coef, T* band,
                          hipStream_t s) {
  switch (ip.q) {
    case 1: hipLaunchKernelGGL((fill_kernel<ND, FORM, 1, T, MULTI>), grid, dim3(kChunk), lds, s, ip, g, coef, band); break;
    case 2: hipLaunchKernelGGL((fill_kernel<ND, FORM, 2, T, MULTI>), grid, dim3(kChunk), lds, s, ip, g, coef, band); break;
    case 3: hipLaunchKernelGGL((fill_kernel<ND, FORM, 3, T, MULTI>), grid, dim3(kChunk), lds, s, ip, g, coef, band); break;
    case 4: hipLaunchKernelGGL((fill_kernel<ND, FORM, 4, T, MULTI>), grid, dim3(kChunk), lds, s, ip, g, coef, band); break;
    default: hipLaunchKernelGGL((fill_kernel<ND, FORM, 5, T, MULTI>), grid, dim3(kChunk), lds, s, ip, g, coef, band); break;
  }
}

template <int ND, int FORM, typename T>
static void launch_fill_m(const KInterp<T>& ip, const FillGeom& g, dim3 grid, size_t lds, const double* coef, T* band,
                          hipStream_t s) {
  if (g.npen * 2 * ip.Sd[0] <= kChunk)
    launch_fill_q<ND, FORM, T, false>(ip, g, grid, lds, coef, band, s);
  else
    launch_fill_q<ND, FORM, T, true>(ip, g, grid, lds, coef, band, s);
}

template <int ND, int FORM, typename T, bool STAGE, int NT>
static void launch_fast_q(const KInterp<T>& ip, const FillGeom& g, dim3 grid, size_t lds, const int4* dsl,
                          const double* coef, T* band, hipStream_t s) {
  switch (ip.q) {
    case 1: hipLaunchKernelGGL((fill_fast_kernel<ND, FORM, 1, T, STAGE, NT>), grid, dim3(kChunk), lds, s, ip, g, dsl, coef, band); break;
    case 2: hipLaunchKernelGGL((fill_fast_kernel<ND, FORM, 2, T, STAGE, NT>), grid, dim3(kChunk), lds, s, ip, g, dsl, coef, band); break;
    case 3: hipLaunchKernelGGL((fill_fast_kernel<ND, FORM, 3, T, STAGE, NT>), grid, dim3(kChunk), lds, s, ip, g, dsl, coef, band); break;
    case 4: hipLaunchKernelGGL((fill_fast_kernel<ND, FORM, 4, T, STAGE, NT>), grid, dim3(kChunk), lds, s, ip, g, dsl, coef, band); break;
    default: hipLaunchKernelGGL((fill_fast_kernel<ND, FORM, 5, T, STAGE, NT>), grid, dim3(kChunk), lds, s, ip, g, dsl, coef, band); break;
  }
}

// stage: coefficient blocks staged in LDS where they fit (else the one-task,
// prefetching form); two tasks per thread need staging
template <int ND, int FORM, typename T>
static void launch_fast_s(const KInterp<T>& ip, const FillGeom& g, bool stage, dim3 grid, size_t lds,
                          const int4* dsl, const double* coef, T* band, hipStream_t s) {
  const bool two = g.npen * 2 * ip.Sd[0] > kChunk;
  if (stage && two)
    launch_fast_q<ND, FORM, T, true, 2>(ip, g, grid, lds, dsl, coef, band, s);
  else if (stage)
    launch_fast_q<ND, FORM, T, true, 1>(ip, g, grid, lds, dsl, coef, band, s);
  else
    launch_fast_q<ND, FORM, T, false, 1>(ip, g, grid, lds, dsl, coef, band, s);
}

template <typename T>
hipError_t launch_fill(const KInterp<T>& ip, int form, const Dims& d, const int* chunks, int nchunks, int chunk_rows,
                       int n2max, int n3max, const int4* dsl, const double* coef, T* band, hipStream_t s) {
  if (fill_is_2d(d)) return launch_fill2d<T>(ip, form, d, dsl, coef, band, s);
  FillGeom g;
  g.n = d.n;
  g.P = d.p;
  g.m1 = d.m[0];
  g.m2 = d.m[1];
  g.m3 = d.m[2];
  g.N = d.N;
  g.ld = d.ld;
  g.S = d.S;
  g.npen = fill_npen(d, chunk_rows);
  g.nchunks = nchunks;
  g.chunks = chunks;
  g.n2max = n2max;
  g.n3max = n3max;
  const bool fast = chunk_rows == kChunk * kRows;
  const bool two = g.npen * 2 * ip.Sd[0] > kChunk;
  // one task per thread: stage when every block fits (else prefetch); two
  // tasks: blocks capped at kStage*kChunk, larger ones gathered from memory
  const int blk = two ? std::min(n2max * n3max * ip.Sd[0], kStage * kChunk) : n2max * n3max * ip.Sd[0];
  const bool stage = fast && (two || blk <= kStage * kChunk) && fill_lds_bytes<T>(ip, g.npen, d, blk) <= 160 * 1024;
  if (fast && two && !stage) return hipErrorInvalidValue;
  const size_t lds = fill_lds_bytes<T>(ip, g.npen, d, stage ? blk : 0);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (nchunks == 0) return hipSuccess;
  dim3 grid(nchunks, d.batch);
  if (fast) {
    if (d.n == 3) {
      if (form == IGS_MASS)
        launch_fast_s<3, IGS_MASS, T>(ip, g, stage, grid, lds, dsl, coef, band, s);
      else
        launch_fast_s<3, IGS_STIFFNESS, T>(ip, g, stage, grid, lds, dsl, coef, band, s);
    } else {
      if (form == IGS_MASS)
        launch_fast_s<2, IGS_MASS, T>(ip, g, stage, grid, lds, dsl, coef, band, s);
      else
        launch_fast_s<2, IGS_STIFFNESS, T>(ip, g, stage, grid, lds, dsl, coef, band, s);
    }
    return hipGetLastError();
  }
  if (d.n == 3) {
    if (form == IGS_MASS)
      launch_fill_m<3, IGS_MASS, T>(ip, g, grid, lds, coef, band, s);
    else
      launch_fill_m<3, IGS_STIFFNESS, T>(ip, g, grid, lds, coef, band, s);
  } else {
    if (form == IGS_MASS)
      launch_fill_m<2, IGS_MASS, T>(ip, g, grid, lds, coef, band, s);
    else
      launch_fill_m<2, IGS_STIFFNESS, T>(ip, g, grid, lds, coef, band, s);
  }
  return hipGetLastError();
}

template hipError_t launch_fill<double>(const KInterp<double>&, int, const Dims&, const int*, int, int, int, int,
                                        const int4*, const double*, double*, hipStream_t);
template hipError_t launch_fill<float>(const KInterp<float>&, int, const Dims&, const int*, int, int, int, int,
                                       const int4*, const double*, float*, hipStream_t);
template size_t fill_lds_bytes<double>(const KInterp<double>&, int, const Dims&, int);
template size_t fill_lds_bytes<float>(const KInterp<float>&, int, const Dims&, int);

// ------------------------------------------------------ matrix-free apply ----

// xm = x with the Dirichlet dofs zeroed
template <typename T>
__global__ void mask_dirichlet_kernel(int n, int m1, int m2, int m3, int64_t N, int batch, const T* __restrict__ x,
                                      T* __restrict__ xm) {
  const int64_t total = N * batch;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = t % N;
    const int i1 = int(i % m1), i2 = int((i / m1) % m2), i3 = n == 3 ? int(i / (int64_t(m1) * m2)) : 0;
    const bool dr = i1 == 0 || i1 == m1 - 1 || i2 == 0 || i2 == m2 - 1 || (n == 3 && (i3 == 0 || i3 == m3 - 1));
    xm[t] = dr ? T(0) : x[t];
  }
}

template <int FORM, int Q, typename T>
static void launch_mf_eval(const KInterp<T>& ip, const FillGeom& g, bool stage, dim3 grid, size_t lds,
                           const int4* dsl, const double* coef, T* band, hipStream_t s) {
  if (g.npen * 2 * ip.Sd[0] > kChunk)
    hipLaunchKernelGGL((fill_fast_kernel<3, FORM, Q, T, true, 2, true>), grid, dim3(kChunk), lds, s, ip, g, dsl, coef,
                       band);
  else if (stage)
    hipLaunchKernelGGL((fill_fast_kernel<3, FORM, Q, T, true, 1, true>), grid, dim3(kChunk), lds, s, ip, g, dsl, coef,
                       band);
  else
    hipLaunchKernelGGL((fill_fast_kernel<3, FORM, Q, T, false, 1, true>), grid, dim3(kChunk), lds, s, ip, g, dsl,
                       coef, band);
}

template <int FORM, int P, typename T>
static void launch_mf_copy(const KInterp<T>& ip, const Dims& d, const int* rows, int nrows, T* band, const T* x, T* y,
                           hipStream_t s) {
  if (nrows == 0) return;
  dim3 grid((nrows + 63) / 64, d.batch);
  hipLaunchKernelGGL((copy_kernel<3, FORM, P, T, true>), grid, dim3(64 * kCopyWaves), 0, s, ip, d.m[0], d.m[1], d.ld,
                     d.S, rows, nrows, band, x, y, d.N);
}

// y = A~ x, matrix-free for the analysis-domain rows (3-D, fast chunked
// fill): the evaluation of those rows from the spline coefficients, their
// exact partner entries from the stored rows, and the stored rows
// themselves.  xm: scratch of N*batch values, used when dirichlet is set and
// x_masked is false.
template <typename T>
hipError_t launch_apply_mf(const KInterp<T>& ip, int form, const Dims& d, const int* chunks, int nchunks,
                           int chunk_rows, int n2max, int n3max, const int4* dsl, const double* coef, const T* band,
                           const int* crow, int ncopy, const int* brow, int nbrow, const T* x, T* y, T* xm,
                           int dirichlet, bool x_masked, hipStream_t s) {
  if (d.n != 3 || chunk_rows != kChunk * kRows) return hipErrorInvalidValue;
  FillGeom g;
  g.n = d.n;
  g.P = d.p;
  g.m1 = d.m[0];
  g.m2 = d.m[1];
  g.m3 = d.m[2];
  g.N = d.N;
  g.ld = d.ld;
  g.S = d.S;
  g.npen = fill_npen(d, chunk_rows);
  g.nchunks = nchunks;
  g.chunks = chunks;
  g.n2max = n2max;
  g.n3max = n3max;
  // as in launch_fill: two tasks per thread need staging (capped blocks)
  const bool two = g.npen * 2 * ip.Sd[0] > kChunk;
  if (g.npen * 2 * ip.Sd[0] > 2 * kChunk) return hipErrorInvalidValue;
  const int blk = two ? std::min(n2max * n3max * ip.Sd[0], kStage * kChunk) : n2max * n3max * ip.Sd[0];
  const bool stage = (two || blk <= kStage * kChunk) && fill_lds_bytes<T>(ip, g.npen, d, blk) <= 160 * 1024;
  if (two && !stage) return hipErrorInvalidValue;
  const size_t lds = fill_lds_bytes<T>(ip, g.npen, d, stage ? blk : 0);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const T* xin = x;
  if (dirichlet && !x_masked) {
    const int64_t total = d.N * d.batch;
    hipLaunchKernelGGL((mask_dirichlet_kernel<T>), dim3(int(std::min<int64_t>((total + 255) / 256, 8192))), dim3(256),
                       0, s, d.n, d.m[0], d.m[1], d.m[2], d.N, d.batch, x, xm);
    xin = xm;
  }
  g.ax = xin;
  g.ay = y;
  T* bandw = const_cast<T*>(band);  // read only in the apply modes
  {
    PhaseTimer t("mf_domain_rows", s);
    if (nchunks > 0) {
      dim3 grid(nchunks, d.batch);
      const bool mass = form == IGS_MASS;
      switch (ip.q) {
        case 1: mass ? launch_mf_eval<IGS_MASS, 1, T>(ip, g, stage, grid, lds, dsl, coef, bandw, s) : launch_mf_eval<IGS_STIFFNESS, 1, T>(ip, g, stage, grid, lds, dsl, coef, bandw, s); break;
        case 2: mass ? launch_mf_eval<IGS_MASS, 2, T>(ip, g, stage, grid, lds, dsl, coef, bandw, s) : launch_mf_eval<IGS_STIFFNESS, 2, T>(ip, g, stage, grid, lds, dsl, coef, bandw, s); break;
        case 3: mass ? launch_mf_eval<IGS_MASS, 3, T>(ip, g, stage, grid, lds, dsl, coef, bandw, s) : launch_mf_eval<IGS_STIFFNESS, 3, T>(ip, g, stage, grid, lds, dsl, coef, bandw, s); break;
        case 4: mass ? launch_mf_eval<IGS_MASS, 4, T>(ip, g, stage, grid, lds, dsl, coef, bandw, s) : launch_mf_eval<IGS_STIFFNESS, 4, T>(ip, g, stage, grid, lds, dsl, coef, bandw, s); break;
        default: mass ? launch_mf_eval<IGS_MASS, 5, T>(ip, g, stage, grid, lds, dsl, coef, bandw, s) : launch_mf_eval<IGS_STIFFNESS, 5, T>(ip, g, stage, grid, lds, dsl, coef, bandw, s); break;
      }
    }
  }
  {
    PhaseTimer t("mf_copied_entries", s);
    const bool mass = form == IGS_MASS;
    switch (d.p) {
      case 1: mass ? launch_mf_copy<IGS_MASS, 1, T>(ip, d, crow, ncopy, bandw, xin, y, s) : launch_mf_copy<IGS_STIFFNESS, 1, T>(ip, d, crow, ncopy, bandw, xin, y, s); break;
      case 2: mass ? launch_mf_copy<IGS_MASS, 2, T>(ip, d, crow, ncopy, bandw, xin, y, s) : launch_mf_copy<IGS_STIFFNESS, 2, T>(ip, d, crow, ncopy, bandw, xin, y, s); break;
      case 3: mass ? launch_mf_copy<IGS_MASS, 3, T>(ip, d, crow, ncopy, bandw, xin, y, s) : launch_mf_copy<IGS_STIFFNESS, 3, T>(ip, d, crow, ncopy, bandw, xin, y, s); break;
      default: mass ? launch_mf_copy<IGS_MASS, 4, T>(ip, d, crow, ncopy, bandw, xin, y, s) : launch_mf_copy<IGS_STIFFNESS, 4, T>(ip, d, crow, ncopy, bandw, xin, y, s); break;
    }
  }
  {
    PhaseTimer t("mf_stored_rows", s);
    if (nbrow > 0)
      hipLaunchKernelGGL((rows_spmv_kernel<T>), dim3((nbrow + 255) / 256, d.batch), dim3(256), 0, s, d.n, d.p, d.m[0],
                         d.m[1], d.m[2], d.N, d.ld, d.S, brow, nbrow, band, xin, y, dirichlet);
  }
  return hipGetLastError();
}
template hipError_t launch_apply_mf<double>(const KInterp<double>&, int, const Dims&, const int*, int, int, int, int,
                                            const int4*, const double*, const double*, const int*, int, const int*,
                                            int, const double*, double*, double*, int, bool, hipStream_t);

// rows outside the analysis domain, in flat order (the rows the matrix-free
// apply multiplies from the band)
std::vector<int> boundary_rows(const Dims& d) {
  std::vector<int> out;
  const int p = d.p;
  for (int64_t i = 0; i < d.N; ++i) {
    const int i1 = int(i % d.m[0]), i2 = int((i / d.m[0]) % d.m[1]);
    const int i3 = d.n == 3 ? int(i / (int64_t(d.m[0]) * d.m[1])) : 2 * p;
    const bool in = i1 >= 2 * p && i1 <= d.m[0] - 2 * p - 1 && i2 >= 2 * p && i2 <= d.m[1] - 2 * p - 1 &&
                    (d.n == 2 || (i3 >= 2 * p && i3 <= d.m[2] - 2 * p - 1));
    if (!in) out.push_back(int(i));
  }
  return out;
}

// analysis-domain rows within p-1 of the domain's edge in some direction: the
// rows whose stencil reaches outside the analysis domain, in flat order
std::vector<int> copy_rows(const Dims& d, int c) {
  const int p = d.p;
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int k = 0; k < d.n; ++k) {
    lo[k] = c;
    hi[k] = d.m[k] - c - 1;
  }
  auto edge = [&](int k, int i) { return k < d.n && (i < lo[k] + p || i > hi[k] - p); };
  std::vector<int> out;
  for (int i3 = lo[2]; i3 <= hi[2]; ++i3)
    for (int i2 = lo[1]; i2 <= hi[1]; ++i2) {
      const int64_t base = int64_t(d.m[0]) * (i2 + int64_t(d.m[1]) * i3);
      if (edge(1, i2) || edge(2, i3)) {
        for (int i1 = lo[0]; i1 <= hi[0]; ++i1) out.push_back(int(base + i1));
      } else {
        // only the rows near the two ends of the pencil's domain range
        for (int i1 = lo[0]; i1 <= hi[0]; ++i1) {
          if (!edge(0, i1)) i1 = std::max(i1, hi[0] - p + 1);
          if (i1 <= hi[0]) out.push_back(int(base + i1));
        }
      }
    }
  return out;
}

template <int ND, int FORM, int P, typename T, bool FIXUP>
static void launch_copy_pp(const KInterp<T>& ip, const Dims& d, const int* rows, int nrows, T* band, hipStream_t s) {
  dim3 grid((nrows + 63) / 64, d.batch);
  hipLaunchKernelGGL((copy_kernel<ND, FORM, P, T, false, FIXUP>), grid, dim3(64 * kCopyWaves), 0, s, ip, d.m[0],
                     d.m[1], d.ld, d.S, rows, nrows, band, static_cast<const T*>(nullptr), static_cast<T*>(nullptr),
                     int64_t(0));
}

template <int ND, int FORM, typename T, bool FIXUP = false>
static void launch_copy_p(const KInterp<T>& ip, const Dims& d, const int* rows, int nrows, T* band, hipStream_t s) {
  switch (d.p) {
    case 1: launch_copy_pp<ND, FORM, 1, T, FIXUP>(ip, d, rows, nrows, band, s); break;
    case 2: launch_copy_pp<ND, FORM, 2, T, FIXUP>(ip, d, rows, nrows, band, s); break;
    case 3: launch_copy_pp<ND, FORM, 3, T, FIXUP>(ip, d, rows, nrows, band, s); break;
    default: launch_copy_pp<ND, FORM, 4, T, FIXUP>(ip, d, rows, nrows, band, s); break;
  }
}

// 3-D: the boundary-row quadrature has stored the copied entries (transposed
// stores, KProblem::transpose), so only the stiffness diagonal is fixed up.
// 2-D: the copy kernel proper.
template <typename T>
hipError_t launch_copy(const KInterp<T>& ip, int form, const Dims& d, const int* rows, int nrows, T* band,
                       hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  if (d.n == 3) {
    if (form == IGS_STIFFNESS) launch_copy_p<3, IGS_STIFFNESS, T, true>(ip, d, rows, nrows, band, s);
  } else {
    if (form == IGS_MASS)
      launch_copy_p<2, IGS_MASS, T>(ip, d, rows, nrows, band, s);
    else
      launch_copy_p<2, IGS_STIFFNESS, T>(ip, d, rows, nrows, band, s);
  }
  return hipGetLastError();
}

template hipError_t launch_copy<double>(const KInterp<double>&, int, const Dims&, const int*, int, double*,
                                        hipStream_t);
template hipError_t launch_copy<float>(const KInterp<float>&, int, const Dims&, const int*, int, float*, hipStream_t);

template <typename T>
hipError_t launch_zero_pad(T* band, int64_t N, int64_t ld, int slots_total, hipStream_t s) {
  if (ld == N) return hipSuccess;
  int64_t total = (ld - N) * slots_total;
  int blocks = int(std::min<int64_t>((total + 255) / 256, 4096));
  hipLaunchKernelGGL((zero_pad_kernel<T>), dim3(blocks), dim3(256), 0, s, band, N, ld, slots_total);
  return hipGetLastError();
}

template hipError_t launch_zero_pad<double>(double*, int64_t, int64_t, int, hipStream_t);
template hipError_t launch_zero_pad<float>(float*, int64_t, int64_t, int, hipStream_t);

}  // namespace igs
