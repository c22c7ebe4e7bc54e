// Banded SpMV and conjugate gradients on the stencil-major band.
//
// y_i = sum_s band[s][i] x[i + off_s], off_s = delta_1 + m1 delta_2 + m1 m2
// delta_3 (the colex offset of the slot's delta).  A thread owns two
// consecutive rows and walks the slots: for a fixed slot the lanes of a wave
// read consecutive band entries (one 8- or 16-byte load per slot for the
// pair) and consecutive x entries, so both streams are coalesced; the band is
// streamed once (non-temporal), x stays in L2 (FP64) or is staged in LDS per
// (delta2, delta3) run (FP32).  Entries whose column leaves the index box are
// stored as 0, so the column index is only clamped into [0, N) to keep the
// read in bounds.  Workgroups are remapped so that each XCD walks a contiguous
// range of rows (its L2 then holds the x halo).
//
// CG (Dirichlet-restricted, Sec. 6, eq. BlockSystem with u_D = 0) keeps every
// vector zero on the Dirichlet dofs, so the restriction reduces to zeroing
// those rows of A p.  Reductions are two-stage and deterministic (per-block
// partials, then one block in a fixed order): no floating-point atomics.
#include <algorithm>
#include <cmath>
#include <functional>
#include <vector>

#include "igs_internal.h"
#include "profile.h"

namespace igs {

constexpr int kSpmvBlock = 256;
constexpr int kRedBlock = 256;

struct SpmvGeom {
  int n, p, W, S;
  int m[3];
  int64_t N, ld;
};

__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  // blocks are dealt round-robin to the 8 XCDs; give XCD x the logical range
  // [x*per, (x+1)*per) so neighbouring rows share an L2
  const int per = nblk / 8;
  if (per == 0 || bid >= per * 8) return bid;
  return (bid % 8) * per + bid / 8;
}

__device__ __forceinline__ bool on_dirichlet(const SpmvGeom& g, int64_t i) {
  const int i1 = int(i % g.m[0]);
  int64_t r = i / g.m[0];
  const int i2 = int(r % g.m[1]);
  const int i3 = int(r / g.m[1]);
  bool d = (i1 == 0) | (i1 == g.m[0] - 1) | (i2 == 0) | (i2 == g.m[1] - 1);
  if (g.n == 3) d |= (i3 == 0) | (i3 == g.m[2] - 1);
  return d;
}

// part[k0] + part[k0 + kRedBlock] + ... (k < n), added in that order; the
// loads go out eight at a time
__device__ __forceinline__ double strided_sum(const double* __restrict__ part, int k0, int n) {
  double s = 0.0;
#pragma unroll 8
  for (int k = k0; k < n; k += kRedBlock) s += part[k];
  return s;
}

// Per-problem scalars, kept on the device between kernels.
struct CgScalars {
  double rr;      // r^T r
  double alpha, beta;
  double tol2;    // stop when rr <= tol2
  double rr_ref;  // residual replacement: |f - A u|^2 at the last replacement
  int done;       // converged or broken down
  int breakdown;
  int iters;
  int replace;    // residual replacement due after this iteration
  int nrep;       // replacements made
  int pad;
  // fused scalars: r^T r of iterations k (rrv[k & 1]) and k + 1
  // (rrv[(k + 1) & 1]); the kernels of iteration k read one and write the other
  double rrv[2];
  // fused residual replacement: what launch slot k does (kSlotStep or
  // kSlotReplace), in kind[k & 1]
  int kind[2];
};
constexpr int kSlotStep = 0, kSlotReplace = 1;
// residual replacement: when the FP32 recursive |r|^2 has fallen by kReplace^2
constexpr double kReplace = 0.1;

// Banded SpMV for both band types.  A thread owns R consecutive rows, so one
// 16-byte band load per slot serves all of them (R = 2 for FP64, 4 for FP32):
// a one-row kernel would issue four (FP32) or two (FP64) times the
// vector-memory instructions and be bound by them rather than by HBM.  For
// each (delta2, delta3) run the thread needs the 2P+R values x[r0 + off - P ..]
// that its rows' delta1 windows cover.  FP64 reads them from L2; FP32 stages
// the block's windows in LDS one delta3 plane at a time (W windows of
// kSpmvBlock + 2P values, one per delta2), which keeps the LDS per block small
// enough for many blocks per CU.  The rows start at a multiple of R and ld is a
// multiple of 64, so the band load is aligned and stays inside the slot; row
// indices past N read padding and are not stored.  Modes:
//   0  y = A x (Dirichlet rows 0 when mask is set)
//   1  CG product: w = A r (Dirichlet rows 0), then on the thread's own rows
//      p = r + beta p and q = w + beta q, which is A p by linearity, so the
//      direction update needs neither a pass of its own nor the halo of p;
//      finished problems skipped; per-block partials of p^T q
//   2  (FP64) r = f - A u, Dirichlet rows 0, partials of r^T r and f^T f
//   3  (FP64) r32 = float(f - A u) on problems with a residual replacement
//      due, partials of r^T r
// Sum over a workgroup of NT threads (a multiple of 64), returned to every
// thread: a butterfly within each wavefront (lane exchanges, no LDS), then the
// wavefronts' sums added in wavefront order.  Fixed order: deterministic.
template <int NT>
__device__ __forceinline__ double block_sum_n(double v) {
  static_assert(NT % 64 == 0, "whole wavefronts");
  __shared__ double red[NT / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int k = 1; k < NT / 64; ++k) s += red[k];
  __syncthreads();  // red is reused by a following call
  return s;
}

template <typename T, int R>
struct VecR {
  typedef T v __attribute__((ext_vector_type(R)));
};
template <typename T>
struct Pair2 {
  typedef T v __attribute__((ext_vector_type(2)));
};

template <typename T>
struct SpmvShape {
  static constexpr int R = 16 / sizeof(T);   // rows per thread: one 16-byte band load per slot
  static constexpr bool STAGE = sizeof(T) == 4;
  static constexpr int NT = kSpmvBlock / R;  // threads per block
};

// Sum of part[b][0..n) in exactly the order of a kRedBlock-thread reduction
// (strided per-thread sums, the wavefront butterfly, wavefront sums in order),
// computed by a workgroup of NT threads (a multiple of 64): thread t plays the
// virtual threads t + j NT below kRedBlock.  Any NT therefore gives the same
// bits as sum_parts below.  In two halves: load() issues the loads (no
// barrier, so a kernel can start it early and let other loads overlap it),
// combine() adds up across the workgroup.
template <int NT>
struct PartSum {
  static constexpr int V = (kRedBlock + NT - 1) / NT;
  static_assert(NT % 64 == 0, "whole wavefronts");
  double v[V];
  __device__ __forceinline__ void load(const double* __restrict__ part, int b, int n) {
    const double* pb = part + size_t(b) * n;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int vt = threadIdx.x + j * NT;  // the same validity across a wavefront
      v[j] = vt < kRedBlock ? strided_sum(pb, vt, n) : 0.0;
    }
  }
  __device__ __forceinline__ double combine() {
    __shared__ double red[kRedBlock / 64];
#pragma unroll
    for (int j = 0; j < V; ++j)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_xor(v[j], off, 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const int vt = threadIdx.x + j * NT;
        if (vt < kRedBlock) red[vt >> 6] = v[j];
      }
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int k = 1; k < kRedBlock / 64; ++k) s += red[k];
    __syncthreads();
    return s;
  }
};

// r^T r after `it` completed CG steps: record it and decide convergence
__device__ __forceinline__ void record_rr(CgScalars& c, double s, int it) {
  c.rrv[it & 1] = s;
  c.iters = it;
  if (!isfinite(s)) {
    c.done = 1;
    c.breakdown = 1;
  } else if (s <= c.tol2) {
    c.done = 1;
  }
}

// Direction update of the CG product (mode 1): p = r + beta p, q = w + beta q.
//   bsrc 0  first step: p = r, q = w
//   bsrc 1  beta from the per-problem scalars
//   bsrc 2  plain CG with fused scalars: every workgroup sums the previous
//           step's partials of r^T r (rrp) itself, beta = rr_new / rr_old, and
//           workgroup 0 records rr_new (record_rr with `it`)
//   bsrc 3  FP32 CG with FP64 residual replacement, fused scalars: launch
//           slot `it` decides its role (replace_slot)
template <typename T>
struct CgDir {
  T* p;
  const double* rrp;   // partials of r^T r after the previous step
  const double* rrp2;  // bsrc 3: partials of |f - A u|^2 of the previous slot's replacement
  int it;
  int bsrc;
};

// FP32 CG with FP64 residual replacement, fused scalars (at most kFuseParts
// partials per problem).  Every launch slot runs the product and the update
// kernel; from what slot it - 1 left, the product decides whether slot it is
// a step (the product runs, then the update) or a replacement (only the
// update kernel runs, as the FP64 residual, giving r and rr_ref).  After a
// step: |r|^2 from its partials; non-finite -> breakdown; fallen by kReplace^2
// since the last replacement, or at the tolerance -> a replacement slot;
// otherwise beta = |r|^2 / rr.  After a replacement: |r|^2 of the FP64
// residual is the new rr and rr_ref, converged when at the tolerance, else
// beta = |r|^2 / rr (rr of the step before the replacement).  Every workgroup
// computes the same sums and decisions; workgroup 0 (rec) records them in the
// slots of parity it & 1, which no workgroup of this kernel reads.  ps holds
// the loaded partials (cg_product_load).  Returns false when the slot runs no
// product.
template <int NT>
__device__ __forceinline__ bool replace_slot(CgScalars& c, PartSum<NT>& ps, int it, bool rec, double* beta) {
  const int cur = it & 1, prv = cur ^ 1;
  const double rr_old = c.rrv[prv];
  if (c.kind[prv] == kSlotStep) {
    const double s = ps.combine();
    const bool bad = !isfinite(s);
    const bool rep = !bad && (s <= kReplace * kReplace * c.rr_ref || s <= c.tol2);
    if (rec) {
      if (bad) {
        c.done = 1;
        c.breakdown = 1;
      } else if (rep) {
        c.kind[cur] = kSlotReplace;
        c.rrv[cur] = rr_old;
      } else {
        c.kind[cur] = kSlotStep;
        c.rrv[cur] = s;
        c.iters += 1;
      }
    }
    if (bad || rep) return false;
    *beta = s / rr_old;
    return true;
  }
  const double s = ps.combine();
  const bool bad = !isfinite(s);
  const bool conv = !bad && s <= c.tol2;
  if (rec) {
    c.nrep += 1;
    c.iters += 1;
    if (bad) {
      c.done = 1;
      c.breakdown = 1;
    } else {
      c.rr_ref = s;
      c.rrv[cur] = s;
      c.kind[cur] = kSlotStep;
      if (conv) c.done = 1;
    }
  }
  if (bad || conv) return false;
  *beta = s / rr_old;
  return true;
}

// The partials a CG product workgroup (mode 1, see CgDir) of NT threads
// reduces for its direction-update scalar, loaded at its start.
template <typename T, int NT>
__device__ __forceinline__ void cg_product_load(const CgScalars* sc, const CgDir<T>& cd, int b, int nparts,
                                                PartSum<NT>& ps) {
  if (cd.bsrc == 2) ps.load(cd.rrp, b, nparts);
  if (cd.bsrc == 3) ps.load(sc[b].kind[(cd.it - 1) & 1] == kSlotStep ? cd.rrp : cd.rrp2, b, nparts);
}

// The direction-update scalar itself, from the loaded partials; rec: the
// workgroup that records the scalars.  False when the workgroup has nothing
// to do (the problem has finished, or the slot is a replacement).
template <typename T, int NT>
__device__ __forceinline__ bool cg_product_beta(CgScalars* sc, const CgDir<T>& cd, int b, bool rec, PartSum<NT>& ps,
                                                T* beta) {
  *beta = T(0);
  if (cd.bsrc == 2) {
    const double s = ps.combine();
    const double rr_old = sc[b].rrv[(cd.it - 1) & 1];
    const bool stop = !isfinite(s) || s <= sc[b].tol2;  // the same in every workgroup
    if (rec) record_rr(sc[b], s, cd.it);
    if (stop) return false;
    *beta = T(s / rr_old);
  } else if (cd.bsrc == 1) {
    *beta = T(sc[b].beta);
  } else if (cd.bsrc == 3) {
    double bt = 0.0;
    if (!replace_slot<NT>(sc[b], ps, cd.it, rec, &bt)) return false;
    *beta = T(bt);
  }
  return true;
}

template <typename T, int P, int ND, int MODE, bool STREAM>
__global__ void __launch_bounds__(SpmvShape<T>::NT)
    spmv_band_kernel(SpmvGeom g, const T* __restrict__ band, const T* __restrict__ x, const double* __restrict__ f,
                     T* __restrict__ y, float* __restrict__ y32, int mask, CgScalars* __restrict__ sc,
                     double* __restrict__ part, double* __restrict__ part2, CgDir<T> cd) {
  static_assert(MODE < 2 || sizeof(T) == 8, "residual modes take the FP64 band");
  constexpr int R = SpmvShape<T>::R, NT = SpmvShape<T>::NT;
  constexpr bool STAGE = SpmvShape<T>::STAGE;
  typedef typename VecR<T, R>::v VT;
  typedef typename Pair2<T>::v PT;
  constexpr int W = 2 * P + 1;
  constexpr int NZ = ND == 3 ? W : 1;        // delta3 planes
  constexpr int NX = 2 * P + R;              // x values per run and thread
  constexpr int XW = kSpmvBlock + 2 * P;     // staged window length
  constexpr int XP = (XW + 3) & ~3;          // LDS pitch (elements)
  __shared__ __align__(16) T xs[STAGE ? W * XP : 1];
  const int b = blockIdx.y;
  if (MODE == 1 && sc[b].done) return;
  if (MODE == 3 && (sc[b].done || !sc[b].replace)) return;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t i0 = int64_t(lb) * kSpmvBlock;
  const int tid = threadIdx.x;
  const int64_t r0 = i0 + R * tid;
  // mode 1: the direction-update scalar before the band loop (after it, the
  // staged FP32 kernel needs more registers than three wavefronts per SIMD
  // allow; spmv2_kernel, the 2D product, overlaps its reduction instead)
  T beta = T(0);
  if constexpr (MODE == 1) {
    PartSum<NT> ps;
    cg_product_load<T, NT>(sc, cd, b, gridDim.x, ps);
    if (!cg_product_beta<T, NT>(sc, cd, b, lb == 0 && tid == 0, ps, &beta)) return;
  }
  const T* xb = x + size_t(b) * g.N;
  const T* bb = band + size_t(b) * g.S * g.ld;
  const int64_t m1 = g.m[0], m12 = int64_t(g.m[0]) * g.m[1];
  T acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) acc[q] = T(0);
  // mode 1: the thread's rows of r, p and q; for FP64 loaded before the band
  // loop so that their latency hides behind it (FP32: after it, since the
  // early loads cost the staged kernel its occupancy)
  constexpr bool PREF = MODE == 1 && sizeof(T) == 8;
  T rown[R], pown[R], qown[R];
  auto load_own = [&]() {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t i = r0 + q < g.N ? r0 + q : g.N - 1;
      const size_t k0 = size_t(b) * g.N + i;
      rown[q] = xb[i];
      pown[q] = cd.bsrc == 0 ? T(0) : cd.p[k0];
      qown[q] = cd.bsrc == 0 ? T(0) : y[k0];
    }
  };
  if constexpr (PREF) load_own();
  for (int z = 0; z < NZ; ++z) {
    const int64_t o3 = ND == 3 ? (z - P) * m12 : 0;
    if constexpr (STAGE) {
      // one window at a time: its loads go out together, then into LDS
      constexpr int NS = (XW + NT - 1) / NT;
      if (z > 0) __syncthreads();  // every thread is done with the previous plane
      for (int k = 0; k < W; ++k) {
        const int64_t base = i0 + (k - P) * m1 + o3 - P;
        T st[NS];
#pragma unroll
        for (int u = 0; u < NS; ++u) {
          const int t = tid + u * NT;
          const int64_t j = base + t;
          st[u] = (t < XW && j >= 0 && j < g.N) ? xb[j] : T(0);
        }
#pragma unroll
        for (int u = 0; u < NS; ++u)
          if (tid + u * NT < XW) xs[k * XP + tid + u * NT] = st[u];
      }
      __syncthreads();
    }
    if (r0 < g.N) {
#pragma unroll
      for (int k = 0; k < W; ++k) {
        T xw[NX];
        if constexpr (STAGE) {
          const PT* xp = reinterpret_cast<const PT*>(xs + k * XP + R * tid);
#pragma unroll
          for (int e = 0; e < NX / 2; ++e) {
            const PT v = xp[e];
            xw[2 * e] = v.x;
            xw[2 * e + 1] = v.y;
          }
        } else {
          // columns outside [0, N) carry zero band entries: clamp to stay in bounds
          const int64_t base = r0 + (k - P) * m1 + o3 - P;
#pragma unroll
          for (int e = 0; e < NX; ++e) {
            int64_t j = base + e;
            j = j < 0 ? 0 : (j >= g.N ? g.N - 1 : j);
            xw[e] = xb[j];
          }
        }
        // all W band loads of the run go out before their products
        const T* bk = bb + size_t(z * W + k) * W * g.ld + r0;
        VT bv[W];
#pragma unroll
        for (int d1 = 0; d1 < W; ++d1)
          bv[d1] = STREAM ? __builtin_nontemporal_load(reinterpret_cast<const VT*>(bk + size_t(d1) * g.ld))
                          : *reinterpret_cast<const VT*>(bk + size_t(d1) * g.ld);
#pragma unroll
        for (int d1 = 0; d1 < W; ++d1)
#pragma unroll
          for (int q = 0; q < R; ++q) acc[q] = fma(bv[d1][q], xw[d1 + q], acc[q]);
      }
    }
  }
  if constexpr (MODE == 1 && !PREF) load_own();
  double sa = 0.0, sf = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int64_t i = r0 + q;
    if (i >= g.N) break;
    const bool dir = on_dirichlet(g, i);
    const size_t k0 = size_t(b) * g.N + i;
    T o;
    double fv = 0.0;
    if (MODE == 0) {
      o = (mask && dir) ? T(0) : acc[q];
    } else if (MODE == 1) {
      const T w = dir ? T(0) : acc[q];
      T pn = rown[q];
      if (cd.bsrc == 0) {
        o = w;
      } else {
        pn = pn + beta * pown[q];
        o = w + beta * qown[q];
      }
      cd.p[k0] = pn;
      sa += double(pn) * double(o);
    } else {
      fv = dir ? 0.0 : f[k0];
      o = dir ? T(0) : T(fv - double(acc[q]));
    }
    if (MODE == 3)
      y32[k0] = float(o);
    else
      y[k0] = o;
    if (MODE >= 2) {
      sa += double(o) * double(o);
      sf += fv * fv;
    }
  }
  if (MODE == 0) return;
  const double a = block_sum_n<NT>(sa);
  if (MODE == 2) {
    const double c = block_sum_n<NT>(sf);
    if (threadIdx.x == 0) part2[size_t(b) * gridDim.x + lb] = c;
  }
  if (threadIdx.x == 0) part[size_t(b) * gridDim.x + lb] = a;
}

// 2D products (modes 0 and 1) with one wavefront per delta2 run.  A workgroup
// of W = 2P+1 wavefronts owns kSpmvBlock rows; wavefront k forms the partial
// sums of run k (delta2 = k - P) for all of them (4 rows per lane: W band
// loads of 4 values and 2P+4 values of x from L2 per lane), the partials meet
// in LDS, and the threads add them in run order and finish the rows (the
// epilogue of spmv_band_kernel; one row per thread, two for P = 1).  W times the wavefronts of
// spmv_band_kernel, each with a W times shorter load chain: on the small
// batches of 2D solves one wavefront per 256 rows left a few per SIMD and the
// products latency-bound.
template <typename T, int P, int MODE, bool STREAM>
__global__ void __launch_bounds__(64 * (2 * P + 1))
    spmv2_kernel(SpmvGeom g, const T* __restrict__ band, const T* __restrict__ x, T* __restrict__ y, int mask,
                 CgScalars* __restrict__ sc, double* __restrict__ part, CgDir<T> cd) {
  static_assert(MODE < 2, "products only");
  constexpr int W = 2 * P + 1, NT = 64 * W, R = 4, NX = 2 * P + R;
  typedef typename VecR<T, R>::v VT;
  __shared__ __align__(16) T red[W * kSpmvBlock];
  const int b = blockIdx.y;
  if (MODE == 1 && sc[b].done) return;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t i0 = int64_t(lb) * kSpmvBlock;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const T* xb = x + size_t(b) * g.N;
  // mode 1: the partials of the direction-update scalar, loaded now and added
  // up after the band loop
  PartSum<NT> ps;
  if constexpr (MODE == 1) cg_product_load<T, NT>(sc, cd, b, gridDim.x, ps);
  // the rows this thread finishes (t = tid + f NT below kSpmvBlock; FR = 2 for
  // P = 1, whose workgroup has 192 threads), and (mode 1) their r, p and q,
  // loaded early
  constexpr int FR = (kSpmvBlock + NT - 1) / NT;
  T rown[FR], pown[FR], qown[FR];
#pragma unroll
  for (int f = 0; f < FR; ++f) {
    const int t = tid + f * NT;
    const int64_t io = i0 + t;
    rown[f] = pown[f] = qown[f] = T(0);
    if (MODE == 1 && t < kSpmvBlock && io < g.N) {
      const size_t ko = size_t(b) * g.N + io;
      rown[f] = xb[io];
      if (cd.bsrc != 0) {
        pown[f] = cd.p[ko];
        qown[f] = y[ko];
      }
    }
  }
  const int64_t r0 = i0 + R * lane;
  VT acc;
#pragma unroll
  for (int q = 0; q < R; ++q) acc[q] = T(0);
  if (r0 < g.N) {
    // columns outside [0, N) carry zero band entries: clamp to stay in bounds
    const int64_t base = r0 + int64_t(wv - P) * g.m[0] - P;
    T xw[NX];
#pragma unroll
    for (int e = 0; e < NX; ++e) {
      int64_t j = base + e;
      j = j < 0 ? 0 : (j >= g.N ? g.N - 1 : j);
      xw[e] = xb[j];
    }
    const T* bk = band + size_t(b) * g.S * g.ld + size_t(wv) * W * g.ld + r0;
    VT bv[W];
#pragma unroll
    for (int d1 = 0; d1 < W; ++d1)
      bv[d1] = STREAM ? __builtin_nontemporal_load(reinterpret_cast<const VT*>(bk + size_t(d1) * g.ld))
                      : *reinterpret_cast<const VT*>(bk + size_t(d1) * g.ld);
#pragma unroll
    for (int d1 = 0; d1 < W; ++d1)
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] = fma(bv[d1][q], xw[d1 + q], acc[q]);
  }
  *reinterpret_cast<VT*>(red + wv * kSpmvBlock + R * lane) = acc;
  __syncthreads();
  // the scalars after the band loop (nothing is written before this point, so
  // a slot without a product only loses its reads): the latency of their
  // reduction then overlaps the band loads
  T beta = T(0);
  if constexpr (MODE == 1)
    if (!cg_product_beta<T, NT>(sc, cd, b, lb == 0 && tid == 0, ps, &beta)) return;
  double sa = 0.0;
#pragma unroll
  for (int f = 0; f < FR; ++f) {
    const int t = tid + f * NT;
    const int64_t io = i0 + t;
    if (t >= kSpmvBlock || io >= g.N) continue;
    const size_t ko = size_t(b) * g.N + io;
    T a = red[t];
#pragma unroll
    for (int k = 1; k < W; ++k) a += red[k * kSpmvBlock + t];
    const bool dir = on_dirichlet(g, io);
    if (MODE == 0) {
      y[ko] = (mask && dir) ? T(0) : a;
    } else {
      const T w = dir ? T(0) : a;
      T pn = rown[f], o = w;
      if (cd.bsrc != 0) {
        pn = rown[f] + beta * pown[f];
        o = w + beta * qown[f];
      }
      cd.p[ko] = pn;
      y[ko] = o;
      sa += double(pn) * double(o);
    }
  }
  if constexpr (MODE == 1) {
    const double a = block_sum_n<NT>(sa);
    if (tid == 0) part[size_t(b) * gridDim.x + lb] = a;
  }
}

// Bands of at most this many bytes (all problems of a call) are read with
// ordinary loads, so that they stay in the 256 MiB last-level cache between the
// products of a solve; larger ones stream past it with non-temporal loads,
// which keeps the vectors cached (2D p=3 batch-8, 210 MB FP64: product 38.0 ->
// 33.1 us, CG 35.6 -> 30.6 ms; 3D p=3 128^3, 6.2 GB: ordinary loads 1.06
// instead of 0.98 ms).  The residual modes always stream.
constexpr size_t kResidentBand = size_t(224) << 20;

template <typename T, int MODE>
static void launch_spmv_band(const SpmvGeom& g, int nblk, int batch, const T* band, const T* x, const double* f,
                             T* y, float* y32, int mask, CgScalars* sc, double* part, double* part2, hipStream_t s,
                             const CgDir<T>& cd = CgDir<T>{}) {
  const dim3 grid(nblk, batch), block(SpmvShape<T>::NT);
  const bool stream = MODE >= 2 || size_t(batch) * g.S * g.ld * sizeof(T) > kResidentBand;
#define IGS_SPMV(PP, NDD)                                                                                            \
  do {                                                                                                                \
    if (stream || MODE >= 2)                                                                                          \
      hipLaunchKernelGGL((spmv_band_kernel<T, PP, NDD, MODE, true>), grid, block, 0, s, g, band, x, f, y, y32, mask, \
                         sc, part, part2, cd);                                                                        \
    else                                                                                                              \
      hipLaunchKernelGGL((spmv_band_kernel<T, PP, NDD, MODE, MODE < 2 ? false : true>), grid, block, 0, s, g, band, \
                         x, f, y, y32, mask, sc, part, part2, cd);                                                    \
  } while (0)
  if (g.n == 3) {
    switch (g.p) {
      case 1: IGS_SPMV(1, 3); break;
      case 2: IGS_SPMV(2, 3); break;
      case 3: IGS_SPMV(3, 3); break;
      default: IGS_SPMV(4, 3); break;
    }
  } else if constexpr (MODE < 2) {
#define IGS_SPMV2(PP)                                                                                             \
  do {                                                                                                            \
    const dim3 blk2(64 * (2 * PP + 1));                                                                           \
    if (stream)                                                                                                   \
      hipLaunchKernelGGL((spmv2_kernel<T, PP, MODE, true>), grid, blk2, 0, s, g, band, x, y, mask, sc, part, cd);  \
    else                                                                                                          \
      hipLaunchKernelGGL((spmv2_kernel<T, PP, MODE, false>), grid, blk2, 0, s, g, band, x, y, mask, sc, part, cd); \
  } while (0)
    switch (g.p) {
      case 1: IGS_SPMV2(1); break;
      case 2: IGS_SPMV2(2); break;
      case 3: IGS_SPMV2(3); break;
      default: IGS_SPMV2(4); break;
    }
#undef IGS_SPMV2
  } else {
    switch (g.p) {
      case 1: IGS_SPMV(1, 2); break;
      case 2: IGS_SPMV(2, 2); break;
      case 3: IGS_SPMV(3, 2); break;
      default: IGS_SPMV(4, 2); break;
    }
  }
#undef IGS_SPMV
}

template <int MODE>
static void launch_spmv32(const SpmvGeom& g, int nblk, int batch, const float* band, const float* x, float* y,
                          int mask, CgScalars* sc, double* part, hipStream_t s) {
  launch_spmv_band<float, MODE>(g, nblk, batch, band, x, nullptr, y, nullptr, mask, sc, part, nullptr, s);
}

template <int MODE>
static void launch_spmv64(const SpmvGeom& g, int nblk, int batch, const double* band, const double* x,
                          const double* f, double* y, float* y32, int mask, CgScalars* sc, double* part,
                          double* part2, hipStream_t s) {
  launch_spmv_band<double, MODE>(g, nblk, batch, band, x, f, y, y32, mask, sc, part, part2, s);
}

// CG product (mode 1): from r, p = r + beta p and q = A r + beta q = A p in
// place (see CgDir), partials of p^T q
template <typename T>
static void launch_cg_product(const SpmvGeom& g, int nblk, int batch, const T* band, const T* r, const CgDir<T>& cd,
                              T* q, CgScalars* sc, double* pap, hipStream_t s) {
  launch_spmv_band<T, 1>(g, nblk, batch, band, r, nullptr, q, nullptr, 1, sc, pap, nullptr, s, cd);
}

// x with its Dirichlet dofs zeroed (the restriction of igs_apply)
template <typename T>
__global__ void mask_copy_kernel(SpmvGeom g, int batch, const T* __restrict__ x, T* __restrict__ y) {
  const int64_t total = g.N * batch;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x)
    y[t] = on_dirichlet(g, t % g.N) ? T(0) : x[t];
}

// --------------------------------------------------------------- CG state --


template <typename T>
__device__ __forceinline__ double block_sum(double v) {
  return block_sum_n<kRedBlock>(v);
}

// out[b] = sum of part[b][0..nblk) in a fixed order (one block per problem)
__global__ void __launch_bounds__(kRedBlock) reduce_kernel(const double* __restrict__ part, int nblk, double* out) {
  const int b = blockIdx.x;
  double s = strided_sum(part + size_t(b) * nblk, threadIdx.x, nblk);
  s = block_sum<double>(s);
  if (threadIdx.x == 0) out[b] = s;
}

// inner CG start: rhat = r / scale (type T), d = 0 (the first step's product
// takes p = rhat)
template <typename T>
__global__ void cg_init_kernel(int64_t N, int batch, const double* __restrict__ r, const double* __restrict__ scale,
                               T* __restrict__ rh, T* __restrict__ d) {
  const int64_t total = N * batch;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int b = int(t / N);
    const double s = scale[b];
    rh[t] = s > 0.0 ? T(r[t] / s) : T(0);
    d[t] = T(0);
  }
}

__global__ void cg_setup_kernel(int batch, const double* __restrict__ rr, const double* __restrict__ tol2,
                                const int* __restrict__ active, CgScalars* sc) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  CgScalars s;
  s.rr = rr[b];
  s.alpha = s.beta = 0.0;
  s.tol2 = tol2[b];
  s.done = (!active[b] || s.rr <= s.tol2) ? 1 : 0;
  s.breakdown = 0;
  s.iters = 0;
  s.rr_ref = s.rr;
  s.replace = 0;
  s.nrep = 0;
  s.pad = 0;
  s.kind[0] = s.kind[1] = kSlotStep;
  s.rrv[0] = s.rr;
  s.rrv[1] = 0.0;
  sc[b] = s;
}

// alpha = rr / (p^T A p)
__global__ void __launch_bounds__(kRedBlock) cg_alpha_kernel(const double* __restrict__ part, int nblk, CgScalars* sc) {
  const int b = blockIdx.x;
  if (sc[b].done) return;
  double s = 0.0;
  s += strided_sum(part + size_t(b) * nblk, threadIdx.x, nblk);
  s = block_sum<double>(s);
  if (threadIdx.x == 0) {
    if (!(s > 0.0) || !isfinite(s)) {
      sc[b].done = 1;
      sc[b].breakdown = 1;
      sc[b].alpha = 0.0;
    } else {
      sc[b].alpha = sc[b].rr / s;
    }
  }
}

// d += alpha p, r -= alpha q, partial r^T r
template <typename T>
__global__ void __launch_bounds__(kSpmvBlock)
    cg_update_kernel(int64_t N, const CgScalars* __restrict__ sc, const T* __restrict__ p, const T* __restrict__ q,
                     T* __restrict__ d, T* __restrict__ r, double* __restrict__ part) {
  const int b = blockIdx.y;
  if (sc[b].done) return;
  const T alpha = T(sc[b].alpha);
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t i = int64_t(lb) * kSpmvBlock + threadIdx.x;
  double v = 0.0;
  if (i < N) {
    const size_t k = size_t(b) * N + i;
    d[k] += alpha * p[k];
    const T rn = r[k] - alpha * q[k];
    r[k] = rn;
    v = double(rn) * double(rn);
  }
  v = block_sum<double>(v);
  if (threadIdx.x == 0) part[size_t(b) * gridDim.x + lb] = v;
}

// beta = rr_new / rr; convergence on the recursive residual
__global__ void __launch_bounds__(kRedBlock) cg_beta_kernel(const double* __restrict__ part, int nblk, CgScalars* sc) {
  const int b = blockIdx.x;
  if (sc[b].done) return;
  double s = 0.0;
  s += strided_sum(part + size_t(b) * nblk, threadIdx.x, nblk);
  s = block_sum<double>(s);
  if (threadIdx.x == 0) {
    sc[b].beta = s / sc[b].rr;
    sc[b].rr = s;
    sc[b].iters += 1;
    if (!isfinite(s)) {
      sc[b].done = 1;
      sc[b].breakdown = 1;
    } else if (s <= sc[b].tol2) {
      sc[b].done = 1;
    }
  }
}

// p = r + beta p
template <typename T>
__global__ void cg_pupdate_kernel(int64_t N, const CgScalars* __restrict__ sc, const T* __restrict__ r,
                                  T* __restrict__ p) {
  const int b = blockIdx.y;
  if (sc[b].done) return;
  const T beta = T(sc[b].beta);
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < N; i += int64_t(gridDim.x) * blockDim.x) {
    const size_t k = size_t(b) * N + i;
    p[k] = r[k] + beta * p[k];
  }
}

// Fused CG scalars, for problems with at most kFuseParts partial sums per
// problem (each workgroup reads all of them, so the cost grows with their
// square).  Every workgroup reduces the same per-block partial sums in the
// same order, so all of them hold the same scalar and none waits for another;
// only workgroup 0 records it.  Step k reads r^T r from rrv[k & 1]; the
// product of step k + 1 writes rrv[(k + 1) & 1].
constexpr int kFuseParts = 1024;
__device__ __forceinline__ double sum_parts(const double* __restrict__ part, int b, int nparts) {
  double s = 0.0;
  s += strided_sum(part + size_t(b) * nparts, threadIdx.x, nparts);
  return block_sum<double>(s);
}

// alpha = rr / (p^T A p); d += alpha p, r -= alpha q, partial r^T r
template <typename T>
__global__ void __launch_bounds__(kSpmvBlock)
    cg_step_kernel(int64_t N, int par, CgScalars* __restrict__ sc, const double* __restrict__ pap,
                   const T* __restrict__ p, const T* __restrict__ q, T* __restrict__ d, T* __restrict__ r,
                   double* __restrict__ part) {
  const int b = blockIdx.y;
  if (sc[b].done) return;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t i = int64_t(lb) * kSpmvBlock + threadIdx.x;
  const size_t k = size_t(b) * N + i;
  // the partials of p^T q and this row's vectors go out together
  PartSum<kSpmvBlock> ps;
  ps.load(pap, b, gridDim.x);
  T pv = T(0), qv = T(0), dv = T(0), rv = T(0);
  if (i < N) {
    pv = p[k];
    qv = q[k];
    dv = d[k];
    rv = r[k];
  }
  const double s = ps.combine();
  if (!(s > 0.0) || !isfinite(s)) {
    if (lb == 0 && threadIdx.x == 0) {
      sc[b].done = 1;
      sc[b].breakdown = 1;
    }
    return;
  }
  const T alpha = T(sc[b].rrv[par] / s);
  double v = 0.0;
  if (i < N) {
    d[k] = dv + alpha * pv;
    const T rn = rv - alpha * qv;
    r[k] = rn;
    v = double(rn) * double(rn);
  }
  v = block_sum<double>(v);
  if (threadIdx.x == 0) part[size_t(b) * gridDim.x + lb] = v;
}

// r^T r after `it` steps from the step's partials, recorded as the next
// step's product would record it (the same sum in the same order), so the
// host sees convergence at the end of a chunk of steps
__global__ void __launch_bounds__(kRedBlock) cg_rr_kernel(const double* __restrict__ rrp, int nparts,
                                                          CgScalars* sc, int it) {
  const int b = blockIdx.x;
  if (sc[b].done) return;
  const double s = sum_parts(rrp, b, nparts);
  if (threadIdx.x == 0) record_rr(sc[b], s, it);
}

// u += scale * d (FP64 update of the refinement)
template <typename T>
__global__ void axpy_update_kernel(int64_t N, int batch, const double* __restrict__ scale, const T* __restrict__ d,
                                   double* __restrict__ u) {
  const int64_t total = N * batch;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x)
    u[t] += scale[t / N] * double(d[t]);
}

// zero u on Dirichlet dofs
__global__ void zero_dirichlet_kernel(SpmvGeom g, int batch, double* __restrict__ u) {
  const int64_t total = g.N * batch;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x)
    if (on_dirichlet(g, t % g.N)) u[t] = 0.0;
}

// ----------------------------------------------------------------- host ----

static SpmvGeom make_geom(const Dims& d) {
  SpmvGeom g;
  g.n = d.n;
  g.p = d.p;
  g.W = d.W;
  g.S = d.S;
  for (int k = 0; k < 3; ++k) g.m[k] = d.m[k];
  g.N = d.N;
  g.ld = d.ld;
  return g;
}

static int grid_stride_blocks(int64_t total) { return int(std::min<int64_t>((total + 255) / 256, 8192)); }

#define HIP_OK(x)                              \
  do {                                         \
    if ((x) != hipSuccess) return IGS_ERR_HIP; \
  } while (0)

template <typename T>
igs_status launch_apply_t(const Dims& d, const T* band, const T* x, T* y, int dirichlet, hipStream_t s) {
  SpmvGeom g = make_geom(d);
  const int nblk = int((d.N + kSpmvBlock - 1) / kSpmvBlock);
  const T* xin = x;
  Arena ar;
  if (dirichlet) {
    igs_status st = ar.alloc(padded(sizeof(T) * d.N * d.batch), s);
    if (st != IGS_OK) return st;
    T* xm = ar.take<T>(size_t(d.N) * d.batch);
    hipLaunchKernelGGL((mask_copy_kernel<T>), dim3(grid_stride_blocks(d.N * d.batch)), dim3(256), 0, s, g, d.batch,
                       x, xm);
    xin = xm;
  }
  {
    PhaseTimer t("spmv", s);
    if constexpr (sizeof(T) == 4)
      launch_spmv32<0>(g, nblk, d.batch, band, xin, y, dirichlet, nullptr, nullptr, s);
    else
      launch_spmv64<0>(g, nblk, d.batch, band, xin, nullptr, y, nullptr, dirichlet, nullptr, nullptr, nullptr, s);
  }
  HIP_OK(hipGetLastError());
  return IGS_OK;
}

igs_status launch_apply(const Dims& d, int dtype, const void* band, const void* x, void* y, int dirichlet,
                        hipStream_t s) {
  if (dtype == IGS_F64)
    return launch_apply_t<double>(d, static_cast<const double*>(band), static_cast<const double*>(x),
                                  static_cast<double*>(y), dirichlet, s);
  return launch_apply_t<float>(d, static_cast<const float*>(band), static_cast<const float*>(x),
                               static_cast<float*>(y), dirichlet, s);
}

template <typename T>
__global__ void __launch_bounds__(kRedBlock)
    dot_kernel(int64_t N, const T* __restrict__ a, const T* __restrict__ c, double* __restrict__ part) {
  const int b = blockIdx.y;
  double v = 0.0;
  for (int64_t i = blockIdx.x * int64_t(kRedBlock) + threadIdx.x; i < N; i += int64_t(gridDim.x) * kRedBlock)
    v += double(a[size_t(b) * N + i]) * double(c[size_t(b) * N + i]);
  v = block_sum<double>(v);
  if (threadIdx.x == 0) part[size_t(b) * gridDim.x + blockIdx.x] = v;
}

struct SolveBufs {
  double* r64;
  double* part;
  double* part2;
  double* rr;
  double* ff;
  double* scale;
  double* tol2;
  int* active;
  CgScalars* sc;
};

// Number of CG steps to enqueue before the host next reads the scalars.  A
// read drains the stream, so the host reads rarely: from the decrease of r^T r
// since its previous read it extrapolates (at the geometric rate observed) the
// steps the slowest unfinished problem still needs to reach its tolerance, and
// enqueues that many (at least 8, at most four times the previous chunk; 32
// at first).  Steps enqueued after a problem has finished return at once.
class ChunkPlanner {
 public:
  // rr0: r^T r of each problem at step 0
  explicit ChunkPlanner(std::vector<double> rr0) : rr_(std::move(rr0)), it_(rr_.size(), 0) {}
  int first() const { return last_; }
  // after a read at step `it`; rr[b] the current r^T r of problem b
  int next(const std::vector<CgScalars>& sc, const std::vector<double>& rr, int it) {
    double need = 0.0;
    bool known = true;
    for (size_t b = 0; b < rr_.size(); ++b) {
      if (sc[b].done) continue;
      const double r1 = rr[b], r0 = rr_[b];
      const int dk = it - it_[b];
      if (!(r1 > 0.0) || !(r0 > 0.0) || dk <= 0 || !(r1 < r0)) {
        known = false;
      } else {
        const double rate = std::log(r1 / r0) / dk;  // < 0
        need = std::max(need, std::log(sc[b].tol2 / r1) / rate);
      }
      rr_[b] = r1;
      it_[b] = it;
    }
    int n = known ? int(std::ceil(need)) : 2 * last_;
    n = std::min(std::max(n, 8), 4 * last_);
    last_ = n;
    return n;
  }

 private:
  std::vector<double> rr_;
  std::vector<int> it_;
  int last_ = 32;
};

// One inner CG on A_T dhat = rhat, rhat = r / scale, from dhat = 0, to
// |rhat - A dhat| <= sqrt(tol2) (per problem), at most `budget` iterations.
// A step is the product kernel (A r, the direction update of p and q = A p,
// p^T q partials) and the update kernel (alpha, dhat and r, r^T r partials);
// with at most kFuseParts partials per problem each kernel sums them itself
// (two launches per step), else one-workgroup kernels compute alpha and beta
// between them.
template <typename T>
static igs_status inner_cg(const Dims& d, const T* band, const SolveBufs& sb, T* rh, T* p, T* q, T* dv, int budget,
                           std::vector<CgScalars>* host_sc, int* iters, hipStream_t s) {
  SpmvGeom g = make_geom(d);
  const int nblk = int((d.N + kSpmvBlock - 1) / kSpmvBlock);
  const int dblk = int(std::min<int64_t>((d.N + kRedBlock - 1) / kRedBlock, 1024));
  hipLaunchKernelGGL((cg_init_kernel<T>), dim3(grid_stride_blocks(d.N * d.batch)), dim3(256), 0, s, d.N, d.batch,
                     sb.r64, sb.scale, rh, dv);
  hipLaunchKernelGGL((dot_kernel<T>), dim3(dblk, d.batch), dim3(kRedBlock), 0, s, d.N, rh, rh, sb.part);
  hipLaunchKernelGGL(reduce_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, sb.part, dblk, sb.rr);
  hipLaunchKernelGGL(cg_setup_kernel, dim3(1), dim3(64), 0, s, d.batch, sb.rr, sb.tol2, sb.active, sb.sc);
  HIP_OK(hipGetLastError());
  const bool fused = nblk <= kFuseParts;
  // |rhat|^2 = 1 for the problems that iterate
  ChunkPlanner plan(std::vector<double>(d.batch, 1.0));
  std::vector<double> rrh(d.batch);
  int chunk = plan.first();
  int it = 0;
  while (it < budget) {
    const int k = std::min(chunk, budget - it);
    for (int j = 0; j < k; ++j, ++it) {
      const CgDir<T> cd{p, sb.part2, nullptr, it, it == 0 ? 0 : (fused ? 2 : 1)};
      {
        PhaseTimer t(sizeof(T) == 8 ? "cg_spmv_f64" : "cg_spmv_f32", s);
        launch_cg_product<T>(g, nblk, d.batch, band, rh, cd, q, sb.sc, sb.part, s);
      }
      PhaseTimer t("cg_vector_ops", s);
      if (fused) {
        hipLaunchKernelGGL((cg_step_kernel<T>), dim3(nblk, d.batch), dim3(kSpmvBlock), 0, s, d.N, it & 1, sb.sc,
                           sb.part, p, q, dv, rh, sb.part2);
      } else {
        hipLaunchKernelGGL(cg_alpha_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, sb.part, nblk, sb.sc);
        hipLaunchKernelGGL((cg_update_kernel<T>), dim3(nblk, d.batch), dim3(kSpmvBlock), 0, s, d.N, sb.sc, p, q,
                           dv, rh, sb.part2);
        hipLaunchKernelGGL(cg_beta_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, sb.part2, nblk, sb.sc);
      }
    }
    if (fused) hipLaunchKernelGGL(cg_rr_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, sb.part2, nblk, sb.sc, it);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(host_sc->data(), sb.sc, sizeof(CgScalars) * d.batch, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    bool all = true;
    for (int b = 0; b < d.batch; ++b) {
      all &= (*host_sc)[b].done != 0;
      rrh[b] = fused ? (*host_sc)[b].rrv[it & 1] : (*host_sc)[b].rr;
    }
    if (all) break;
    chunk = plan.next(*host_sc, rrh, it);
  }
  int mx = 0;
  for (int b = 0; b < d.batch; ++b) mx = std::max(mx, (*host_sc)[b].iters);
  *iters = mx;
  return IGS_OK;
}

template <typename T>
static igs_status refine_loop(const Dims& d, const double* band64, const T* bandT, const double* f, double* u,
                              double rtol, int maxit, double inner_rel, igs_cg_info* info, hipStream_t s) {
  SpmvGeom g = make_geom(d);
  const int nblk = int((d.N + kSpmvBlock - 1) / kSpmvBlock);
  const size_t NB = size_t(d.N) * d.batch;
  const size_t nb = size_t(d.batch);
  Arena ar;
  size_t bytes = padded(sizeof(double) * NB) + 2 * padded(sizeof(double) * nb * nblk) + 4 * padded(sizeof(double) * nb) +
                 padded(sizeof(int) * nb) + padded(sizeof(CgScalars) * nb) + 4 * padded(sizeof(T) * NB);
  igs_status st = ar.alloc(bytes, s);
  if (st != IGS_OK) return st;
  SolveBufs sb;
  sb.r64 = ar.take<double>(NB);
  sb.part = ar.take<double>(nb * nblk);
  sb.part2 = ar.take<double>(nb * nblk);
  sb.rr = ar.take<double>(nb);
  sb.ff = ar.take<double>(nb);
  sb.scale = ar.take<double>(nb);
  sb.tol2 = ar.take<double>(nb);
  sb.active = ar.take<int>(nb);
  sb.sc = ar.take<CgScalars>(nb);
  T* rh = ar.take<T>(NB);
  T* p = ar.take<T>(NB);
  T* q = ar.take<T>(NB);
  T* dv = ar.take<T>(NB);

  hipLaunchKernelGGL(zero_dirichlet_kernel, dim3(grid_stride_blocks(NB)), dim3(256), 0, s, g, d.batch, u);
  std::vector<double> rr(nb), ff(nb), scale(nb), tol2(nb);
  std::vector<int> active(nb);
  std::vector<CgScalars> hsc(nb);
  int total_iters = 0, outer = 0;
  bool breakdown = false;
  igs_status result = IGS_NOT_CONVERGED;
  double worst = 0.0;
  while (true) {
    {
      PhaseTimer t("residual_f64", s);
      launch_spmv64<2>(g, nblk, d.batch, band64, u, f, sb.r64, nullptr, 1, nullptr, sb.part, sb.part2, s);
    }
    hipLaunchKernelGGL(reduce_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, sb.part, nblk, sb.rr);
    hipLaunchKernelGGL(reduce_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, sb.part2, nblk, sb.ff);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(rr.data(), sb.rr, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(ff.data(), sb.ff, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    bool all = true;
    worst = 0.0;
    for (size_t b = 0; b < nb; ++b) {
      const double rel = ff[b] > 0.0 ? std::sqrt(rr[b] / ff[b]) : 0.0;
      if (!std::isfinite(rel)) {
        info->relres = rel;
        info->iterations = total_iters;
        info->outer_iterations = outer;
        info->status = IGS_BREAKDOWN;
        return IGS_BREAKDOWN;
      }
      worst = std::max(worst, rel);
      active[b] = rel > rtol;
      all &= !active[b];
      scale[b] = std::sqrt(rr[b]);
      // inner target relative to |rhat| = 1: enough to meet rtol with margin,
      // never tighter than the inner precision allows
      double t = active[b] ? 0.5 * rtol * std::sqrt(ff[b] / rr[b]) : 1.0;
      t = std::max(t, inner_rel);
      tol2[b] = t * t;
    }
    if (all) {
      result = IGS_OK;
      break;
    }
    if (total_iters >= maxit || (breakdown && outer > 0)) break;
    HIP_OK(hipMemcpyAsync(sb.scale, scale.data(), sizeof(double) * nb, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(sb.tol2, tol2.data(), sizeof(double) * nb, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(sb.active, active.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
    int it = 0;
    st = inner_cg<T>(d, bandT, sb, rh, p, q, dv, maxit - total_iters, &hsc, &it, s);
    if (st != IGS_OK) return st;
    for (size_t b = 0; b < nb; ++b) breakdown |= hsc[b].breakdown != 0;
    total_iters += it;
    ++outer;
    hipLaunchKernelGGL((axpy_update_kernel<T>), dim3(grid_stride_blocks(NB)), dim3(256), 0, s, d.N, d.batch,
                       sb.scale, dv, u);
    HIP_OK(hipGetLastError());
  }
  if (result != IGS_OK && breakdown) result = IGS_BREAKDOWN;
  info->iterations = total_iters;
  info->outer_iterations = outer;
  info->relres = worst;
  info->status = result;
  HIP_OK(hipStreamSynchronize(s));
  return result;
}

// ---------------------------------- FP32 CG with FP64 residual replacement --
//
// Mixed-precision CG that keeps its Krylov space: the iteration runs on the
// FP32 band with FP32 vectors, the solution u accumulates in FP64, and when
// the FP32 recursive residual has fallen by kReplace^2 since the last
// replacement (or claims convergence) it is replaced by the FP64 residual
// f - A64 u of the FP64 band.  Convergence is decided on those FP64 residuals
// only.  (An FP64 iterative refinement whose correction solves are not
// restarted: the search direction survives each correction.)

// r32 = float(r64) (the first step's product takes p = r32)
__global__ void rc_init_kernel(int64_t total, const double* __restrict__ r64, float* __restrict__ r32) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x)
    r32[t] = float(r64[t]);
}

// u += alpha p (FP64), r -= alpha q (FP32), partial |r|^2 (FP64 sums)
__global__ void __launch_bounds__(kSpmvBlock)
    rc_update_kernel(int64_t N, const CgScalars* __restrict__ sc, const float* __restrict__ p,
                     const float* __restrict__ q, double* __restrict__ u, float* __restrict__ r,
                     double* __restrict__ part) {
  const int b = blockIdx.y;
  if (sc[b].done) return;
  const double alpha = sc[b].alpha;
  const float af = float(alpha);
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t i = int64_t(lb) * kSpmvBlock + threadIdx.x;
  double v = 0.0;
  if (i < N) {
    const size_t k = size_t(b) * N + i;
    u[k] += alpha * double(p[k]);
    const float rn = r[k] - af * q[k];
    r[k] = rn;
    v = double(rn) * double(rn);
  }
  v = block_sum<double>(v);
  if (threadIdx.x == 0) part[size_t(b) * gridDim.x + lb] = v;
}

// The second kernel of launch slot `it` of the fused residual-replacement
// loop (replace_slot).  Step slots: rc_update with alpha = rrv / (p^T A p)
// summed by every workgroup (at most kFuseParts partials per problem).
// Replacement slots: r = float(f - A64 u) with Dirichlet rows 0, partials of
// |f - A64 u|^2 (FP64, before rounding) in rep; one row per thread, slots in
// colex order, columns outside [0, N) clamped (their band entries are 0).
// Slower per row than the banded product, but it runs on a few slots only.
__global__ void __launch_bounds__(kSpmvBlock)
    rc_step_kernel(SpmvGeom g, CgScalars* __restrict__ sc, const double* __restrict__ pap,
                   const float* __restrict__ p, const float* __restrict__ q, double* __restrict__ u,
                   float* __restrict__ r, double* __restrict__ part, const double* __restrict__ band64,
                   const double* __restrict__ f, double* __restrict__ rep, int it) {
  const int b = blockIdx.y;
  if (sc[b].done) return;
  const int64_t N = g.N;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  if (sc[b].kind[it & 1] == kSlotReplace) {
    const int64_t i = int64_t(lb) * kSpmvBlock + threadIdx.x;
    double v = 0.0;
    if (i < N) {
      const size_t k = size_t(b) * N + i;
      double o = 0.0;
      if (!on_dirichlet(g, i)) {
        const double* bb = band64 + size_t(b) * g.S * g.ld + i;
        const double* ub = u + size_t(b) * N;
        const int64_t m1 = g.m[0], m12 = int64_t(g.m[0]) * g.m[1];
        const int W = g.W, P = g.p, W3 = g.n == 3 ? W : 1;
        double acc = 0.0;
        for (int c = 0; c < W3; ++c)
          for (int e = 0; e < W; ++e) {
            const int64_t base = i + (g.n == 3 ? (c - P) * m12 : 0) + (e - P) * m1 - P;
            const double* bs = bb + size_t((c * W + e) * W) * g.ld;
            for (int a = 0; a < W; ++a) {
              int64_t j = base + a;
              j = j < 0 ? 0 : (j >= N ? N - 1 : j);
              acc += bs[size_t(a) * g.ld] * ub[j];
            }
          }
        o = f[k] - acc;
      }
      r[k] = float(o);
      v = o * o;
    }
    v = block_sum<double>(v);
    if (threadIdx.x == 0) rep[size_t(b) * gridDim.x + lb] = v;
    return;
  }
  const int64_t i = int64_t(lb) * kSpmvBlock + threadIdx.x;
  const size_t k = size_t(b) * N + i;
  // the partials of p^T q and this row's vectors go out together
  PartSum<kSpmvBlock> ps;
  ps.load(pap, b, gridDim.x);
  float pv = 0.f, qv = 0.f, rv = 0.f;
  double uv = 0.0;
  if (i < N) {
    pv = p[k];
    qv = q[k];
    rv = r[k];
    uv = u[k];
  }
  const double s = ps.combine();
  if (!(s > 0.0) || !isfinite(s)) {
    if (lb == 0 && threadIdx.x == 0) {
      sc[b].done = 1;
      sc[b].breakdown = 1;
    }
    return;
  }
  const double alpha = sc[b].rrv[it & 1] / s;
  const float af = float(alpha);
  double v = 0.0;
  if (i < N) {
    u[k] = uv + alpha * double(pv);
    const float rn = rv - af * qv;
    r[k] = rn;
    v = double(rn) * double(rn);
  }
  v = block_sum<double>(v);
  if (threadIdx.x == 0) part[size_t(b) * gridDim.x + lb] = v;
}

// beta = rr_new / rr, or schedule a replacement (beta then comes from the
// replaced residual)
__global__ void __launch_bounds__(kRedBlock) rc_beta_kernel(const double* __restrict__ part, int nblk, CgScalars* sc) {
  const int b = blockIdx.x;
  if (sc[b].done) return;
  double s = 0.0;
  s += strided_sum(part + size_t(b) * nblk, threadIdx.x, nblk);
  s = block_sum<double>(s);
  if (threadIdx.x == 0) {
    if (!isfinite(s)) {
      sc[b].done = 1;
      sc[b].breakdown = 1;
    } else if (s <= kReplace * kReplace * sc[b].rr_ref || s <= sc[b].tol2) {
      sc[b].replace = 1;
    } else {
      sc[b].beta = s / sc[b].rr;
      sc[b].rr = s;
      sc[b].iters += 1;
    }
  }
}

__global__ void __launch_bounds__(kRedBlock) rc_replace_kernel(const double* __restrict__ part, int nblk,
                                                               CgScalars* sc) {
  const int b = blockIdx.x;
  if (sc[b].done || !sc[b].replace) return;
  double s = 0.0;
  s += strided_sum(part + size_t(b) * nblk, threadIdx.x, nblk);
  s = block_sum<double>(s);
  if (threadIdx.x == 0) {
    sc[b].replace = 0;
    sc[b].nrep += 1;
    sc[b].iters += 1;
    if (!isfinite(s)) {
      sc[b].done = 1;
      sc[b].breakdown = 1;
    } else {
      sc[b].beta = s / sc[b].rr;
      sc[b].rr = s;
      sc[b].rr_ref = s;
      if (s <= sc[b].tol2) sc[b].done = 1;
    }
  }
}

static igs_status replace_cg(const Dims& d, const double* band64, const float* band32, const double* f, double* u,
                             double rtol, int maxit, igs_cg_info* info, hipStream_t s) {
  SpmvGeom g = make_geom(d);
  const int nblk = int((d.N + kSpmvBlock - 1) / kSpmvBlock);
  const size_t NB = size_t(d.N) * d.batch;
  const size_t nb = size_t(d.batch);
  Arena ar;
  size_t bytes = padded(sizeof(double) * NB) + 3 * padded(sizeof(double) * nb * nblk) + 4 * padded(sizeof(double) * nb) +
                 padded(sizeof(int) * nb) + padded(sizeof(CgScalars) * nb) + 3 * padded(sizeof(float) * NB);
  igs_status st = ar.alloc(bytes, s);
  if (st != IGS_OK) return st;
  SolveBufs sb;
  sb.r64 = ar.take<double>(NB);
  sb.part = ar.take<double>(nb * nblk);
  sb.part2 = ar.take<double>(nb * nblk);
  double* part3 = ar.take<double>(nb * nblk);
  sb.rr = ar.take<double>(nb);
  sb.ff = ar.take<double>(nb);
  sb.scale = ar.take<double>(nb);
  sb.tol2 = ar.take<double>(nb);
  sb.active = ar.take<int>(nb);
  sb.sc = ar.take<CgScalars>(nb);
  float* r32 = ar.take<float>(NB);
  float* p = ar.take<float>(NB);
  float* q = ar.take<float>(NB);

  // initial FP64 residual
  hipLaunchKernelGGL(zero_dirichlet_kernel, dim3(grid_stride_blocks(NB)), dim3(256), 0, s, g, d.batch, u);
  auto true_residual = [&](std::vector<double>* rr, std::vector<double>* ff) -> igs_status {
    {
      PhaseTimer t("residual_f64", s);
      launch_spmv64<2>(g, nblk, d.batch, band64, u, f, sb.r64, nullptr, 1, nullptr, sb.part, sb.part2, s);
    }
    hipLaunchKernelGGL(reduce_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, sb.part, nblk, sb.rr);
    hipLaunchKernelGGL(reduce_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, sb.part2, nblk, sb.ff);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(rr->data(), sb.rr, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(ff->data(), sb.ff, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return IGS_OK;
  };
  std::vector<double> rr(nb), ff(nb), tol2(nb);
  std::vector<int> active(nb);
  st = true_residual(&rr, &ff);
  if (st != IGS_OK) return st;
  for (size_t b = 0; b < nb; ++b) {
    tol2[b] = rtol * rtol * ff[b];
    active[b] = rr[b] > tol2[b];
  }
  HIP_OK(hipMemcpyAsync(sb.tol2, tol2.data(), sizeof(double) * nb, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(sb.active, active.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(rc_init_kernel, dim3(grid_stride_blocks(NB)), dim3(256), 0, s, int64_t(NB), sb.r64, r32);
  hipLaunchKernelGGL(cg_setup_kernel, dim3(1), dim3(64), 0, s, d.batch, sb.rr, sb.tol2, sb.active, sb.sc);
  HIP_OK(hipGetLastError());

  // At most kFuseParts partials per problem: launch slots of two kernels
  // (replace_slot): the product (A32 r32, the direction update of p and
  // q = A32 p; it decides the slot's role) and the update (step slots: alpha,
  // u and r32, partials of |r32|^2; replacement slots: the FP64 residual).
  // The last two slots of a solve are the replacement that confirms
  // convergence and the product that records it.
  // Otherwise one-workgroup kernels between them: the product, alpha, the
  // update, beta or a scheduled replacement, the FP64 residual and the
  // replacement's scalars (the last two return at once on the steps that
  // have no replacement).
  const bool fused = nblk <= kFuseParts;
  std::vector<CgScalars> hsc(nb);
  ChunkPlanner plan(rr);
  int chunk = plan.first();
  int it = 0;
  while (it < maxit) {
    const int k = std::min(chunk, maxit - it);
    for (int j = 0; j < k; ++j, ++it) {
      const CgDir<float> cd{p, sb.part2, part3, it, it == 0 ? 0 : (fused ? 3 : 1)};
      {
        PhaseTimer t("cg_spmv_f32", s);
        launch_cg_product<float>(g, nblk, d.batch, band32, r32, cd, q, sb.sc, sb.part, s);
      }
      PhaseTimer t("cg_vector_ops", s);
      if (fused) {
        hipLaunchKernelGGL(rc_step_kernel, dim3(nblk, d.batch), dim3(kSpmvBlock), 0, s, g, sb.sc, sb.part, p, q, u,
                           r32, sb.part2, band64, f, part3, it);
      } else {
        hipLaunchKernelGGL(cg_alpha_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, sb.part, nblk, sb.sc);
        hipLaunchKernelGGL(rc_update_kernel, dim3(nblk, d.batch), dim3(kSpmvBlock), 0, s, d.N, sb.sc, p, q, u, r32,
                           sb.part2);
        hipLaunchKernelGGL(rc_beta_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, sb.part2, nblk, sb.sc);
        launch_spmv64<3>(g, nblk, d.batch, band64, u, f, nullptr, r32, 1, sb.sc, sb.part, nullptr, s);
        hipLaunchKernelGGL(rc_replace_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, sb.part, nblk, sb.sc);
      }
    }
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(hsc.data(), sb.sc, sizeof(CgScalars) * nb, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    bool all = true;
    std::vector<double> rrh(nb);
    for (size_t b = 0; b < nb; ++b) {
      all &= hsc[b].done != 0;
      // fused: the product of slot it - 1 recorded r^T r in rrv[(it - 1) & 1]
      rrh[b] = fused ? hsc[b].rrv[(it - 1) & 1] : hsc[b].rr;
    }
    if (all) break;
    // fused: two more slots confirm and record convergence
    chunk = plan.next(hsc, rrh, fused ? it - 1 : it) + (fused ? 2 : 0);
  }
  // report the FP64 residual of the returned solution
  st = true_residual(&rr, &ff);
  if (st != IGS_OK) return st;
  double worst = 0.0;
  bool breakdown = false;
  int iters = 0, nrep = 0;
  for (size_t b = 0; b < nb; ++b) {
    const double rel = ff[b] > 0.0 ? std::sqrt(rr[b] / ff[b]) : 0.0;
    worst = std::isfinite(rel) ? std::max(worst, rel) : rel;
    breakdown |= hsc[b].breakdown != 0;
    iters = std::max(iters, hsc[b].iters);
    nrep = std::max(nrep, hsc[b].nrep);
  }
  info->iterations = iters;
  info->outer_iterations = nrep;
  info->relres = worst;
  igs_status result = (std::isfinite(worst) && worst <= rtol) ? IGS_OK : (breakdown ? IGS_BREAKDOWN : IGS_NOT_CONVERGED);
  info->status = result;
  return result;
}

igs_status solve_cg(const Dims& d, const double* band64, const float* band32, const double* f, double* u, double rtol,
                    int maxit, igs_cg_info* info, hipStream_t s) {
  if (band32) return replace_cg(d, band64, band32, f, u, rtol, maxit, info, s);
  return refine_loop<double>(d, band64, band64, f, u, rtol, maxit, 0.0, info, s);
}

// ------------------------------------------------- matrix-free CG (FP64) --

// r = f - q with r_D = 0; per-block partials of r^T r and f_I^T f_I
__global__ void __launch_bounds__(kSpmvBlock)
    mf_residual_kernel(SpmvGeom g, const double* __restrict__ f, const double* __restrict__ q, double* __restrict__ r,
                       double* __restrict__ prr, double* __restrict__ pff) {
  const int b = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * kSpmvBlock + threadIdx.x;
  double vr = 0.0, vf = 0.0;
  if (i < g.N) {
    const size_t k = size_t(b) * g.N + i;
    const bool dr = on_dirichlet(g, i);
    const double fv = dr ? 0.0 : f[k];
    const double rv = dr ? 0.0 : fv - q[k];
    r[k] = rv;
    vr = rv * rv;
    vf = fv * fv;
  }
  vr = block_sum<double>(vr);
  vf = block_sum<double>(vf);
  if (threadIdx.x == 0) {
    prr[size_t(b) * gridDim.x + blockIdx.x] = vr;
    pff[size_t(b) * gridDim.x + blockIdx.x] = vf;
  }
}

__global__ void copy_vec_kernel(int64_t total, const double* __restrict__ a, double* __restrict__ c) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x)
    c[t] = a[t];
}

// Plain FP64 CG on A_II u_I = f_I with the operator given as a launcher
// (A(x, y): y = A x with y_D = 0; x is zero on the Dirichlet dofs), the same
// stopping rule as solve_cg: the recursive residual is followed, and at its
// convergence the true residual f - A u decides (CG restarts from u if it is
// not below rtol yet).
igs_status solve_cg_op(const Dims& d, const std::function<igs_status(const double*, double*)>& A, const double* f,
                       double* u, double rtol, int maxit, igs_cg_info* info, hipStream_t s) {
  SpmvGeom g = make_geom(d);
  const int nblk = int((d.N + kSpmvBlock - 1) / kSpmvBlock);
  const int dblk = int(std::min<int64_t>((d.N + kRedBlock - 1) / kRedBlock, 1024));
  const size_t NB = size_t(d.N) * d.batch, nb = size_t(d.batch);
  Arena ar;
  igs_status st = ar.alloc(3 * padded(sizeof(double) * NB) + 2 * padded(sizeof(double) * nb * nblk) +
                               4 * padded(sizeof(double) * nb) + padded(sizeof(int) * nb) +
                               padded(sizeof(CgScalars) * nb),
                           s);
  if (st != IGS_OK) return st;
  double* r = ar.take<double>(NB);
  double* p = ar.take<double>(NB);
  double* q = ar.take<double>(NB);
  double* part = ar.take<double>(nb * nblk);
  double* part2 = ar.take<double>(nb * nblk);
  double* rr = ar.take<double>(nb);
  double* ff = ar.take<double>(nb);
  double* tol2 = ar.take<double>(nb);
  double* spare = ar.take<double>(nb);
  (void)spare;
  int* active = ar.take<int>(nb);
  CgScalars* sc = ar.take<CgScalars>(nb);
  hipLaunchKernelGGL(zero_dirichlet_kernel, dim3(grid_stride_blocks(NB)), dim3(256), 0, s, g, d.batch, u);
  std::vector<double> hrr(nb), hff(nb), htol(nb);
  std::vector<int> hact(nb);
  std::vector<CgScalars> hsc(nb);
  int iters = 0, restarts = 0;
  double worst = 0.0;
  igs_status result = IGS_NOT_CONVERGED;
  while (true) {
    // true residual
    igs_status ast = A(u, q);
    if (ast != IGS_OK) return ast;
    hipLaunchKernelGGL(mf_residual_kernel, dim3(nblk, d.batch), dim3(kSpmvBlock), 0, s, g, f, q, r, part, part2);
    hipLaunchKernelGGL(reduce_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, part, nblk, rr);
    hipLaunchKernelGGL(reduce_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, part2, nblk, ff);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(hrr.data(), rr, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(hff.data(), ff, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    bool all = true;
    worst = 0.0;
    for (size_t b = 0; b < nb; ++b) {
      const double rel = hff[b] > 0.0 ? std::sqrt(hrr[b] / hff[b]) : 0.0;
      if (!std::isfinite(rel)) {
        info->relres = rel;
        info->iterations = iters;
        info->outer_iterations = restarts + 1;
        info->status = IGS_BREAKDOWN;
        return IGS_BREAKDOWN;
      }
      worst = std::max(worst, rel);
      hact[b] = rel > rtol;
      all &= !hact[b];
      // the recursive residual is followed to half the target
      htol[b] = 0.25 * rtol * rtol * hff[b];
    }
    if (all) {
      result = IGS_OK;
      break;
    }
    if (iters >= maxit || restarts >= 8) break;
    HIP_OK(hipMemcpyAsync(tol2, htol.data(), sizeof(double) * nb, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(active, hact.data(), sizeof(int) * nb, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(cg_setup_kernel, dim3(1), dim3(64), 0, s, d.batch, rr, tol2, active, sc);
    hipLaunchKernelGGL(copy_vec_kernel, dim3(grid_stride_blocks(NB)), dim3(256), 0, s, int64_t(NB), r, p);
    HIP_OK(hipGetLastError());
    int local = 0;
    bool stop = false;
    while (!stop) {
      const int k = std::min(32, maxit - iters);
      if (k <= 0) break;
      for (int it = 0; it < k; ++it) {
        ast = A(p, q);
        if (ast != IGS_OK) return ast;
        PhaseTimer t("cg_vector_ops", s);
        hipLaunchKernelGGL((dot_kernel<double>), dim3(dblk, d.batch), dim3(kRedBlock), 0, s, d.N, p, q, part);
        hipLaunchKernelGGL(cg_alpha_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, part, dblk, sc);
        hipLaunchKernelGGL((cg_update_kernel<double>), dim3(nblk, d.batch), dim3(kSpmvBlock), 0, s, d.N, sc, p, q, u,
                           r, part2);
        hipLaunchKernelGGL(cg_beta_kernel, dim3(d.batch), dim3(kRedBlock), 0, s, part2, nblk, sc);
        hipLaunchKernelGGL((cg_pupdate_kernel<double>), dim3(std::min<int64_t>((d.N + 255) / 256, 4096), d.batch),
                           dim3(256), 0, s, d.N, sc, r, p);
      }
      HIP_OK(hipGetLastError());
      HIP_OK(hipMemcpyAsync(hsc.data(), sc, sizeof(CgScalars) * nb, hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      bool done = true, brk = false;
      int mx = 0;
      for (size_t b = 0; b < nb; ++b) {
        done &= hsc[b].done != 0;
        brk |= hsc[b].breakdown != 0;
        mx = std::max(mx, hsc[b].iters);
      }
      iters += mx - local;
      local = mx;
      if (brk) {
        info->relres = worst;
        info->iterations = iters;
        info->outer_iterations = restarts + 1;
        info->status = IGS_BREAKDOWN;
        return IGS_BREAKDOWN;
      }
      stop = done;
    }
    ++restarts;
  }
  info->relres = worst;
  info->iterations = iters;
  info->outer_iterations = restarts;
  info->status = result;
  return result;
}

}  // namespace igs
