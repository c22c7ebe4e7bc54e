// Surrogate with a domain per stencil function (Sec. 4, the remark after the
// analysis domain; entries as in Sec. 5): the fit of every stencil function on
// its own samples and the fill of the cardinal rows.
//
// Offset delta's function lives on the rows i with i and i + delta cardinal;
// per direction its samples, inverse collocation matrix and evaluation tables
// depend on delta_d alone (KInterpPD, index e = delta_d + p).
#include <hip/hip_runtime.h>

#include "igs_internal.h"

namespace igs {

// ------------------------------------------------------------------ fit ----
//
// Coefficient blocks [b][u][k3][k2][k1] (2-D: [b][u][k2][k1]) with extent smax
// per direction; entries past an offset's sample count are 0.  Pass d applies
// ginv of direction d along k_d; pass 0 gathers the samples from the band.
template <int ND, typename BT>
__global__ void fit_pd_kernel(KInterpPD ip, int pass, int64_t ld, int S, int batch, const int* __restrict__ upslot,
                              const BT* __restrict__ band, const double* __restrict__ in, double* __restrict__ out) {
  const int sm = ip.smax, W = ip.W;
  const int64_t per = ND == 3 ? int64_t(sm) * sm * sm : int64_t(sm) * sm;
  const int64_t total = per * ip.nup * batch;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    int64_t r = t;
    const int k1 = int(r % sm);
    r /= sm;
    const int k2 = int(r % sm);
    r /= sm;
    int k3 = 0;
    if (ND == 3) {
      k3 = int(r % sm);
      r /= sm;
    }
    const int u = int(r % ip.nup);
    const int b = int(r / ip.nup);
    const int slot = upslot[u];
    const int e1 = slot % W, e2 = (slot / W) % W, e3 = ND == 3 ? slot / (W * W) : 0;
    const int S1 = ip.S[0][e1], S2 = ip.S[1][e2], S3 = ND == 3 ? ip.S[2][e3] : 1;
    if (k1 >= S1 || k2 >= S2 || k3 >= S3) {
      out[t] = 0.0;
      continue;
    }
    const int kd = pass == 0 ? k1 : (pass == 1 ? k2 : k3);
    const int ed = pass == 0 ? e1 : (pass == 1 ? e2 : e3);
    const int Sd = ip.S[pass][ed];
    const double* g = ip.ginv[pass] + (size_t(ed) * sm + kd) * sm;
    double acc = 0.0;
    if (pass == 0) {
      const BT* bs = band + (size_t(b) * S + slot) * ld;
      const size_t rb = size_t(ip.m[0]) * (ip.U[1][ip.pos[1][e2 * sm + k2]] +
                                           size_t(ip.m[1]) * (ND == 3 ? ip.U[2][ip.pos[2][e3 * sm + k3]] : 0));
      const int* ps = ip.pos[0] + e1 * sm;
      for (int j = 0; j < Sd; ++j) acc += g[j] * double(bs[rb + ip.U[0][ps[j]]]);
    } else {
      const int64_t stride = pass == 1 ? sm : int64_t(sm) * sm;
      const double* src = in + (t - int64_t(kd) * stride);
      for (int j = 0; j < Sd; ++j) acc += g[j] * src[j * stride];
    }
    out[t] = acc;
  }
}

// ----------------------------------------------------------------- fill ----
//
// One wave per pencil (i2, i3) of cardinal rows, lanes along i1 (consecutive
// rows, coalesced stores), every slot in turn.  For slot s with offset delta:
//   * the pencil's rows i1 in the slot's domain range (i and i + delta both
//     cardinal) are interpolated; the others keep the exact entries that the
//     quadrature of the non-cardinal rows stores into them later;
//   * upper delta: Phi~_delta at the row; lower delta: Phi~_{-delta} at the
//     partner i + delta (eq. 5.1b), the same arithmetic as the partner's
//     upper entry, so the two are bitwise equal;
//   * the lanes first contract the coefficients over directions 2 and 3 at
//     the evaluation pencil (t[k1], a line in LDS), then evaluate direction 1.
// Stiffness: each lane sums its row's interpolated entries in slot order and
// stores -sum as the diagonal (eq. 5.1c); the exact entries are subtracted
// afterwards (diagonal fix-up).  Mass: delta = 0 is an upper slot.
constexpr int kPdWaves = 4;
constexpr int kPdChunks = 4;  // rows per lane and segment

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int ND, int FORM, int Q, typename T>
__global__ void __launch_bounds__(64 * kPdWaves)
    fill_pd_kernel(KInterpPD ip, int64_t ld, int S, int npen, const double* __restrict__ coef, T* __restrict__ band) {
  extern __shared__ double tl_all[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int pid = blockIdx.x * kPdWaves + w;
  if (pid >= npen) return;  // whole waves; no barrier across waves below
  const int sm = ip.smax, W = ip.W, p = ip.p;
  double* tl = tl_all + size_t(w) * sm;
  const int m1 = ip.m[0], m2 = ip.m[1];
  const int L2 = m2 - 2 * p;
  const int i2 = p + pid % L2, i3 = ND == 3 ? p + pid / L2 : 0;
  const int b = blockIdx.y;
  T* out = band + size_t(b) * S * ld;
  const int64_t per = ND == 3 ? int64_t(sm) * sm * sm : int64_t(sm) * sm;
  const double* cb = coef + size_t(b) * ip.nup * per;
  const size_t rowbase = size_t(m1) * (i2 + size_t(m2) * i3);
  const int sc = (S - 1) / 2;
  constexpr bool STIFF = FORM == IGS_STIFFNESS;
  const int hi1c = m1 - p - 1;
  for (int seg0 = p; seg0 <= hi1c; seg0 += 64 * kPdChunks) {
    double rs[kPdChunks];
#pragma unroll
    for (int c = 0; c < kPdChunks; ++c) rs[c] = 0.0;
    for (int s = 0; s < S; ++s) {
      if (STIFF && s == sc) continue;
      const int e1 = s % W, e2 = (s / W) % W, e3 = ND == 3 ? s / (W * W) : 0;
      if (i2 < ip.lo[1][e2] || i2 > ip.hi[1][e2]) continue;
      if (ND == 3 && (i3 < ip.lo[2][e3] || i3 > ip.hi[2][e3])) continue;
      const int lo1 = max(ip.lo[0][e1], seg0), hi1 = min(ip.hi[0][e1], seg0 + 64 * kPdChunks - 1);
      if (lo1 > hi1) continue;
      const bool upper = s >= sc;
      // the interpolated function (offset index per direction) and where it is evaluated
      const int f1e = upper ? e1 : W - 1 - e1, f2e = upper ? e2 : W - 1 - e2, f3e = upper ? e3 : W - 1 - e3;
      const int sh1 = upper ? 0 : e1 - p, sh2 = upper ? 0 : e2 - p, sh3 = upper ? 0 : e3 - p;
      const int us = upper ? s : S - 1 - s;
      const int u = us - sc - (STIFF ? 1 : 0);
      const int j2 = i2 + sh2, j3 = i3 + sh3;
      const int f2 = ip.ef[1][f2e * m2 + j2];
      double b2[Q + 1], b3[Q + 1];
#pragma unroll
      for (int a = 0; a <= Q; ++a) b2[a] = ip.eb[1][(size_t(f2e) * (Q + 1) + a) * m2 + j2];
      int f3 = 0;
      if constexpr (ND == 3) {
        const int m3 = ip.m[2];
        f3 = ip.ef[2][f3e * m3 + j3];
#pragma unroll
        for (int a = 0; a <= Q; ++a) b3[a] = ip.eb[2][(size_t(f3e) * (Q + 1) + a) * m3 + j3];
      }
      const int S1 = ip.S[0][f1e];
      const double* cu = cb + size_t(u) * per;
      wave_sync();  // every lane is done reading the previous slot's line
      for (int k1 = lane; k1 < S1; k1 += 64) {
        double acc = 0.0;
        if constexpr (ND == 3) {
#pragma unroll
          for (int a3 = 0; a3 <= Q; ++a3) {
            double r = 0.0;
#pragma unroll
            for (int a2 = 0; a2 <= Q; ++a2) r += cu[(size_t(f3 + a3) * sm + f2 + a2) * sm + k1] * b2[a2];
            acc += r * b3[a3];
          }
        } else {
#pragma unroll
          for (int a2 = 0; a2 <= Q; ++a2) acc += cu[size_t(f2 + a2) * sm + k1] * b2[a2];
        }
        tl[k1] = acc;
      }
      wave_sync();
      const int* ef1 = ip.ef[0] + f1e * m1;
      const double* eb1 = ip.eb[0] + size_t(f1e) * (Q + 1) * m1;
      T* os = out + size_t(s) * ld + rowbase;
#pragma unroll
      for (int c = 0; c < kPdChunks; ++c) {
        const int i1 = seg0 + 64 * c + lane;
        if (i1 >= lo1 && i1 <= hi1) {
          const int j1 = i1 + sh1;
          const int f1 = ef1[j1];
          double v = 0.0;
#pragma unroll
          for (int a = 0; a <= Q; ++a) v += tl[f1 + a] * eb1[size_t(a) * m1 + j1];
          os[i1] = static_cast<T>(v);
          rs[c] += v;
        }
      }
    }
    if constexpr (STIFF) {
#pragma unroll
      for (int c = 0; c < kPdChunks; ++c) {
        const int i1 = seg0 + 64 * c + lane;
        if (i1 <= hi1c) out[size_t(sc) * ld + rowbase + i1] = static_cast<T>(-rs[c]);
      }
    }
  }
}

// 3-D fill.  A block owns one plane i3 and kP2 consecutive pencils i2 (wave w
// takes pencils w, w + 4, ...) and walks the active slots in groups of kGrp.
// Phase 1: per slot of the group, one wave contracts the coefficients over
// direction 3 into a slab C3[k2][k1] covering the coefficient rows k2 the
// block's pencils need (global loads only).  Phase 2: each wave contracts
// direction 2 for one pencil at a time into its line t[k1] and evaluates
// direction 1 along the pencil (LDS reads and band stores only).  Loads and
// stores share one in-order counter on this hardware, so a load issued after
// stores waits for them too; grouping keeps that wait to once per group.  The
// spline rows of directions 1 and 2 at the block's evaluation indices are
// staged in LDS (direction 1 per segment of 128 rows).
constexpr int kP2 = 16;
constexpr int kGrp = 8;
constexpr int kSeg = 64 * 2;  // rows per lane pair and segment

struct Pd3Layout {
  size_t c3, tl, e2b, e2f, e1b, e1f, slist, total;  // byte offsets
};

__host__ __device__ inline Pd3Layout pd3_layout(int sm, int W, int q, int p, int S) {
  Pd3Layout L;
  const size_t NJ = kP2 + 2 * p, NJ1 = kSeg + 2 * p;
  L.c3 = 0;
  L.tl = L.c3 + size_t(kGrp) * (kP2 + q + 1) * sm * sizeof(double);
  L.e2b = L.tl + size_t(kPdWaves) * (kP2 / kPdWaves) * sm * sizeof(double);
  L.e1b = L.e2b + size_t(W) * (q + 1) * NJ * sizeof(double);
  L.e2f = L.e1b + size_t(W) * (q + 1) * NJ1 * sizeof(double);
  L.e1f = L.e2f + size_t(W) * NJ * sizeof(int);
  L.slist = L.e1f + size_t(W) * NJ1 * sizeof(int);
  L.total = L.slist + size_t(S + 1) * sizeof(int);
  return L;
}

// t / d for t, d < 2^16 with a 32-bit multiply-high and one exact correction
// (d and its reciprocal m = floor(2^32 / d) + 1 are wave-uniform)
__device__ __forceinline__ int div_small(int t, int d, unsigned m) {
  int q = int(__umulhi(unsigned(t), m));
  if (t - q * d >= d) ++q;
  if (t - q * d < 0) --q;
  return q;
}

template <int FORM, int P, int Q, typename T>
__global__ void __launch_bounds__(64 * kPdWaves)
    fill_pd3_kernel(KInterpPD ip, int64_t ld, int S, int nchunk2, const double* __restrict__ coef,
                    T* __restrict__ band) {
  extern __shared__ double sh[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, tid = threadIdx.x;
  constexpr int W = 2 * P + 1, p = P;
  const int sm = ip.smax;
  const int m1 = ip.m[0], m2 = ip.m[1], m3 = ip.m[2];
  const Pd3Layout L = pd3_layout(sm, W, Q, p, S);
  char* base = reinterpret_cast<char*>(sh);
  double* C3 = reinterpret_cast<double*>(base + L.c3);
  double* tl = reinterpret_cast<double*>(base + L.tl) + size_t(w) * (kP2 / kPdWaves) * sm;  // [NPW][sm]
  double* E2b = reinterpret_cast<double*>(base + L.e2b);
  double* E1b = reinterpret_cast<double*>(base + L.e1b);
  int* E2f = reinterpret_cast<int*>(base + L.e2f);
  int* E1f = reinterpret_cast<int*>(base + L.e1f);
  int* slist = reinterpret_cast<int*>(base + L.slist);
  constexpr int NJ = kP2 + 2 * p, NJ1 = kSeg + 2 * p;
  const size_t c3n = size_t(kP2 + Q + 1) * sm;  // one slab
  const int c2 = blockIdx.x % nchunk2;
  const int i3 = p + blockIdx.x / nchunk2;
  const int c0 = p + c2 * kP2, c1 = min(c0 + kP2 - 1, m2 - p - 1);
  const int j0 = c0 - p;  // first staged evaluation index of direction 2
  for (int t = tid; t < W * NJ; t += 64 * kPdWaves) {
    const int e = t / NJ, jj = t - e * NJ, j = min(j0 + jj, m2 - 1);
    E2f[t] = ip.ef[1][e * m2 + j];
#pragma unroll
    for (int a = 0; a <= Q; ++a) E2b[(e * (Q + 1) + a) * NJ + jj] = ip.eb[1][(size_t(e) * (Q + 1) + a) * m2 + j];
  }
  const int b = blockIdx.y;
  T* out = band + size_t(b) * S * ld;
  const int64_t per = int64_t(sm) * sm * sm;
  const double* cb = coef + size_t(b) * ip.nup * per;
  const int sc = (S - 1) / 2;
  constexpr bool STIFF = FORM == IGS_STIFFNESS;
  constexpr int NPW = kP2 / kPdWaves;  // pencils per wave
  constexpr int NCH = kSeg / 64;
  const int hi1c = m1 - p - 1;
  // slot s's offsets, function and domain for this block and segment
  struct Prm {
    int e1, e2, e3, f1e, f2e, f3e, sh1, sh2, sh3, u, a2lo, a2hi, lo1, hi1;
  };
  auto prm = [&](int s, int seg0) {
    Prm R;
    R.e1 = s % W;
    R.e2 = (s / W) % W;
    R.e3 = s / (W * W);
    const bool upper = s >= sc;
    R.f1e = upper ? R.e1 : W - 1 - R.e1;
    R.f2e = upper ? R.e2 : W - 1 - R.e2;
    R.f3e = upper ? R.e3 : W - 1 - R.e3;
    R.sh1 = upper ? 0 : R.e1 - p;
    R.sh2 = upper ? 0 : R.e2 - p;
    R.sh3 = upper ? 0 : R.e3 - p;
    R.u = (upper ? s : S - 1 - s) - sc - (STIFF ? 1 : 0);
    R.a2lo = max(c0, ip.lo[1][R.e2]);
    R.a2hi = min(c1, ip.hi[1][R.e2]);
    R.lo1 = max(ip.lo[0][R.e1], seg0);
    R.hi1 = min(ip.hi[0][R.e1], seg0 + kSeg - 1);
    return R;
  };
  for (int seg0 = p; seg0 <= hi1c; seg0 += kSeg) {
    const int J1 = seg0 - p;  // first staged evaluation index of direction 1
    __syncthreads();          // previous segment done with the staged rows
    for (int t = tid; t < W * NJ1; t += 64 * kPdWaves) {
      const int e = t / NJ1, jj = t - e * NJ1, j = min(J1 + jj, m1 - 1);
      E1f[t] = ip.ef[0][e * m1 + j];
#pragma unroll
      for (int a = 0; a <= Q; ++a) E1b[(e * (Q + 1) + a) * NJ1 + jj] = ip.eb[0][(size_t(e) * (Q + 1) + a) * m1 + j];
    }
    if (tid == 0) {
      int n = 0;
      for (int s = 0; s < S; ++s) {
        if (STIFF && s == sc) continue;
        const Prm R = prm(s, seg0);
        if (i3 < ip.lo[2][R.e3] || i3 > ip.hi[2][R.e3] || R.a2lo > R.a2hi || R.lo1 > R.hi1) continue;
        slist[n++] = s;
      }
      slist[S] = n;
    }
    __syncthreads();
    const int nact = slist[S];
    double rs[NPW][NCH];
#pragma unroll
    for (int r = 0; r < NPW; ++r)
#pragma unroll
      for (int c = 0; c < NCH; ++c) rs[r][c] = 0.0;
    for (int g0 = 0; g0 < nact; g0 += kGrp) {
      const int ng = min(kGrp, nact - g0);
      // phase 1: slabs of the group's slots, slot gi by wave gi % 4
      for (int gi = w; gi < ng; gi += kPdWaves) {
        const Prm R = prm(slist[g0 + gi], seg0);
        const int j3 = i3 + R.sh3;
        const int f3 = ip.ef[2][R.f3e * m3 + j3];
        double b3[Q + 1];
#pragma unroll
        for (int a = 0; a <= Q; ++a) b3[a] = ip.eb[2][(size_t(R.f3e) * (Q + 1) + a) * m3 + j3];
        const int K2lo = E2f[R.f2e * NJ + (R.a2lo + R.sh2 - j0)];
        const int nk2 = E2f[R.f2e * NJ + (R.a2hi + R.sh2 - j0)] + Q + 1 - K2lo;
        const int S1 = ip.S[0][R.f1e];
        const double* cu = cb + size_t(R.u) * per;
        double* slab = C3 + size_t(gi) * c3n;
        const int nel = nk2 * S1;
        const unsigned rS1 = unsigned(0xffffffffu / unsigned(S1)) + 1u;
        // four elements per lane and pass: their loads are in flight together
        for (int t0 = 0; t0 < nel; t0 += 256) {
          double v[4][Q + 1];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int t = min(t0 + 64 * j + lane, nel - 1);
            const int kq = div_small(t, S1, rS1);
            const int k2 = K2lo + kq, k1 = t - kq * S1;
#pragma unroll
            for (int a3 = 0; a3 <= Q; ++a3) v[j][a3] = cu[(size_t(f3 + a3) * sm + k2) * sm + k1];
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int t = t0 + 64 * j + lane;
            double acc = 0.0;
#pragma unroll
            for (int a3 = 0; a3 <= Q; ++a3) acc += v[j][a3] * b3[a3];
            if (t < nel) slab[t] = acc;
          }
        }
      }
      __syncthreads();
      // phase 2: every wave, every slot of the group, its pencils
      for (int gi = 0; gi < ng; ++gi) {
        const int s = slist[g0 + gi];
        const Prm R = prm(s, seg0);
        const int K2lo = E2f[R.f2e * NJ + (R.a2lo + R.sh2 - j0)];
        const int S1 = ip.S[0][R.f1e];
        const double* slab = C3 + size_t(gi) * c3n;
        T* os = out + size_t(s) * ld + size_t(m1) * size_t(m2) * i3;
        // this lane's direction-1 rows for the slot
        int f1[NCH];
        double b1[NCH][Q + 1];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const int jj = min(max(seg0 + 64 * c + lane + R.sh1 - J1, 0), NJ1 - 1);
          f1[c] = E1f[R.f1e * NJ1 + jj];
#pragma unroll
          for (int a = 0; a <= Q; ++a) b1[c][a] = E1b[(R.f1e * (Q + 1) + a) * NJ1 + jj];
        }
        // lines t[k1] of the wave's pencils: lane pairs (k1, pencil r)
        wave_sync();  // the previous slot's lines are no longer read
        for (int t = lane; t < NPW * S1; t += 64) {
          const int r = t % NPW, k1 = t / NPW;
          const int i2 = c0 + w + kPdWaves * r;
          const int jj = min(max(i2 + R.sh2 - j0, 0), NJ - 1);
          const bool ok = i2 >= R.a2lo && i2 <= R.a2hi;
          const int f2 = ok ? E2f[R.f2e * NJ + jj] - K2lo : 0;
          const double* e2 = E2b + R.f2e * (Q + 1) * NJ + jj;
          const double* sl = slab + f2 * S1 + k1;
          double acc = 0.0;
#pragma unroll
          for (int a2 = 0; a2 <= Q; ++a2) acc += sl[a2 * S1] * e2[a2 * NJ];
          tl[r * sm + k1] = acc;
        }
        wave_sync();
        // rows: every (pencil, chunk) of this lane
#pragma unroll
        for (int r = 0; r < NPW; ++r) {
          const int i2 = c0 + w + kPdWaves * r;
          if (i2 < R.a2lo || i2 > R.a2hi) continue;  // wave-uniform
          T* orow = os + size_t(m1) * i2;
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            const int i1 = seg0 + 64 * c + lane;
            if (i1 >= R.lo1 && i1 <= R.hi1) {
              double v = 0.0;
#pragma unroll
              for (int a = 0; a <= Q; ++a) v += tl[r * sm + f1[c] + a] * b1[c][a];
              orow[i1] = static_cast<T>(v);
              rs[r][c] += v;
            }
          }
        }
      }
      __syncthreads();  // the group's slabs are no longer read
    }
    if constexpr (STIFF) {
#pragma unroll
      for (int r = 0; r < NPW; ++r) {
        const int i2 = c0 + w + kPdWaves * r;
        if (i2 > c1) continue;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const int i1 = seg0 + 64 * c + lane;
          if (i1 <= hi1c) out[size_t(sc) * ld + size_t(m1) * (i2 + size_t(m2) * i3) + i1] = static_cast<T>(-rs[r][c]);
        }
      }
    }
  }
}

// ------------------------------------------------------------ launchers ----

template <typename BT>
hipError_t launch_fit_pd(const KInterpPD& ip, int n, int64_t ld, int S, int batch, const int* upslot, const BT* band,
                         double* tmp0, double* tmp1, double* coef, hipStream_t s) {
  const int sm = ip.smax;
  const int64_t total = (n == 3 ? int64_t(sm) * sm * sm : int64_t(sm) * sm) * ip.nup * batch;
  const int blocks = int(std::min<int64_t>((total + 255) / 256, 65535));
  double* bufs[3] = {tmp0, tmp1, tmp0};
  const double* in = nullptr;
  for (int pass = 0; pass < n; ++pass) {
    double* o = pass == n - 1 ? coef : bufs[pass];
    if (n == 3)
      hipLaunchKernelGGL((fit_pd_kernel<3, BT>), dim3(blocks), dim3(256), 0, s, ip, pass, ld, S, batch, upslot, band,
                         in, o);
    else
      hipLaunchKernelGGL((fit_pd_kernel<2, BT>), dim3(blocks), dim3(256), 0, s, ip, pass, ld, S, batch, upslot, band,
                         in, o);
    in = o;
  }
  return hipGetLastError();
}

template hipError_t launch_fit_pd<double>(const KInterpPD&, int, int64_t, int, int, const int*, const double*,
                                          double*, double*, double*, hipStream_t);
template hipError_t launch_fit_pd<float>(const KInterpPD&, int, int64_t, int, int, const int*, const float*, double*,
                                         double*, double*, hipStream_t);

template <int ND, int FORM, typename T>
static void launch_fill_pd_q(const KInterpPD& ip, int64_t ld, int S, int npen, int batch, const double* coef, T* band,
                             hipStream_t s) {
  dim3 grid((npen + kPdWaves - 1) / kPdWaves, batch);
  const size_t lds = size_t(kPdWaves) * ip.smax * sizeof(double);
  switch (ip.q) {
    case 1: hipLaunchKernelGGL((fill_pd_kernel<ND, FORM, 1, T>), grid, dim3(64 * kPdWaves), lds, s, ip, ld, S, npen, coef, band); break;
    case 2: hipLaunchKernelGGL((fill_pd_kernel<ND, FORM, 2, T>), grid, dim3(64 * kPdWaves), lds, s, ip, ld, S, npen, coef, band); break;
    case 3: hipLaunchKernelGGL((fill_pd_kernel<ND, FORM, 3, T>), grid, dim3(64 * kPdWaves), lds, s, ip, ld, S, npen, coef, band); break;
    case 4: hipLaunchKernelGGL((fill_pd_kernel<ND, FORM, 4, T>), grid, dim3(64 * kPdWaves), lds, s, ip, ld, S, npen, coef, band); break;
    default: hipLaunchKernelGGL((fill_pd_kernel<ND, FORM, 5, T>), grid, dim3(64 * kPdWaves), lds, s, ip, ld, S, npen, coef, band); break;
  }
}

static size_t fill_pd3_lds(const KInterpPD& ip, int S) { return pd3_layout(ip.smax, ip.W, ip.q, ip.p, S).total; }

size_t fill_pd_lds_bytes(const KInterpPD& ip, int S) {
  return ip.m[2] > 1 ? fill_pd3_lds(ip, S) : size_t(kPdWaves) * ip.smax * sizeof(double);
}

template <int FORM, int P, typename T>
static void launch_fill_pd3_p(const KInterpPD& ip, const Dims& d, const double* coef, T* band, hipStream_t s) {
  const int nchunk2 = (d.m[1] - 2 * d.p + kP2 - 1) / kP2;
  dim3 grid(nchunk2 * (d.m[2] - 2 * d.p), d.batch);
  const size_t lds = fill_pd3_lds(ip, d.S);
  switch (ip.q) {
    case 1: hipLaunchKernelGGL((fill_pd3_kernel<FORM, P, 1, T>), grid, dim3(64 * kPdWaves), lds, s, ip, d.ld, d.S, nchunk2, coef, band); break;
    case 2: hipLaunchKernelGGL((fill_pd3_kernel<FORM, P, 2, T>), grid, dim3(64 * kPdWaves), lds, s, ip, d.ld, d.S, nchunk2, coef, band); break;
    case 3: hipLaunchKernelGGL((fill_pd3_kernel<FORM, P, 3, T>), grid, dim3(64 * kPdWaves), lds, s, ip, d.ld, d.S, nchunk2, coef, band); break;
    case 4: hipLaunchKernelGGL((fill_pd3_kernel<FORM, P, 4, T>), grid, dim3(64 * kPdWaves), lds, s, ip, d.ld, d.S, nchunk2, coef, band); break;
    default: hipLaunchKernelGGL((fill_pd3_kernel<FORM, P, 5, T>), grid, dim3(64 * kPdWaves), lds, s, ip, d.ld, d.S, nchunk2, coef, band); break;
  }
}

template <int FORM, typename T>
static void launch_fill_pd3(const KInterpPD& ip, const Dims& d, const double* coef, T* band, hipStream_t s) {
  switch (d.p) {
    case 1: launch_fill_pd3_p<FORM, 1, T>(ip, d, coef, band, s); break;
    case 2: launch_fill_pd3_p<FORM, 2, T>(ip, d, coef, band, s); break;
    case 3: launch_fill_pd3_p<FORM, 3, T>(ip, d, coef, band, s); break;
    default: launch_fill_pd3_p<FORM, 4, T>(ip, d, coef, band, s); break;
  }
}

template <typename T>
hipError_t launch_fill_pd(const KInterpPD& ip, int form, const Dims& d, const double* coef, T* band, hipStream_t s) {
  const int npen = (d.m[1] - 2 * d.p) * (d.n == 3 ? d.m[2] - 2 * d.p : 1);
  if (npen <= 0) return hipSuccess;
  if (d.n == 3) {
    if (form == IGS_MASS)
      launch_fill_pd3<IGS_MASS, T>(ip, d, coef, band, s);
    else
      launch_fill_pd3<IGS_STIFFNESS, T>(ip, d, coef, band, s);
  } else {
    if (form == IGS_MASS)
      launch_fill_pd_q<2, IGS_MASS, T>(ip, d.ld, d.S, npen, d.batch, coef, band, s);
    else
      launch_fill_pd_q<2, IGS_STIFFNESS, T>(ip, d.ld, d.S, npen, d.batch, coef, band, s);
  }
  return hipGetLastError();
}

template hipError_t launch_fill_pd<double>(const KInterpPD&, int, const Dims&, const double*, double*, hipStream_t);
template hipError_t launch_fill_pd<float>(const KInterpPD&, int, const Dims&, const double*, float*, hipStream_t);

}  // namespace igs
