// 2-D fill of the surrogate band (Sec. 5, eqs. 5.1b and 5.1c): the
// interpolated entries of every analysis-domain row, evaluated separably from
// the tensor spline coefficients of each upper stencil function.
#include <algorithm>

#include "igs_internal.h"

namespace igs {

// 2D fill: one workgroup per analysis-domain pencil (fixed i2), its threads
// striding over the whole pencil (R rows each, consecutive threads on
// consecutive rows, so each store instruction covers a contiguous run).  Per
// interpolated delta u = (d1, d2):
//   A  the pencil's line contractions in direction 2 for pencils i2 (upper
//      entries) and i2 - d2 (lower ones): T[side][c1] = sum_a2 beta2 c_u[f2+a2][c1];
//   B  each row i1 finishes both with its own q+1 direction-1 weights (kept in
//      registers): the upper entry Phi~_u(i1, i2) and the value Phi~_u(i1, i2-d2),
//      which is the lower entry of row i1 + d1; the latter goes to LDS;
//   C  each row reads its lower entry Phi~_u(i1 - d1, i2 - d2) from LDS.
// Nothing is staged but the two contraction lines and one pencil of values, so
// the LDS footprint is (2 S1 + m1) values whatever the mesh.  Only the rows of
// the fill range [lo1, hi1] are stored (the rows outside it come from the
// boundary-row quadrature, which may run before this kernel); entries that
// are not interpolated get placeholders (0), which the copy kernel
// overwrites.
// PF: every direction-2 task has its own thread (2 S1 <= blockDim.x); its
// operands for the next delta are loaded while the rows finish this one.
// WREG: each row's q+1 direction-1 weights stay in registers for the whole
// delta loop; without it (long pencils, R = 8 rows per thread) they are
// loaded again for every delta (L2 hits).
template <int FORM, int Q, int R, typename T, bool PF, bool WREG>
__global__ void __launch_bounds__(1024)
    fill2d_kernel(KInterp<T> ip, int m1, int64_t N, int64_t ld, int S, const int4* __restrict__ dsl,
                  const double* __restrict__ coef, T* __restrict__ band) {
  // the last workgroup of each problem zeroes its band's padding columns
  // [N, ld) (no launch of its own after the fill)
  if (blockIdx.x == gridDim.x - 1) {
    T* bb = band + size_t(blockIdx.y) * S * ld;
    const int64_t pad = ld - N;
    for (int64_t t = threadIdx.x; t < pad * S; t += blockDim.x) {
      const int64_t sl = t / pad;
      bb[sl * ld + N + (t - sl * pad)] = T(0);
    }
    return;
  }
  extern __shared__ char smem_raw[];
  const int S1 = ip.Sd[0], S2 = ip.Sd[1];
  T* Tl = reinterpret_cast<T*>(smem_raw);  // [2][S1]
  T* Lb = Tl + 2 * S1;                     // [m1]
  const int nt = blockDim.x, tid = threadIdx.x;
  const int i2 = ip.lo[1] + blockIdx.x;
  const int b = blockIdx.y;
  const int sc = (S - 1) / 2;
  T* bnd = band + size_t(b) * S * ld + size_t(i2) * m1;
  const double* cb = coef + size_t(b) * ip.nup * S1 * S2;

  T w1[WREG ? R : 1][Q + 1];
  int f1[R];
  bool in1[R];
  T dsum[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i1 = tid + r * nt;
    in1[r] = i1 < m1 && i1 >= ip.lo[0] && i1 <= ip.hi[0];
    f1[r] = in1[r] ? ip.ef[0][i1] : 0;
    if constexpr (WREG) {
#pragma unroll
      for (int a = 0; a <= Q; ++a) w1[r][a] = in1[r] ? ip.eb[0][size_t(i1) * (Q + 1) + a] : T(0);
    }
    dsum[r] = T(0);
  }

  // operands of this thread's direction-2 task for delta u (PF only): every
  // lane loads (tasks past 2 S1 repeat the last one, tasks of a pencil outside
  // the domain read pencil i2 with zero weights)
  double cv[PF ? Q + 1 : 1];
  T wv[PF ? Q + 1 : 1];
  auto task_load = [&](int u) {
    const int4 dd = dsl[u];
    const bool hl = FORM == IGS_STIFFNESS || dd.x != sc;
    const int t = min(tid, 2 * S1 - 1);
    const int side = t >= S1;
    const int c1 = side ? t - S1 : t;
    const bool ok = side ? (hl && i2 - dd.z >= ip.lo[1]) : (i2 + dd.z <= ip.hi[1]);
    const int p2 = (ok && side) ? i2 - dd.z : i2;
    const int f2 = ip.ef[1][p2];
    const double* cu = cb + size_t(u) * S1 * S2 + c1;
    const T z = ok ? T(1) : T(0);
#pragma unroll
    for (int a = 0; a < (PF ? Q + 1 : 1); ++a) {
      cv[a] = cu[size_t(f2 + a) * S1];
      wv[a] = z * ip.eb[1][size_t(p2) * (Q + 1) + a];
    }
  };
  if constexpr (PF) task_load(0);

  for (int u = 0; u < ip.nup; ++u) {
    const int4 dd = dsl[u];
    const int s = dd.x, d1 = dd.y, d2 = dd.z;
    const bool has_lo = FORM == IGS_STIFFNESS || s != sc;
    const bool up2 = i2 + d2 <= ip.hi[1];          // d2 >= 0 for upper deltas
    const int j2 = i2 - d2;
    const bool lo2 = has_lo && j2 >= ip.lo[1];
    // A: direction-2 contractions of the two pencils
    if constexpr (PF) {
      T v = T(0);
#pragma unroll
      for (int a = 0; a <= Q; ++a) v += wv[a] * T(cv[a]);
      if (tid < 2 * S1) Tl[tid] = v;
      if (u + 1 < ip.nup) task_load(u + 1);
    } else {
      const double* cu = cb + size_t(u) * S1 * S2;
      for (int t = tid; t < 2 * S1; t += nt) {
        const int side = t >= S1;
        const int c1 = side ? t - S1 : t;
        const int p2 = side ? j2 : i2;
        T v = T(0);
        if (side ? lo2 : up2) {
          const int f2 = ip.ef[1][p2];
          const T* w2 = ip.eb[1] + size_t(p2) * (Q + 1);
#pragma unroll
          for (int a = 0; a <= Q; ++a) v += w2[a] * T(cu[size_t(f2 + a) * S1 + c1]);
        }
        Tl[t] = v;
      }
    }
    __syncthreads();
    // B: upper entries; values at pencil i2 - d2 for the lower partners
    T vu[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i1 = tid + r * nt;
      vu[r] = T(0);
      T vl = T(0);
      if (in1[r]) {
        T wr[Q + 1];
#pragma unroll
        for (int a = 0; a <= Q; ++a) {
          if constexpr (WREG)
            wr[a] = w1[WREG ? r : 0][a];
          else
            wr[a] = ip.eb[0][size_t(i1) * (Q + 1) + a];
        }
#pragma unroll
        for (int a = 0; a <= Q; ++a) {
          vu[r] += wr[a] * Tl[f1[r] + a];
          vl += wr[a] * Tl[S1 + f1[r] + a];
        }
        if (!(up2 && i1 + d1 >= ip.lo[0] && i1 + d1 <= ip.hi[0])) vu[r] = T(0);
      }
      if (i1 < m1) Lb[i1] = vl;
    }
    __syncthreads();
    // C: lower entries, stores
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i1 = tid + r * nt;
      if (!in1[r]) continue;
      T vl = T(0);
      if (in1[r] && lo2) {
        const int k1 = i1 - d1;
        if (k1 >= ip.lo[0] && k1 <= ip.hi[0]) vl = Lb[k1];
      }
      bnd[size_t(s) * ld + i1] = vu[r];
      if (has_lo) bnd[size_t(S - 1 - s) * ld + i1] = vl;
      if (FORM == IGS_STIFFNESS) dsum[r] += vu[r] + vl;
    }
  }
  if (FORM == IGS_STIFFNESS) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i1 = tid + r * nt;
      if (in1[r]) bnd[size_t(sc) * ld + i1] = -dsum[r];
    }
  }
}

template <int FORM, int R, typename T, bool PF, bool WREG>
static void launch_fill2d_q(const KInterp<T>& ip, const Dims& d, int nt, size_t lds, const int4* dsl,
                            const double* coef, T* band, hipStream_t s) {
  dim3 grid(ip.hi[1] - ip.lo[1] + 2, d.batch);  // + the padding workgroup
  switch (ip.q) {
    case 1: hipLaunchKernelGGL((fill2d_kernel<FORM, 1, R, T, PF, WREG>), grid, dim3(nt), lds, s, ip, d.m[0], d.N, d.ld, d.S, dsl, coef, band); break;
    case 2: hipLaunchKernelGGL((fill2d_kernel<FORM, 2, R, T, PF, WREG>), grid, dim3(nt), lds, s, ip, d.m[0], d.N, d.ld, d.S, dsl, coef, band); break;
    case 3: hipLaunchKernelGGL((fill2d_kernel<FORM, 3, R, T, PF, WREG>), grid, dim3(nt), lds, s, ip, d.m[0], d.N, d.ld, d.S, dsl, coef, band); break;
    case 4: hipLaunchKernelGGL((fill2d_kernel<FORM, 4, R, T, PF, WREG>), grid, dim3(nt), lds, s, ip, d.m[0], d.N, d.ld, d.S, dsl, coef, band); break;
    default: hipLaunchKernelGGL((fill2d_kernel<FORM, 5, R, T, PF, WREG>), grid, dim3(nt), lds, s, ip, d.m[0], d.N, d.ld, d.S, dsl, coef, band); break;
  }
}

template <int FORM, int R, typename T, bool WREG>
static void launch_fill2d_pf(const KInterp<T>& ip, const Dims& d, int nt, size_t lds, const int4* dsl,
                             const double* coef, T* band, hipStream_t s) {
  // prefetching needs one thread per task; at q = 5 its registers beside the
  // rows' weights spill, and the plain loop is faster there
  if (2 * ip.Sd[0] <= nt && ip.q <= 4)
    launch_fill2d_q<FORM, R, T, true, WREG>(ip, d, nt, lds, dsl, coef, band, s);
  else
    launch_fill2d_q<FORM, R, T, false, WREG>(ip, d, nt, lds, dsl, coef, band, s);
}

// 2D pencils of up to kFill2dRows rows take fill2d_kernel with the weights in
// registers; up to kFill2dWideRows, when the plan found that the LDS
// footprint fits (Dims::wide2d), with the weights reloaded per delta
constexpr int kFill2dR = 4;
constexpr int kFill2dRows = 1024 * kFill2dR;
constexpr int kFill2dWideR = 8;
constexpr int kFill2dWideRows = 1024 * kFill2dWideR;

static size_t fill2d_lds(int S1, int m1, size_t tsize) { return (size_t(2) * S1 + m1) * tsize; }

bool fill_is_2d(const Dims& d) {
  return d.n == 2 && (d.m[0] <= kFill2dRows || (d.wide2d && d.m[0] <= kFill2dWideRows));
}

bool fill2d_wide_fits(const Dims& d, int S1, size_t tsize) {
  return d.n == 2 && d.m[0] > kFill2dRows && d.m[0] <= kFill2dWideRows &&
         fill2d_lds(S1, d.m[0], tsize) <= 160 * 1024;
}

template <typename T>
hipError_t launch_fill2d(const KInterp<T>& ip, int form, const Dims& d, const int4* dsl, const double* coef, T* band,
                         hipStream_t s) {
  const bool wide = d.m[0] > kFill2dRows;
  const int R = wide ? kFill2dWideR : kFill2dR;
  const int rows_per = (d.m[0] + R - 1) / R;
  const int nt = std::min(1024, (rows_per + 63) / 64 * 64);
  const size_t lds = fill2d_lds(ip.Sd[0], d.m[0], sizeof(T));
  if (lds > 160 * 1024 || d.m[0] > kFill2dWideRows) return hipErrorInvalidValue;
  if (ip.hi[1] < ip.lo[1]) return hipSuccess;
  if (wide) {
    // no prefetch: its registers beside eight rows' sums would spill
    if (form == IGS_MASS)
      launch_fill2d_q<IGS_MASS, kFill2dWideR, T, false, false>(ip, d, nt, lds, dsl, coef, band, s);
    else
      launch_fill2d_q<IGS_STIFFNESS, kFill2dWideR, T, false, false>(ip, d, nt, lds, dsl, coef, band, s);
  } else {
    if (form == IGS_MASS)
      launch_fill2d_pf<IGS_MASS, kFill2dR, T, true>(ip, d, nt, lds, dsl, coef, band, s);
    else
      launch_fill2d_pf<IGS_STIFFNESS, kFill2dR, T, true>(ip, d, nt, lds, dsl, coef, band, s);
  }
  return hipGetLastError();
}

template hipError_t launch_fill2d<double>(const KInterp<double>&, int, const Dims&, const int4*, const double*,
                                          double*, hipStream_t);
template hipError_t launch_fill2d<float>(const KInterp<float>&, int, const Dims&, const int4*, const double*, float*,
                                         hipStream_t);

}  // namespace igs
