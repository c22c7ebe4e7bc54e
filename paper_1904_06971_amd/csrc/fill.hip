// Surrogate interpolation: fit and fill kernels (Secs. 4.1, 5, 8).
//
// fit:  for every interpolated ("upper") stencil delta, the sample values
//       V_delta[k] = A_{s(k), s(k)+delta} (read from the band rows that the
//       quadrature kernel wrote) become tensor spline coefficients
//       c_delta = (G_n^-1 x ... x G_1^-1) V_delta, one direction per pass.
// fill: every analysis-domain row gets, for each upper delta, Phi~_delta at
//       its own index (upper entry) and at the index of its lower partner
//       (lower entry, eq. 5.1b/5.1c copy rule), or the exact entry of the
//       boundary row when the partner leaves the analysis domain; the
//       stiffness diagonal is minus the sum of the row (eq. 5.1c).  A
//       workgroup evaluates the interpolant separably on its tile (plus the
//       halo that the lower entries need) through two LDS stages and writes
//       each band slot of its rows exactly once, stencil-major and coalesced.
#include "igs_internal.h"

namespace igs {

// ------------------------------------------------------------------ fit ----

// out[b][u][..k_d..] = sum_j ginv_d[k_d][j] in[b][u][..j..]; pass 0 gathers
// `in` from the band at the sample rows.
template <typename BT, bool GATHER>
__global__ void fit_pass_kernel(KInterp<double> ip, int d, int n, int m1, int m2, int64_t ld, int S, int batch,
                                const BT* __restrict__ band, const double* __restrict__ in, double* __restrict__ out) {
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
    const double* g = ip.ginv[d] + size_t(kd) * Sd;
    double acc = 0.0;
    if constexpr (GATHER) {
      const BT* bs = band + (size_t(b) * S + ip.upslot[u]) * ld;
      const size_t rowbase = size_t(m1) * (ip.samp[1][k2] + size_t(m2) * (n == 3 ? ip.samp[2][k3] : 0));
      for (int j = 0; j < Sd; ++j) acc += g[j] * double(bs[rowbase + ip.samp[0][j]]);
    } else {
      const double* src = in + (size_t(b) * ip.nup + u) * per;
      for (int j = 0; j < Sd; ++j) {
        const int a1 = (d == 0) ? j : k1, a2 = (d == 1) ? j : k2, a3 = (d == 2) ? j : k3;
        acc += g[j] * src[(size_t(a3) * S2 + a2) * S1 + a1];
      }
    }
    out[t] = acc;
  }
}

// ----------------------------------------------------------------- fill ----

constexpr int kFillTX = 64;   // rows along direction 1 per tile (one per lane)
constexpr int kFillTY3 = 4;   // 3D: rows along direction 2 (one per wave)
constexpr int kFillTZ3 = 4;   // 3D: rows along direction 3 (loop)
constexpr int kFillTY2 = 16;  // 2D: rows along direction 2 (4 waves x 4)

template <typename T>
__device__ __forceinline__ T interp1(const T* __restrict__ beta, int q, const T* __restrict__ x, int stride) {
  T v = T(0);
#pragma unroll 6
  for (int c = 0; c <= q; ++c) v += beta[c] * x[c * stride];
  return v;
}

template <int FORM, typename T>
__global__ void __launch_bounds__(256)
    fill3d_kernel(KInterp<T> ip, int P, int m1, int m2, int64_t ld, int S, const double* __restrict__ coef,
                  T* __restrict__ band) {
  extern __shared__ char smem_raw[];
  constexpr int TX = kFillTX, TY = kFillTY3, TZ = kFillTZ3;
  const int W = 2 * P + 1;
  const int q = ip.q;
  const int B1 = TX + P, B2 = TY + P;
  const int nc2 = ip.nc[1], nc3 = ip.nc[2];
  T* X1 = reinterpret_cast<T*>(smem_raw);
  T* X2 = X1 + size_t(nc3) * nc2 * B1;

  const int L1 = ip.hi[0] - ip.lo[0] + 1, L2 = ip.hi[1] - ip.lo[1] + 1;
  const int nt1 = (L1 + TX - 1) / TX, nt2 = (L2 + TY - 1) / TY;
  int bid = blockIdx.x;
  const int t1 = bid % nt1;
  bid /= nt1;
  const int t2 = bid % nt2;
  const int t3 = bid / nt2;
  const int b = blockIdx.y;
  const int A1 = ip.lo[0] + t1 * TX, A2 = ip.lo[1] + t2 * TY, A3 = ip.lo[2] + t3 * TZ;
  const int tid = threadIdx.x;
  const int r1 = tid & 63, r2 = tid >> 6;
  const int i1 = A1 + r1, i2 = A2 + r2;
  const bool row_ok = i1 <= ip.hi[0] && i2 <= ip.hi[1];
  const int S1 = ip.Sd[0], S2 = ip.Sd[1], S3 = ip.Sd[2];
  const size_t per = size_t(S1) * S2 * S3;
  const size_t plane = size_t(m1) * m2;
  T* bnd = band + size_t(b) * S * ld;
  T dsum[TZ];
#pragma unroll
  for (int r = 0; r < TZ; ++r) dsum[r] = T(0);

  for (int u = 0; u < ip.nup; ++u) {
    const int s = ip.upslot[u];
    const int dl1 = s % W - P, dl2 = (s / W) % W - P, dl3 = s / (W * W) - P;
    const int64_t off = dl1 + int64_t(m1) * dl2 + int64_t(plane) * dl3;
    // evaluation box: the tile and the tile shifted by -delta, inside the analysis domain
    const int lo1 = max(ip.lo[0], A1 - max(dl1, 0)), hi1 = min(ip.hi[0], A1 + TX - 1 - min(dl1, 0));
    const int lo2 = max(ip.lo[1], A2 - max(dl2, 0)), hi2 = min(ip.hi[1], A2 + TY - 1 - min(dl2, 0));
    const int lo3 = max(ip.lo[2], A3 - max(dl3, 0)), hi3 = min(ip.hi[2], A3 + TZ - 1 - min(dl3, 0));
    const int c1lo = ip.ef[0][lo1];
    const int c2lo = ip.ef[1][lo2], c2n = ip.ef[1][hi2] + q - c2lo + 1;
    const int c3lo = ip.ef[2][lo3], c3n = ip.ef[2][hi3] + q - c3lo + 1;
    const int b1w = hi1 - lo1 + 1, b2w = hi2 - lo2 + 1;
    (void)c1lo;
    const double* cu = coef + (size_t(b) * ip.nup + u) * per;
    // stage X: direction-1 evaluation of the coefficient block
    for (int t = tid; t < c3n * c2n * b1w; t += 256) {
      const int x = t % b1w;
      const int rr = t / b1w;
      const int c2 = rr % c2n, c3 = rr / c2n;
      const int ii1 = lo1 + x;
      const T* beta = ip.eb[0] + size_t(ii1) * (q + 1);
      const double* crow = cu + (size_t(c3lo + c3) * S2 + c2lo + c2) * S1 + ip.ef[0][ii1];
      T v = T(0);
#pragma unroll 6
      for (int c = 0; c <= q; ++c) v += beta[c] * T(crow[c]);
      X1[(c3 * nc2 + c2) * B1 + x] = v;
    }
    __syncthreads();
    // stage Y: direction 2
    for (int t = tid; t < c3n * b2w * b1w; t += 256) {
      const int x = t % b1w;
      const int rr = t / b1w;
      const int y = rr % b2w, c3 = rr / b2w;
      const int ii2 = lo2 + y;
      const T* beta = ip.eb[1] + size_t(ii2) * (q + 1);
      X2[(c3 * B2 + y) * B1 + x] = interp1<T>(beta, q, X1 + (c3 * nc2 + ip.ef[1][ii2] - c2lo) * B1 + x, B1);
    }
    __syncthreads();
    // stage Z (direction 3, per thread) and the stores
    if (row_ok) {
      const bool up_in1 = i1 + dl1 >= ip.lo[0] && i1 + dl1 <= ip.hi[0];
      const bool up_in2 = i2 + dl2 >= ip.lo[1] && i2 + dl2 <= ip.hi[1];
      const bool lo_in1 = i1 - dl1 >= ip.lo[0] && i1 - dl1 <= ip.hi[0];
      const bool lo_in2 = i2 - dl2 >= ip.lo[1] && i2 - dl2 <= ip.hi[1];
#pragma unroll
      for (int r3 = 0; r3 < TZ; ++r3) {
        const int i3 = A3 + r3;
        if (i3 > ip.hi[2]) continue;
        const size_t idx = size_t(i1) + size_t(m1) * i2 + plane * i3;
        T val;
        if (up_in1 && up_in2 && i3 + dl3 >= ip.lo[2] && i3 + dl3 <= ip.hi[2]) {
          const T* beta = ip.eb[2] + size_t(i3) * (q + 1);
          val = interp1<T>(beta, q, X2 + ((ip.ef[2][i3] - c3lo) * B2 + (i2 - lo2)) * B1 + (i1 - lo1), B2 * B1);
        } else {
          val = bnd[size_t(S - 1 - s) * ld + idx + off];  // exact A_ji of boundary row j = i + delta
        }
        bnd[size_t(s) * ld + idx] = val;
        if (FORM == IGS_STIFFNESS) dsum[r3] += val;
        if (FORM == IGS_STIFFNESS || s != (S - 1) / 2) {
          const int j3 = i3 - dl3;
          if (lo_in1 && lo_in2 && j3 >= ip.lo[2] && j3 <= ip.hi[2]) {
            const T* beta = ip.eb[2] + size_t(j3) * (q + 1);
            val = interp1<T>(beta, q,
                             X2 + ((ip.ef[2][j3] - c3lo) * B2 + (i2 - dl2 - lo2)) * B1 + (i1 - dl1 - lo1), B2 * B1);
          } else {
            val = bnd[size_t(s) * ld + idx - off];  // exact A_{j,j+delta} of boundary row j = i - delta
          }
          bnd[size_t(S - 1 - s) * ld + idx] = val;
          if (FORM == IGS_STIFFNESS) dsum[r3] += val;
        }
      }
    }
  }
  if (FORM == IGS_STIFFNESS && row_ok) {
#pragma unroll
    for (int r3 = 0; r3 < TZ; ++r3) {
      const int i3 = A3 + r3;
      if (i3 > ip.hi[2]) continue;
      bnd[size_t((S - 1) / 2) * ld + size_t(i1) + size_t(m1) * i2 + plane * i3] = -dsum[r3];
    }
  }
}

template <int FORM, typename T>
__global__ void __launch_bounds__(256)
    fill2d_kernel(KInterp<T> ip, int P, int m1, int64_t ld, int S, const double* __restrict__ coef,
                  T* __restrict__ band) {
  extern __shared__ char smem_raw[];
  constexpr int TX = kFillTX, TY = kFillTY2, RY = TY / 4;
  const int W = 2 * P + 1;
  const int q = ip.q;
  const int B1 = TX + P;
  T* X1 = reinterpret_cast<T*>(smem_raw);
  const int L1 = ip.hi[0] - ip.lo[0] + 1;
  const int nt1 = (L1 + TX - 1) / TX;
  const int t1 = blockIdx.x % nt1, t2 = blockIdx.x / nt1;
  const int b = blockIdx.y;
  const int A1 = ip.lo[0] + t1 * TX, A2 = ip.lo[1] + t2 * TY;
  const int tid = threadIdx.x;
  const int r1 = tid & 63, w = tid >> 6;
  const int i1 = A1 + r1;
  const bool col_ok = i1 <= ip.hi[0];
  const int S1 = ip.Sd[0], S2 = ip.Sd[1];
  const size_t per = size_t(S1) * S2;
  T* bnd = band + size_t(b) * S * ld;
  T dsum[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) dsum[r] = T(0);

  for (int u = 0; u < ip.nup; ++u) {
    const int s = ip.upslot[u];
    const int dl1 = s % W - P, dl2 = s / W - P;
    const int64_t off = dl1 + int64_t(m1) * dl2;
    const int lo1 = max(ip.lo[0], A1 - max(dl1, 0)), hi1 = min(ip.hi[0], A1 + TX - 1 - min(dl1, 0));
    const int lo2 = max(ip.lo[1], A2 - max(dl2, 0)), hi2 = min(ip.hi[1], A2 + TY - 1 - min(dl2, 0));
    const int c2lo = ip.ef[1][lo2], c2n = ip.ef[1][hi2] + q - c2lo + 1;
    const int b1w = hi1 - lo1 + 1;
    const double* cu = coef + (size_t(b) * ip.nup + u) * per;
    for (int t = tid; t < c2n * b1w; t += 256) {
      const int x = t % b1w, c2 = t / b1w;
      const int ii1 = lo1 + x;
      const T* beta = ip.eb[0] + size_t(ii1) * (q + 1);
      const double* crow = cu + size_t(c2lo + c2) * S1 + ip.ef[0][ii1];
      T v = T(0);
#pragma unroll 6
      for (int c = 0; c <= q; ++c) v += beta[c] * T(crow[c]);
      X1[c2 * B1 + x] = v;
    }
    __syncthreads();
    if (col_ok) {
      const bool up_in1 = i1 + dl1 >= ip.lo[0] && i1 + dl1 <= ip.hi[0];
      const bool lo_in1 = i1 - dl1 >= ip.lo[0] && i1 - dl1 <= ip.hi[0];
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const int i2 = A2 + w + 4 * r;
        if (i2 > ip.hi[1]) continue;
        const size_t idx = size_t(i1) + size_t(m1) * i2;
        T val;
        if (up_in1 && i2 + dl2 >= ip.lo[1] && i2 + dl2 <= ip.hi[1]) {
          const T* beta = ip.eb[1] + size_t(i2) * (q + 1);
          val = interp1<T>(beta, q, X1 + (ip.ef[1][i2] - c2lo) * B1 + (i1 - lo1), B1);
        } else {
          val = bnd[size_t(S - 1 - s) * ld + idx + off];
        }
        bnd[size_t(s) * ld + idx] = val;
        if (FORM == IGS_STIFFNESS) dsum[r] += val;
        if (FORM == IGS_STIFFNESS || s != (S - 1) / 2) {
          const int j2 = i2 - dl2;
          if (lo_in1 && j2 >= ip.lo[1] && j2 <= ip.hi[1]) {
            const T* beta = ip.eb[1] + size_t(j2) * (q + 1);
            val = interp1<T>(beta, q, X1 + (ip.ef[1][j2] - c2lo) * B1 + (i1 - dl1 - lo1), B1);
          } else {
            val = bnd[size_t(s) * ld + idx - off];
          }
          bnd[size_t(S - 1 - s) * ld + idx] = val;
          if (FORM == IGS_STIFFNESS) dsum[r] += val;
        }
      }
    }
    __syncthreads();
  }
  if (FORM == IGS_STIFFNESS && col_ok) {
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int i2 = A2 + w + 4 * r;
      if (i2 > ip.hi[1]) continue;
      bnd[size_t((S - 1) / 2) * ld + size_t(i1) + size_t(m1) * i2] = -dsum[r];
    }
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

// ------------------------------------------------------------ launchers ----

void fill_tile_box(int n, int p, int box[3]) {
  box[0] = kFillTX + p;
  box[1] = (n == 3 ? kFillTY3 : kFillTY2) + p;
  box[2] = kFillTZ3 + p;
}

template <typename BT>
hipError_t launch_fit(const KInterp<double>& ip, int n, int m1, int m2, int64_t ld, int S, int batch, const BT* band,
                      double* tmp0, double* tmp1, double* coef, hipStream_t s) {
  int64_t total = int64_t(ip.Sd[0]) * ip.Sd[1] * (n == 3 ? ip.Sd[2] : 1) * ip.nup * batch;
  int blocks = int(std::min<int64_t>((total + 255) / 256, 65535));
  double* bufs[3];
  if (n == 3) {
    bufs[0] = tmp0; bufs[1] = tmp1; bufs[2] = coef;
  } else {
    bufs[0] = tmp0; bufs[1] = coef; bufs[2] = nullptr;
  }
  hipLaunchKernelGGL((fit_pass_kernel<BT, true>), dim3(blocks), dim3(256), 0, s, ip, 0, n, m1, m2, ld, S, batch, band,
                     nullptr, bufs[0]);
  for (int d = 1; d < n; ++d)
    hipLaunchKernelGGL((fit_pass_kernel<BT, false>), dim3(blocks), dim3(256), 0, s, ip, d, n, m1, m2, ld, S, batch,
                       band, bufs[d - 1], bufs[d]);
  return hipGetLastError();
}

template hipError_t launch_fit<double>(const KInterp<double>&, int, int, int, int64_t, int, int, const double*,
                                       double*, double*, double*, hipStream_t);
template hipError_t launch_fit<float>(const KInterp<double>&, int, int, int, int64_t, int, int, const float*,
                                      double*, double*, double*, hipStream_t);

template <typename T>
size_t fill_lds_bytes(const KInterp<T>& ip, int n, int p) {
  if (n == 3) return (size_t(ip.nc[2]) * ip.nc[1] * (kFillTX + p) + size_t(ip.nc[2]) * (kFillTY3 + p) * (kFillTX + p)) * sizeof(T);
  return size_t(ip.nc[1]) * (kFillTX + p) * sizeof(T);
}

template <typename T>
hipError_t launch_fill(const KInterp<T>& ip, int form, int n, int p, int m1, int m2, int64_t ld, int S, int batch,
                       const double* coef, T* band, hipStream_t s) {
  const int L1 = ip.hi[0] - ip.lo[0] + 1, L2 = ip.hi[1] - ip.lo[1] + 1;
  const size_t lds = fill_lds_bytes<T>(ip, n, p);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (n == 3) {
    const int L3 = ip.hi[2] - ip.lo[2] + 1;
    const int tiles = ((L1 + kFillTX - 1) / kFillTX) * ((L2 + kFillTY3 - 1) / kFillTY3) * ((L3 + kFillTZ3 - 1) / kFillTZ3);
    dim3 grid(tiles, batch);
    if (form == IGS_MASS)
      hipLaunchKernelGGL((fill3d_kernel<IGS_MASS, T>), grid, dim3(256), lds, s, ip, p, m1, m2, ld, S, coef, band);
    else
      hipLaunchKernelGGL((fill3d_kernel<IGS_STIFFNESS, T>), grid, dim3(256), lds, s, ip, p, m1, m2, ld, S, coef, band);
  } else {
    const int tiles = ((L1 + kFillTX - 1) / kFillTX) * ((L2 + kFillTY2 - 1) / kFillTY2);
    dim3 grid(tiles, batch);
    if (form == IGS_MASS)
      hipLaunchKernelGGL((fill2d_kernel<IGS_MASS, T>), grid, dim3(256), lds, s, ip, p, m1, ld, S, coef, band);
    else
      hipLaunchKernelGGL((fill2d_kernel<IGS_STIFFNESS, T>), grid, dim3(256), lds, s, ip, p, m1, ld, S, coef, band);
  }
  return hipGetLastError();
}

template hipError_t launch_fill<double>(const KInterp<double>&, int, int, int, int, int, int64_t, int, int,
                                        const double*, double*, hipStream_t);
template hipError_t launch_fill<float>(const KInterp<float>&, int, int, int, int, int, int64_t, int, int,
                                       const double*, float*, hipStream_t);
template size_t fill_lds_bytes<double>(const KInterp<double>&, int, int);
template size_t fill_lds_bytes<float>(const KInterp<float>&, int, int);

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
