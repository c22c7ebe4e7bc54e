// Spline fit of the surrogate (Sec. 4.1) for large sample counts: the passes
// c = (G_n^-1 x ... x G_1^-1) V as tiled FP64 matrix products.  The dense
// per-output passes of fill.hip read each input value once per output along
// the contracted direction; at S ~ 255 samples that traffic through L2 bounds
// the fit.  Here a workgroup computes a 64 x 64 block of a pass with its
// operands staged in LDS in slices of 16 along the contracted index, so every
// staged value serves 64 outputs.
#include <algorithm>

#include "igs_internal.h"

namespace igs {

namespace {

constexpr int kTM = 64, kTN = 64, kTK = 16;

// C[o][i][c] = sum_j A[o][i][j] B[o][j][c] for i < rows, c < cols, j < K, with
// arbitrary element strides (a zero batch stride shares an operand).  a_jfast
// / b_jfast pick the staging order so that consecutive lanes read consecutive
// addresses (the operand's unit stride is along j, or along i / c).
__global__ void __launch_bounds__(256)
    fit_gemm_kernel(int rows, int cols, int K, const double* __restrict__ A, int64_t sAo, int64_t sAi, int64_t sAj,
                    bool a_jfast, const double* __restrict__ B, int64_t sBo, int64_t sBj, int64_t sBc, bool b_jfast,
                    double* __restrict__ C, int64_t sCo, int64_t sCi, int64_t sCc) {
  __shared__ double As[kTK][kTM + 1];
  __shared__ double Bs[kTK][kTN + 1];
  const int64_t o = blockIdx.z;
  const int i0 = blockIdx.y * kTM, c0 = blockIdx.x * kTN;
  A += o * sAo;
  B += o * sBo;
  C += o * sCo;
  const int tid = threadIdx.x;
  const int ti = tid / 16, tc = tid % 16;  // rows ti*4 .. ti*4+3, columns tc + 16 q
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[r][q] = 0.0;

  for (int j0 = 0; j0 < K; j0 += kTK) {
    for (int e = tid; e < kTK * kTM; e += 256) {
      const int jj = a_jfast ? e % kTK : e / kTM;
      const int ii = a_jfast ? e / kTK : e % kTM;
      const int i = i0 + ii, j = j0 + jj;
      As[jj][ii] = (i < rows && j < K) ? A[i * sAi + j * sAj] : 0.0;
    }
    for (int e = tid; e < kTK * kTN; e += 256) {
      const int jj = b_jfast ? e % kTK : e / kTN;
      const int cc = b_jfast ? e / kTK : e % kTN;
      const int c = c0 + cc, j = j0 + jj;
      Bs[jj][cc] = (c < cols && j < K) ? B[j * sBj + c * sBc] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int jj = 0; jj < kTK; ++jj) {
      double a[4], bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[jj][ti * 4 + r];
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[q] = Bs[jj][tc + 16 * q];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] += a[r] * bv[q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + ti * 4 + r, c = c0 + tc + 16 * q;
      if (i < rows && c < cols) C[i * sCi + c * sCc] = acc[r][q];
    }
}

// V[b][u][k3][k2][k1] = band value of upper slot u at sample row (k1, k2, k3)
template <typename BT>
__global__ void fit_gather_kernel(KInterp<double> ip, int n, int m1, int m2, int64_t ld, int S, int batch,
                                  const BT* __restrict__ band, double* __restrict__ V) {
  const int S1 = ip.Sd[0], S2 = ip.Sd[1], S3 = (n == 3) ? ip.Sd[2] : 1;
  const int64_t total = int64_t(S1) * S2 * S3 * ip.nup * batch;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    int64_t r = t;
    const int k1 = int(r % S1);
    r /= S1;
    const int k2 = int(r % S2);
    r /= S2;
    const int k3 = int(r % S3);
    r /= S3;
    const int u = int(r % ip.nup);
    const int b = int(r / ip.nup);
    const size_t row = size_t(ip.samp[0][k1]) +
                       size_t(m1) * (ip.samp[1][k2] + size_t(m2) * (n == 3 ? ip.samp[2][k3] : 0));
    V[t] = double(band[(size_t(b) * S + ip.upslot[u]) * ld + row]);
  }
}

hipError_t gemm(int nbatch, int rows, int cols, int K, const double* A, int64_t sAo, int64_t sAi, int64_t sAj,
                const double* B, int64_t sBo, int64_t sBj, int64_t sBc, double* C, int64_t sCo, int64_t sCi,
                int64_t sCc, hipStream_t s) {
  if (nbatch <= 0 || rows <= 0 || cols <= 0) return hipSuccess;
  if (nbatch > 65535 || (rows + kTM - 1) / kTM > 65535) return hipErrorInvalidValue;
  dim3 grid((cols + kTN - 1) / kTN, (rows + kTM - 1) / kTM, nbatch);
  hipLaunchKernelGGL(fit_gemm_kernel, grid, dim3(256), 0, s, rows, cols, K, A, sAo, sAi, sAj, sAj == 1, B, sBo, sBj,
                     sBc, sBj == 1, C, sCo, sCi, sCc);
  return hipGetLastError();
}

}  // namespace

// The fit runs as tiled products when some direction has at least 192
// samples (and the product batches fit a launch's z extent).  Measured in 2D
// at 1024^2 elements, q = 5: 255 samples 0.36 -> 0.15 ms, but 128 samples
// 0.069 -> 0.086 ms and 79 samples 0.026 -> 0.052 ms (three launches and
// mostly empty 64 x 64 tiles against the per-output passes).
bool fit_use_gemm(const KInterp<double>& ip, int n, int batch) {
  int smax = 0;
  for (int d = 0; d < n; ++d) smax = std::max(smax, ip.Sd[d]);
  const int64_t b2 = int64_t(ip.nup) * batch * (n == 3 ? ip.Sd[2] : 1);
  return smax >= 192 && b2 <= 65535;
}

// Same contract as launch_fit: coefficients into `coef` ([batch][nup][S3][S2][S1]);
// tmp0 and tmp1 are scratch of the same size.  ginv[d] row-major [Sd][Sd].
template <typename BT>
hipError_t launch_fit_gemm(const KInterp<double>& ip, int n, int m1, int m2, int64_t ld, int S, int batch,
                           const BT* band, double* tmp0, double* tmp1, double* coef, hipStream_t s) {
  const int S1 = ip.Sd[0], S2 = ip.Sd[1], S3 = (n == 3) ? ip.Sd[2] : 1;
  const int64_t per = int64_t(S1) * S2 * S3;
  const int64_t total = per * ip.nup * batch;
  // buffers: gather -> g, direction 1 -> p0, direction 2 -> p1, direction 3 -> coef
  double* g = (n == 3) ? coef : tmp1;
  double* p0 = tmp0;
  double* p1 = (n == 3) ? tmp1 : coef;
  const int blocks = int(std::min<int64_t>((total + 255) / 256, 65535));
  hipLaunchKernelGGL((fit_gather_kernel<BT>), dim3(blocks), dim3(256), 0, s, ip, n, m1, m2, ld, S, batch, band, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // direction 1: rows = all lines (b, u, k3, k2), C[line][k1] = sum_j V[line][j] G1[k1][j]
  const int64_t lines = total / S1;
  for (int64_t l0 = 0; l0 < lines; l0 += int64_t(65535) * kTM) {
    const int nl = int(std::min<int64_t>(lines - l0, int64_t(65535) * kTM));
    e = gemm(1, nl, S1, S1, g + l0 * S1, 0, S1, 1, ip.ginv[0], 0, 1, S1, p0 + l0 * S1, 0, S1, 1, s);
    if (e != hipSuccess) return e;
  }
  // direction 2: per (b, u, k3), C[k2][k1] = sum_j G2[k2][j] X[j][k1]
  e = gemm(int(total / (int64_t(S1) * S2)), S2, S1, S2, ip.ginv[1], 0, S2, 1, p0, int64_t(S1) * S2, S1, 1, p1,
           int64_t(S1) * S2, S1, 1, s);
  if (e != hipSuccess || n == 2) return e;
  // direction 3: per (b, u), C[k3][c] = sum_j G3[k3][j] X[j][c], c over (k2, k1)
  return gemm(int(total / per), S3, S1 * S2, S3, ip.ginv[2], 0, S3, 1, p1, per, int64_t(S1) * S2, 1, coef, per,
              int64_t(S1) * S2, 1, s);
}

template hipError_t launch_fit_gemm<double>(const KInterp<double>&, int, int, int, int64_t, int, int, const double*,
                                            double*, double*, double*, hipStream_t);
template hipError_t launch_fit_gemm<float>(const KInterp<double>&, int, int, int, int64_t, int, int, const float*,
                                           double*, double*, double*, hipStream_t);

}  // namespace igs
