// Quadrature kernels: exact stiffness / mass rows and the load vector.
//
// A row i of the stiffness matrix holds A_{i,i+delta} = int grad B_i^T K grad
// B_{i+delta} over supp B_i (Sec. 3.2, eqs. BilinearFormPoissonTensor,
// ChangeOfVars).  The tensor-product structure B_i = prod_d b_{i_d} turns the
// sum over Gauss points into per-direction contractions (sum factorisation):
//   stage 1: contract the direction-1 points into (i1, delta1) pairs,
//   stage 2: contract the direction-2 points into (i2, delta2) pairs,
//   stage 3: contract the direction-3 points into (i3, delta3) pairs.
// A workgroup owns a tile of rows (TX x TY in (i1, i2)) and streams through
// the element layers of the last direction; each layer's Gauss points update
// a rolling window of p+1 rows held in registers, and a row is written out
// (stencil-major, one writer per band slot, no atomics) as soon as its last
// layer has been processed.  Geometry (Jacobian, determinant, K) is
// recomputed at the points of the tile's footprint and staged in LDS.
#include <cstdio>

#include "igs_internal.h"

namespace igs {

template <int N>
struct IntC {
  static constexpr int value = N;
};

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(IntC<B>{});
    static_for<B + 1, E>(f);
  }
}

// ------------------------------------------------------------- geometry ----

// Jacobian J[r][c] = dF_r/dxi_c of the geometry map at a Gauss point.
template <int ND>
__device__ __forceinline__ void jacobian(const KProblem& kp, const int* g, const double* xi, double J[ND][ND]) {
#pragma unroll
  for (int r = 0; r < ND; ++r)
#pragma unroll
    for (int c = 0; c < ND; ++c) J[r][c] = (r == c) ? 1.0 : 0.0;
  const double a = kp.ga;
  if (kp.geom == IGS_GEOM_SINE) {
    double s1[ND], c1[ND], s2[ND], c2[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const double* tr = kp.t[d].trig + 4 * g[d];
      s1[d] = tr[0];
      c1[d] = tr[1];
      s2[d] = tr[2];
      c2[d] = tr[3];
    }
    if constexpr (ND == 2) {
      J[0][0] += a * c1[0] * s2[1];
      J[0][1] += a * s1[0] * c2[1];
      J[1][0] += a * c2[0] * s1[1];
      J[1][1] += a * s2[0] * c1[1];
    } else {
      J[0][0] += a * c1[0] * s2[1] * s1[2];
      J[0][1] += a * s1[0] * c2[1] * s1[2];
      J[0][2] += a * s1[0] * s2[1] * c1[2];
      J[1][0] += a * c2[0] * s1[1] * s1[2];
      J[1][1] += a * s2[0] * c1[1] * s1[2];
      J[1][2] += a * s2[0] * s1[1] * c1[2];
      J[2][0] += a * c1[0] * s1[1] * s2[2];
      J[2][1] += a * s1[0] * c1[1] * s2[2];
      J[2][2] += a * s1[0] * s1[1] * c2[2];
    }
  } else if (kp.geom == IGS_GEOM_POLY2) {
    double q[ND], dq[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      q[d] = xi[d] * (1.0 - xi[d]);
      dq[d] = 1.0 - 2.0 * xi[d];
    }
#pragma unroll
    for (int c = 0; c < ND; ++c) {
      double dprod = dq[c];
#pragma unroll
      for (int d = 0; d < ND; ++d)
        if (d != c) dprod *= q[d];
#pragma unroll
      for (int r = 0; r < ND; ++r) J[r][c] += a * (r + 1) * dprod;
    }
  }
}

// Physical point F(xi) (needed only by the SINE3 coefficient).
template <int ND>
__device__ __forceinline__ void phys_point(const KProblem& kp, const int* g, const double* xi, double* F) {
#pragma unroll
  for (int d = 0; d < ND; ++d) F[d] = xi[d];
  const double a = kp.ga;
  if (kp.geom == IGS_GEOM_SINE) {
    double s1[ND], s2[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      s1[d] = kp.t[d].trig[4 * g[d]];
      s2[d] = kp.t[d].trig[4 * g[d] + 2];
    }
    if constexpr (ND == 2) {
      F[0] += a * s1[0] * s2[1];
      F[1] += a * s2[0] * s1[1];
    } else {
      F[0] += a * s1[0] * s2[1] * s1[2];
      F[1] += a * s2[0] * s1[1] * s1[2];
      F[2] += a * s1[0] * s1[1] * s2[2];
    }
  } else if (kp.geom == IGS_GEOM_POLY2) {
    double prod = 1.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) prod *= xi[d] * (1.0 - xi[d]);
#pragma unroll
    for (int r = 0; r < ND; ++r) F[r] += a * (r + 1) * prod;
  }
}

// g(xi) = sum_k c_k N_k(xi) for the coefficient spline of problem b.
template <int ND>
__device__ __forceinline__ double coef_spline(const KProblem& kp, int b, const int* g) {
  const double* cc = kp.cc + b * kp.cstride;
  const int nd = kp.cdeg + 1;
  const double* cb0 = kp.t[0].cb + g[0] * nd;
  const double* cb1 = kp.t[1].cb + g[1] * nd;
  const int f0 = kp.t[0].cf[g[0]], f1 = kp.t[1].cf[g[1]];
  double s = 0.0;
  if constexpr (ND == 2) {
    for (int a1 = 0; a1 < nd; ++a1) {
      double r = 0.0;
      const double* row = cc + (f1 + a1) * kp.cn[0] + f0;
      for (int a0 = 0; a0 < nd; ++a0) r += cb0[a0] * row[a0];
      s += cb1[a1] * r;
    }
  } else {
    const double* cb2 = kp.t[2].cb + g[2] * nd;
    const int f2 = kp.t[2].cf[g[2]];
    for (int a2 = 0; a2 < nd; ++a2) {
      double r2 = 0.0;
      for (int a1 = 0; a1 < nd; ++a1) {
        double r = 0.0;
        const double* row = cc + ((f2 + a2) * kp.cn[1] + f1 + a1) * kp.cn[0] + f0;
        for (int a0 = 0; a0 < nd; ++a0) r += cb0[a0] * row[a0];
        r2 += cb1[a1] * r;
      }
      s += cb2[a2] * r2;
    }
  }
  return s;
}

template <int ND>
__device__ __forceinline__ double kappa_at(const KProblem& kp, int b, const int* g, const double* xi) {
  switch (kp.coef) {
    case IGS_COEF_SINE3: {
      double F[ND];
      phys_point<ND>(kp, g, xi, F);
      // sin(2 pi x) as sinpi(2x): a reduction without the large-argument
      // path (no private-memory table) and no rounding of 2 pi x
      double v = sinpi(2.0 * F[0]) * cospi(2.0 * F[1]);
      if constexpr (ND == 3) v *= sinpi(2.0 * F[2]);
      return kp.c0 + kp.camp * v;
    }
    case IGS_COEF_SPLINE:
      return coef_spline<ND>(kp, b, g);
    case IGS_COEF_EXP_SPLINE:
      return exp(coef_spline<ND>(kp, b, g));
    default:
      return kp.c0;
  }
}

// Integrand data at one Gauss point: the symmetric K scaled by weight*kappa
// (K = kappa |det J| J^-1 J^-T = kappa adj(J) adj(J)^T / |det J|) or the
// mass weight w |det J|.  Flags det J <= 0.  VC = false: the coefficient is the
// constant c0 (no coefficient code in the kernel).
template <int ND, int FORM, bool VC = true>
__device__ __forceinline__ void point_data(const KProblem& kp, int b, const int* g, double* out) {
  double xi[ND], w = 1.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    xi[d] = kp.t[d].x[g[d]];
    w *= kp.t[d].w[g[d]];
  }
  double J[ND][ND];
  jacobian<ND>(kp, g, xi, J);
  double adj[ND][ND], det;
  if constexpr (ND == 2) {
    adj[0][0] = J[1][1];
    adj[0][1] = -J[0][1];
    adj[1][0] = -J[1][0];
    adj[1][1] = J[0][0];
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  } else {
    adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
  }
  if (!(det > 0.0)) atomicOr(kp.flag, 1);
  const double ad = fabs(det);
  if constexpr (FORM == IGS_MASS) {
    out[0] = w * ad;
  } else {
    const double s = w * (VC ? kappa_at<ND>(kp, b, g, xi) : kp.c0) / ad;
    int k = 0;
#pragma unroll
    for (int r = 0; r < ND; ++r)
#pragma unroll
      for (int c = r; c < ND; ++c) {
        double v = 0.0;
#pragma unroll
        for (int e = 0; e < ND; ++e) v += adj[r][e] * adj[c][e];
        out[k++] = s * v;
      }
  }
}

// Read-only table viewed in the constant address space: loads at wave-uniform
// addresses then go through the scalar cache into SGPRs.
typedef const __attribute__((address_space(4))) double* cdptr;
__device__ __forceinline__ cdptr uniform_table(const double* p) { return (cdptr)p; }

template <int P>
struct Q3BShape;
template <> struct Q3BShape<1> { static constexpr int TY = 5; };
template <> struct Q3BShape<2> { static constexpr int TY = 3; };
template <> struct Q3BShape<3> { static constexpr int TY = 2; };
template <> struct Q3BShape<4> { static constexpr int TY = 1; };

// Stage-1 wave tasks.  A task fixes i1 and one of three product modes; its
// lanes hold (component, l2).  Codes written to Ys (pair, half):
//   0 dd.K11  1 dv.K12 | 2 dv.K13  3 vd.K12 | 4 vd.K13  5 vv.K22 | 6 vv.K23  7 vv.K33
// (d/v = derivative/value of the i- and j-function in direction 1).
//   S1_DDV  components K11, K12, K13: dd (kept for K11) and dv (kept for K12, K13)
//   S1_VD   components K12, K13: vd
//   S1_VV   components K22, K23, K33 (or the mass weight): vv
enum { S1_DDV = 0, S1_VD = 1, S1_VV = 2 };

template <int P, int FORM>
struct Q3B {
  static constexpr int NQ = P + 1, W = 2 * P + 1;
  static constexpr int TX = 64 / W, TY = Q3BShape<P>::TY;
  static constexpr int NWAVE = TY * W;
  static constexpr int BLOCK = 64 * NWAVE;
  // direction-2 elements held in LDS at a time.  Up to p = 3 the tile's whole
  // footprint (TY + P elements); at p = 4 the five elements of a row's
  // footprint would need more LDS than a CU has (Cs and Ys together about
  // 171 KB), so each Gauss plane is taken in groups of up to three elements.
  static constexpr int EG2 = P <= 3 ? TY + P : 3;
  static constexpr int NG2 = (TY + P + EG2 - 1) / EG2;  // groups per plane (at most)
  static constexpr int NQ1 = (TX + P) * NQ, NQ2 = EG2 * NQ;
  static constexpr bool STIFF = FORM == IGS_STIFFNESS;
  static constexpr int NC = STIFF ? 6 : 1;
  static constexpr int NMODE = STIFF ? 3 : 1;
  // Cs component stride, congruent to NQ2 mod 32: lanes (component, l2) of a
  // stage-1 wave then address consecutive banks
  static constexpr int CS = (NQ1 * NQ2 + 31) / 32 * 32 + NQ2 % 32;
  static constexpr int NPAIR = STIFF ? 4 : 1;  // Y codes, two per double2
  static constexpr int YL = 65;                // odd lane pitch (double2) of Ys
  static_assert(3 * NQ2 <= 64, "stage-1 lanes");
};

// Direction-1 contraction of one component column for one wave-uniform i1.
// MODE S1_DDV: y0 = dd, y1 = dv;  S1_VD: y0 = vd;  S1_VV: y0 = vv.
// cb points at the lane's component value at l1 = 0, ls is the l1 stride.
// The basis values are wave-uniform and come through scalar loads; they are
// fetched for a batch of NB Gauss points at once (all of an element's points
// for the vd and vv products, half of them for dd/dv, which need both value
// and derivative rows) so that one wait covers the whole batch.
template <int P, int MODE>
__device__ __forceinline__ void stage1_core(const KProblem& kp, const double* cb, int ls, int i1, int E1a,
                                            double* y0, double* y1) {
  constexpr int NQ = P + 1, W = 2 * P + 1, NP = P + 1;
  // points per batch (their basis rows live in SGPRs: at p = 4 smaller batches)
  constexpr int NB = MODE == S1_DDV ? (P <= 3 ? (NQ + 1) / 2 : 2) : (P <= 3 ? NQ : 3);
#pragma unroll
  for (int d = 0; d < W; ++d) y0[d] = y1[d] = 0.0;
  const int nel1 = kp.nelem[0];
  cdptr tv = uniform_table(kp.t[0].bv), td = uniform_table(kp.t[0].bd);
#pragma unroll
  for (int a = 0; a <= P; ++a) {
    const int e1 = i1 - a;
    if (e1 < 0 || e1 >= nel1) continue;
    const size_t g0 = size_t(e1) * NQ;
    const double* cp = cb + (e1 - E1a) * NQ * ls;
#pragma unroll
    for (int k0 = 0; k0 < NQ; k0 += NB) {
      // batch loads: TB rows (values or derivatives of the p+1 functions) and ta
      double tb[NB][NP], tb2[NB][NP], ta[NB], c[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (k0 + k >= NQ) break;
        const size_t g = g0 + k0 + k;
#pragma unroll
        for (int b = 0; b < NP; ++b) {
          if constexpr (MODE == S1_DDV) {
            tb[k][b] = td[g * NP + b];
            tb2[k][b] = tv[g * NP + b];
          } else if constexpr (MODE == S1_VD) {
            tb[k][b] = td[g * NP + b];
          } else {
            tb[k][b] = tv[g * NP + b];
          }
        }
        if constexpr (MODE == S1_VD) ta[k] = tv[g * NP + a];
        c[k] = cp[(k0 + k) * ls];
      }
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (k0 + k >= NQ) break;
        if constexpr (MODE == S1_DDV) {
          const double u = tb[k][a] * c[k];
#pragma unroll
          for (int b = 0; b <= P; ++b) {
            y0[b - a + P] += u * tb[k][b];
            y1[b - a + P] += u * tb2[k][b];
          }
        } else if constexpr (MODE == S1_VD) {
          const double u = ta[k] * c[k];
#pragma unroll
          for (int b = 0; b <= P; ++b) y0[b - a + P] += u * tb[k][b];
        } else {
          const double u = tb[k][a] * c[k];
#pragma unroll
          for (int b = 0; b <= P; ++b) y0[b - a + P] += u * tb[k][b];
        }
      }
    }
  }
}

// Lane -> (component, code) of a stage-1 task; ok = false for idle lanes.
template <int MODE, bool STIFF>
__device__ __forceinline__ void stage1_slot(int cl, int* comp, int* code0, int* code1, bool* ok) {
  if constexpr (!STIFF) {
    *ok = *ok && cl == 0;
    *comp = 0;
    *code0 = 0;
    *code1 = -1;
  } else if constexpr (MODE == S1_DDV) {
    *ok = *ok && cl < 3;
    *comp = cl;
    *code0 = cl == 0 ? 0 : -1;  // dd.K11
    *code1 = cl == 0 ? -1 : cl;  // dv.K12, dv.K13
  } else if constexpr (MODE == S1_VD) {
    *ok = *ok && cl < 2;
    *comp = 1 + cl;
    *code0 = 3 + cl;  // vd.K12, vd.K13
    *code1 = -1;
  } else {
    *ok = *ok && cl < 3;
    *comp = 3 + cl;
    *code0 = 5 + cl;  // vv.K22, vv.K23, vv.K33
    *code1 = -1;
  }
  if (!*ok) *comp = 0;
}

template <int P, int FORM, int MODE>
__device__ __forceinline__ void stage1_b(const KProblem& kp, const double* __restrict__ Cs,
                                         double* __restrict__ Ysd, int i1, int r1, int E1a, int nq2, int lane) {
  using C = Q3B<P, FORM>;
  constexpr int W = C::W, TX = C::TX, NQ2 = C::NQ2;
  const int cl = lane / NQ2, l2 = lane - cl * NQ2;
  bool ok = l2 < nq2;
  int comp, code0, code1;
  stage1_slot<MODE, C::STIFF>(cl, &comp, &code0, &code1, &ok);
  double y0[W], y1[W];
  stage1_core<P, MODE>(kp, Cs + comp * C::CS + (ok ? l2 : 0), NQ2, i1, E1a, y0, y1);
  if (!ok) return;
  double* row0 = Ysd + ((code0 >> 1) * NQ2 + l2) * (2 * C::YL) + (code0 & 1);
  double* row1 = Ysd + ((code1 >> 1) * NQ2 + l2) * (2 * C::YL) + (code1 & 1);
#pragma unroll
  for (int d1 = 0; d1 < W; ++d1) {
    const int col = 2 * (d1 * TX + r1);
    if (code0 >= 0) row0[col] = y0[d1];
    if (MODE == S1_DDV && code1 >= 0) row1[col] = y1[d1];
  }
}

// ------------------------------------------------ 3-D rows, register-blocked ---
//
// Sum factorisation of the row quadrature, one direction at a time.  Wave
// w owns the direction-2 combination (i2, delta2) = (tile.i2 + w / W, w % W - P)
// and lane l the direction-1 combination (i1, delta1) = (tile.i1 + l % TX,
// l / TX - P): one thread carries one (delta1, delta2) column of a row pencil
// and its window of the P+1 rows that the current element layer touches.
// Row e3 + a of the window has collected delta3 in [-P, P - a] so far, so slot
// a keeps W - a values; after the last plane of layer e3, row e3 is complete,
// is stored, and the window shifts by one row.  Per Gauss plane:
//   stage 1  direction-1 contraction: wave tasks (i1, mode) with wave-uniform
//            basis values (scalar loads), lanes (component, l2); -> Ys
//   stage 2  direction-2 contraction, basis values wave-uniform again, into 4
//            direction-3 codes;
//   stage 3  direction-3 products into the window;
//   phase A  integrand data of the next plane at the footprint points -> Cs
//            (same barrier interval as stages 2-3: they touch other buffers).

template <int P, int FORM, bool VC, typename OutT>
__global__ void __launch_bounds__((Q3B<P, FORM>::BLOCK))
    quad3d_tile_kernel(KProblem kp, const QTile* __restrict__ tiles, OutT* __restrict__ band) {
  using C = Q3B<P, FORM>;
  constexpr int NQ = C::NQ, W = C::W, TX = C::TX, NQ2 = C::NQ2, YL = C::YL;
  __shared__ double Cs[C::NC * C::CS];
  __shared__ double2 Ys[C::NPAIR * NQ2 * YL];
  // work counters: [0] stage-1 tasks, [1] phase-A passes of 64 points.  Waves
  // take the next item as they finish one, so that waves with less stage-2
  // work (large |delta2|) absorb more geometry points and the heavier stage-1
  // tasks (listed first) do not pile up on one SIMD.
  __shared__ int qctr[2];

  const QTile tile = tiles[blockIdx.x];
  const int b = blockIdx.y;
  OutT* out = band + size_t(b) * kp.S * kp.ld;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nel1 = kp.nelem[0], nel2 = kp.nelem[1], nel3 = kp.nelem[2];
  const int E1a = max(0, tile.i1 - P), E1b = min(nel1 - 1, tile.i1 + tile.nx - 1);
  const int E2a = max(0, tile.i2 - P), E2b = min(nel2 - 1, tile.i2 + tile.ny - 1);
  const int nq1 = (E1b - E1a + 1) * NQ;
  // direction-2 element groups of a plane (block-uniform): group g holds the
  // elements from E2a + g EG2 on (a single group up to p = 3)
  const int ng2 = C::NG2 == 1 ? 1 : (E2b - E2a + C::EG2) / C::EG2;
  auto grp_e2 = [&](int grp) { return C::NG2 == 1 ? E2a : E2a + grp * C::EG2; };
  auto grp_nq2 = [&](int grp) {
    return C::NG2 == 1 ? (E2b - E2a + 1) * NQ : min(C::EG2, E2b + 1 - grp_e2(grp)) * NQ;
  };

  // stage-2/3 identity of this thread
  const int r2 = wave / W, d2 = wave - r2 * W;
  const int d1 = lane / TX, r1 = lane - d1 * TX;
  const bool active = lane < TX * W && r1 < tile.nx && r2 < tile.ny;
  const int i1 = tile.i1 + r1, i2 = tile.i2 + r2;
  // this thread's column (delta1, delta2) of row (i1, i2, 0); delta3 steps by W^2 slots
  OutT* const colp = out + size_t(d1 + W * d2) * kp.ld + size_t(i1) + size_t(kp.m[0]) * i2;
  const size_t sstride = size_t(W * W) * kp.ld;
  const size_t plane = size_t(kp.m[0]) * kp.m[1];

  // window: acc[a][d] = row e3 + a, delta3 = d - P, d <= W - 1 - a
  double acc[P + 1][W];
#pragma unroll
  for (int a = 0; a <= P; ++a)
#pragma unroll
    for (int d = 0; d < W; ++d) acc[a][d] = 0.0;

  // next item of counter c for the whole wave (lane 0 takes it)
  auto fetch = [&](int c) {
    int v = 0;
    if (lane == 0) v = atomicAdd(&qctr[c], 1);
    return __builtin_amdgcn_readfirstlane(v);
  };
  auto phase_a = [&](int g3, int grp) {
    const int nq2 = grp_nq2(grp), e2g = grp_e2(grp);
    const int npt = nq1 * nq2;
    for (int pass = fetch(1); pass * 64 < npt; pass = fetch(1)) {
      const int t = pass * 64 + lane;
      if (t >= npt) continue;
      const int l1 = t / nq2, l2 = t - l1 * nq2;
      const int g[3] = {E1a * NQ + l1, e2g * NQ + l2, g3};
      double v[C::NC];
      point_data<3, FORM, VC>(kp, b, g, v);
#pragma unroll
      for (int c = 0; c < C::NC; ++c) Cs[c * C::CS + l1 * NQ2 + l2] = v[c];
    }
  };
  auto stage1 = [&](int nq2) {
    double* Ysd = reinterpret_cast<double*>(Ys);
    for (int task = fetch(0); task < C::NMODE * TX; task = fetch(0)) {
      const int mode = task / TX, rr1 = task - mode * TX;
      if (rr1 >= tile.nx) continue;
      if (!C::STIFF || mode == S1_VV)
        stage1_b<P, FORM, S1_VV>(kp, Cs, Ysd, tile.i1 + rr1, rr1, E1a, nq2, lane);
      else if (mode == S1_DDV)
        stage1_b<P, FORM, S1_DDV>(kp, Cs, Ysd, tile.i1 + rr1, rr1, E1a, nq2, lane);
      else
        stage1_b<P, FORM, S1_VD>(kp, Cs, Ysd, tile.i1 + rr1, rr1, E1a, nq2, lane);
    }
  };
  // transposed stores (kp.transpose): partner j = i + delta inside the box
  // [tr_lo, tr_hi]^3 takes A_ij as its entry at slot -delta; in directions 1
  // and 2 the test is fixed per thread, in direction 3 per delta3
  const bool tr12 = kp.transpose && i1 + d1 - P >= kp.tr_lo[0] && i1 + d1 - P <= kp.tr_hi[0] &&
                    i2 + d2 - P >= kp.tr_lo[1] && i2 + d2 - P <= kp.tr_hi[1];
  const int64_t troff = int64_t(d1 - P) + int64_t(kp.m[0]) * (d2 - P);
  auto store_row = [&](int i3, int a) {
    if (active && i3 >= tile.z0 && i3 < tile.z1) {
      OutT* p = colp + plane * i3;
      const size_t irow = size_t(i1) + size_t(kp.m[0]) * i2 + plane * i3;
#pragma unroll
      for (int d3 = 0; d3 < W; ++d3) {
        // entries beyond the triangle belong to partners past the last function: zero
        double v = 0.0;
        static_for<0, P + 1>([&](auto ac) {
          constexpr int A = decltype(ac)::value;
          if (A == a && d3 <= W - 1 - A) v = acc[A][d3];
        });
        p[d3 * sstride] = static_cast<OutT>(v);
        const int j3 = i3 + d3 - P;
        if (tr12 && j3 >= kp.tr_lo[2] && j3 <= kp.tr_hi[2]) {
          const int s = d1 + W * (d2 + W * d3);
          out[size_t(kp.S - 1 - s) * kp.ld + size_t(int64_t(irow) + troff + int64_t(plane) * (d3 - P))] =
              static_cast<OutT>(v);
        }
      }
    }
  };

  const int Elo = max(0, tile.z0 - P), Ehi = min(nel3 - 1, tile.z1 - 1);
  const int g0 = Elo * NQ, glast = Ehi * NQ + NQ - 1;
  if (tid == 0) qctr[0] = qctr[1] = 0;
  __syncthreads();
  phase_a(g0, 0);
  __syncthreads();

  // items (plane g3, direction-2 group); the direction-3 products of a plane
  // follow its last group
  double Zc[4] = {0.0, 0.0, 0.0, 0.0};  // a plane's direction-2 sums carried between groups
  const int nitem = (glast - g0 + 1) * ng2;
  for (int it = 0; it < nitem; ++it) {
    const int g3 = C::NG2 == 1 ? g0 + it : g0 + it / ng2;
    const int grp = C::NG2 == 1 ? 0 : it - (g3 - g0) * ng2;
    const int e3 = g3 / NQ, k3 = g3 - e3 * NQ;
    const bool last_grp = grp == ng2 - 1;
    stage1(grp_nq2(grp));
    // the phase-A counter is idle in this interval (its last use ended at the
    // previous barrier), the stage-1 counter in the next one
    if (tid == 0) qctr[1] = 0;
    __syncthreads();
    if (tid == 0) qctr[0] = 0;
    if (active) {
      // the overlap of the supports of i2 and j2 = i2 + delta2: elements
      // i2 - a2 with partner index b2 = a2 + delta2 in [0, P]; per point one
      // scalar load brings the four products (value/derivative of i2 times
      // value/derivative of j2), each then a single FMA operand
      double Z00 = 0.0, Z10 = 0.0, Z01 = 0.0, Z11 = 0.0;
      if (C::NG2 > 1 && grp > 0) {
        Z00 = Zc[0];
        Z10 = Zc[1];
        Z01 = Zc[2];
        Z11 = Zc[3];
      }
      const int e2g = grp_e2(grp);
      constexpr int PP = (P + 1) * (P + 1) * 4;  // product-table doubles per point
      cdptr tab2 = uniform_table(kp.t[1].bpr);
#pragma unroll
      for (int a2 = 0; a2 <= P; ++a2) {
        const int e2 = i2 - a2;
        const int b2 = a2 + d2 - P;
        if (e2 < 0 || e2 >= nel2 || b2 < 0 || b2 > P) continue;
        if (C::NG2 > 1 && (e2 < e2g || e2 >= e2g + C::EG2)) continue;  // another group's element
        cdptr row = tab2 + size_t(e2) * NQ * PP + (a2 * (P + 1) + b2) * 4;
        const double2* yp = Ys + (e2 - e2g) * NQ * YL + lane;
#pragma unroll 2
        for (int k2 = 0; k2 < NQ; ++k2) {
          cdptr rk = row + k2 * PP;
          const double vv = rk[0], vd = rk[1], dv = rk[2], dd = rk[3];
          const double2* yk = yp + k2 * YL;
          // chained FMAs into the accumulators (one instruction per product)
          if constexpr (C::STIFF) {
            const double2 p0 = yk[0], p1 = yk[NQ2 * YL], p2 = yk[2 * NQ2 * YL], p3 = yk[3 * NQ2 * YL];
            Z00 = fma(vv, p0.x, Z00);
            Z00 = fma(vd, p0.y, Z00);
            Z00 = fma(dv, p1.y, Z00);
            Z00 = fma(dd, p2.y, Z00);
            Z10 = fma(vv, p2.x, Z10);
            Z10 = fma(vd, p3.x, Z10);
            Z01 = fma(vv, p1.x, Z01);
            Z01 = fma(dv, p3.x, Z01);
            Z11 = fma(vv, p3.y, Z11);
          } else {
            Z00 = fma(vv, yk[0].x, Z00);
          }
        }
      }
      if (C::NG2 > 1 && !last_grp) {
        Zc[0] = Z00;
        Zc[1] = Z10;
        Zc[2] = Z01;
        Zc[3] = Z11;
      } else {
        cdptr v3 = uniform_table(kp.t[2].bv) + size_t(g3) * (P + 1);
        cdptr t3 = uniform_table(kp.t[2].bd) + size_t(g3) * (P + 1);
#pragma unroll
        for (int b3 = 0; b3 <= P; ++b3) {
          double U, V;
          if constexpr (C::STIFF) {
            U = v3[b3] * Z00 + t3[b3] * Z01;
            V = v3[b3] * Z10 + t3[b3] * Z11;
          } else {
            U = v3[b3] * Z00;
            V = 0.0;
          }
#pragma unroll
          for (int a3 = 0; a3 <= P; ++a3) {
            double& w = acc[a3][b3 - a3 + P];
            w = fma(v3[a3], U, w);
            if constexpr (C::STIFF) w = fma(t3[a3], V, w);
          }
        }
      }
    }
    if (last_grp && k3 == NQ - 1) {
      if (e3 < nel3 - 1) {
        // row e3 is complete: store it and shift the window
        store_row(e3, 0);
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
          for (int d = 0; d < W; ++d) acc[a][d] = (d < W - 1 - a) ? acc[a + 1][d] : 0.0;
#pragma unroll
        for (int d = 0; d < W; ++d) acc[P][d] = 0.0;
      } else {
        // last layer of the domain: every row of the window is complete
#pragma unroll
        for (int a = 0; a <= P; ++a) store_row(e3 + a, a);
      }
    }
    if (it + 1 < nitem) phase_a(last_grp ? g3 + 1 : g3, last_grp ? 0 : grp + 1);
    __syncthreads();
  }
}

// ------------------------------------------------ 3-D single rows -------------
//
// One workgroup per isolated row (the surrogate's sample rows): no other row of
// the workgroup would share its footprint.  The row's support holds at most
// (P+1)^3 elements; planes of direction 3 are streamed as above, stage 1 uses
// the same wave-uniform tasks, stage 2 runs one thread per (delta1, delta2),
// and stage 3 accumulates that thread's W delta3 values (one row: no window).

template <int P, int FORM>
struct Q3R {
  static constexpr int NQ = P + 1, W = 2 * P + 1;
  static constexpr int NQR = (P + 1) * NQ;  // Gauss points of the row's support per direction
  static constexpr bool STIFF = FORM == IGS_STIFFNESS;
  static constexpr int NC = STIFF ? 6 : 1;
  static constexpr int NMODE = STIFF ? 3 : 1;
  static constexpr int NY = STIFF ? 8 : 1;
  static constexpr int NSUB = (3 * NQR + 63) / 64;  // waves per stage-1 task
  static constexpr int CS = (NQR * NQR + 31) / 32 * 32 + NQR % 32;  // component stride of Cs
  static constexpr int BLOCK = 256;
  static_assert(W * W <= BLOCK, "stage-2 threads");
};

// Constant coefficient, p <= 3: at least five waves per SIMD (96 VGPRs at
// p = 3 instead of 108, 8 bytes of spill): 3-4% faster sample rows and 5%
// faster face/edge single rows at 128^3 p = 3; the variable-coefficient
// variants would spill 136-232 bytes, and p = 4 cannot reach five waves, so
// they keep the compiler's choice.
template <int P, int FORM, bool VC, typename OutT>
__global__ void __launch_bounds__(256, (VC || P == 4) ? 1 : 5)
    quad3d_row_kernel(KProblem kp, const QTile* __restrict__ tiles, OutT* __restrict__ band) {
  using C = Q3R<P, FORM>;
  constexpr int NQ = C::NQ, W = C::W, NQR = C::NQR;
  __shared__ double Cs[C::NC * C::CS];
  __shared__ double Ys[C::NY][W][NQR + 1];  // odd row pitch: the delta1 rows of a stage-2 read use distinct banks

  const QTile tile = tiles[blockIdx.x];
  const int b = blockIdx.y;
  OutT* out = band + size_t(b) * kp.S * kp.ld;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i1 = tile.i1, i2 = tile.i2, i3 = tile.z0;
  const int nel1 = kp.nelem[0], nel2 = kp.nelem[1], nel3 = kp.nelem[2];
  const int E1a = max(0, i1 - P), E1b = min(nel1 - 1, i1);
  const int E2a = max(0, i2 - P), E2b = min(nel2 - 1, i2);
  const int E3a = max(0, i3 - P), E3b = min(nel3 - 1, i3);
  const int nq1 = (E1b - E1a + 1) * NQ, nq2 = (E2b - E2a + 1) * NQ;

  // stage-2/3 identity: column (delta1, delta2) and element group.  The
  // waves split the direction-2 elements of the row's support (element a2
  // goes to group a2 mod G, a group being one wave, two for p = 4), so every
  // wave has stage-2 work; stage 3 is linear in the stage-2 sums, so each group
  // accumulates its own partial stencil, and the groups' partials are added
  // (in group order) once, after the last plane.
  constexpr int NCOL = W * W, WPG = (NCOL + 63) / 64;
  constexpr int G = (P + 1) < (C::BLOCK / 64) / WPG ? (P + 1) : (C::BLOCK / 64) / WPG;
  const int grp = wave / WPG;
  const int col = tid - grp * WPG * 64;
  const bool active = grp < G && col < NCOL;
  const int d1 = col % W, d2 = col / W;
  const int j2 = i2 + d2 - P;
  double acc[W];
#pragma unroll
  for (int d = 0; d < W; ++d) acc[d] = 0.0;

  auto phase_a = [&](int g3) {
    for (int t = tid; t < nq1 * nq2; t += C::BLOCK) {
      const int l1 = t / nq2, l2 = t - l1 * nq2;
      const int g[3] = {E1a * NQ + l1, E2a * NQ + l2, g3};
      double v[C::NC];
      point_data<3, FORM, VC>(kp, b, g, v);
#pragma unroll
      for (int c = 0; c < C::NC; ++c) Cs[c * C::CS + l1 * NQR + l2] = v[c];
    }
  };
  auto stage1_task = [&](auto modec, int sub) {
    constexpr int MODE = decltype(modec)::value;
    const int idx = sub * 64 + lane;
    const int cl = idx / NQR, l2 = idx - cl * NQR;
    bool ok = l2 < nq2;
    int comp, code0, code1;
    stage1_slot<MODE, C::STIFF>(cl, &comp, &code0, &code1, &ok);
    double y0[W], y1[W];
    stage1_core<P, MODE>(kp, Cs + comp * C::CS + (ok ? l2 : 0), NQR, i1, E1a, y0, y1);
    if (!ok) return;
#pragma unroll
    for (int dd = 0; dd < W; ++dd) {
      if (code0 >= 0) Ys[code0][dd][l2] = y0[dd];
      if (MODE == S1_DDV && code1 >= 0) Ys[code1][dd][l2] = y1[dd];
    }
  };
  auto stage1 = [&]() {
    for (int task = wave; task < C::NMODE * C::NSUB; task += C::BLOCK / 64) {
      const int mode = task / C::NSUB, sub = task - mode * C::NSUB;
      if (!C::STIFF || mode == S1_VV)
        stage1_task(IntC<S1_VV>{}, sub);
      else if (mode == S1_DDV)
        stage1_task(IntC<S1_DDV>{}, sub);
      else
        stage1_task(IntC<S1_VD>{}, sub);
    }
  };

  const int glast = E3b * NQ + NQ - 1;
  phase_a(E3a * NQ);
  __syncthreads();
  for (int g3 = E3a * NQ; g3 <= glast; ++g3) {
    stage1();
    __syncthreads();
    if (active) {
      double Z00 = 0.0, Z10 = 0.0, Z01 = 0.0, Z11 = 0.0;
#pragma unroll
      for (int a2 = 0; a2 <= P; ++a2) {
        if (a2 % G != grp) continue;
        const int e2 = i2 - a2;
        const int b2 = j2 - e2;
        if (e2 < 0 || e2 >= nel2 || b2 < 0 || b2 > P) continue;
#pragma unroll 1
        for (int k2 = 0; k2 < NQ; ++k2) {
          const int g2 = e2 * NQ + k2;
          const int l2 = (e2 - E2a) * NQ + k2;
          const double* tv = kp.t[1].bv + size_t(g2) * (P + 1);
          const double* td = kp.t[1].bd + size_t(g2) * (P + 1);
          const double vi = tv[a2], vj = tv[b2];
          if constexpr (C::STIFF) {
            const double di = td[a2], dj = td[b2];
            Z00 += vi * (vj * Ys[0][d1][l2] + dj * Ys[1][d1][l2]) + di * (vj * Ys[3][d1][l2] + dj * Ys[5][d1][l2]);
            Z10 += vi * (vj * Ys[4][d1][l2] + dj * Ys[6][d1][l2]);
            Z01 += vj * (vi * Ys[2][d1][l2] + di * Ys[6][d1][l2]);
            Z11 += vi * vj * Ys[7][d1][l2];
          } else {
            Z00 += vi * vj * Ys[0][d1][l2];
          }
        }
      }
      // the row's local index in element e3 is uniform: dispatch it at compile time
      const int a3 = i3 - g3 / NQ;
      cdptr v3 = uniform_table(kp.t[2].bv) + size_t(g3) * (P + 1);
      cdptr t3 = uniform_table(kp.t[2].bd) + size_t(g3) * (P + 1);
      static_for<0, P + 1>([&](auto av) {
        constexpr int A3 = decltype(av)::value;
        if (a3 != A3) return;
        const double va = v3[A3], da = t3[A3];
#pragma unroll
        for (int b3 = 0; b3 <= P; ++b3) {
          if constexpr (C::STIFF)
            acc[b3 - A3 + P] += va * (v3[b3] * Z00 + t3[b3] * Z01) + da * (v3[b3] * Z10 + t3[b3] * Z11);
          else
            acc[b3 - A3 + P] += va * v3[b3] * Z00;
        }
      });
    }
    if (g3 < glast) phase_a(g3 + 1);
    __syncthreads();
  }
  // the groups' partial stencils meet in LDS (the point buffer Cs, free after
  // the last barrier of the plane loop, when it is large enough: stiffness),
  // added in group order by group 0
  constexpr bool IN_CS = G * NCOL * W <= C::NC * C::CS;
  __shared__ double Rx[IN_CS ? 1 : G * NCOL * W];
  double* red = IN_CS ? Cs : Rx;
  if (active && grp > 0) {
#pragma unroll
    for (int d = 0; d < W; ++d) red[(size_t(grp) * NCOL + col) * W + d] = acc[d];
  }
  __syncthreads();
  if (active && grp == 0) {
    for (int g = 1; g < G; ++g)
#pragma unroll
      for (int d = 0; d < W; ++d) acc[d] += red[(size_t(g) * NCOL + col) * W + d];
    const size_t idx = size_t(i1) + size_t(kp.m[0]) * (i2 + size_t(kp.m[1]) * i3);
#pragma unroll
    for (int d3 = 0; d3 < W; ++d3) out[size_t(d1 + W * (d2 + W * d3)) * kp.ld + idx] = static_cast<OutT>(acc[d3]);
  }
}

// ------------------------------------------------------------ 2-D rows -----

template <int P, int FORM>
struct Q2 {
  static constexpr int NQ = P + 1, W = 2 * P + 1;
  static constexpr int TX = P == 4 ? 32 : 64;  // LDS: two element rows of point data
  static constexpr int NQ1 = (TX + P) * NQ;
  static constexpr int NC = FORM == IGS_STIFFNESS ? 3 : 1;
  static constexpr int BLOCK = (TX * W + 63) / 64 * 64;
  // p <= 2: ask for 4 waves per SIMD (128 VGPRs, a few spills at p = 2);
  // larger p would spill heavily
  static constexpr int MINW = P <= 2 ? 4 : 1;
};

// A workgroup owns TX consecutive i1 of a tile and streams its element rows
// e2 (direction 2); thread (r1, d1) accumulates the column delta1 = d1 - P of
// row i1 for every delta2, over a ring of the P+1 rows the current element row
// touches.  The pulled-back coefficients of a whole element row (all NQ Gauss
// lines, the tile's direction-1 footprint) are computed into one LDS buffer
// while the rows consume the other, so an element row costs one barrier.
template <int P, int FORM, typename OutT>
__global__ void __launch_bounds__((Q2<P, FORM>::BLOCK), (Q2<P, FORM>::MINW))
    quad2d_kernel(KProblem kp, const QTile* __restrict__ tiles, OutT* __restrict__ band) {
  using C = Q2<P, FORM>;
  constexpr int NQ = C::NQ, W = C::W, TX = C::TX, NQ1 = C::NQ1;
  __shared__ double Cs[2][C::NC][NQ][NQ1];
  __shared__ double T1v[P + 1][NQ1], T1d[P + 1][NQ1];

  const QTile tile = tiles[blockIdx.x];
  const int b = blockIdx.y;
  OutT* out = band + size_t(b) * kp.S * kp.ld;
  const int tid = threadIdx.x;
  const int nel1 = kp.nelem[0], nel2 = kp.nelem[1];
  const int E1a = max(0, tile.i1 - P), E1b = min(nel1 - 1, tile.i1 + tile.nx - 1);
  const int nq1 = (E1b - E1a + 1) * NQ;
  for (int t = tid; t < nq1 * (P + 1); t += C::BLOCK) {
    T1v[t % (P + 1)][t / (P + 1)] = kp.t[0].bv[size_t(E1a) * NQ * (P + 1) + t];
    T1d[t % (P + 1)][t / (P + 1)] = kp.t[0].bd[size_t(E1a) * NQ * (P + 1) + t];
  }
  const int r1 = tid % TX, d1 = tid / TX;
  const bool active = tid < TX * W && r1 < tile.nx;
  const int i1 = tile.i1 + r1, j1 = i1 + d1 - P;

  double acc[P + 1][W];
#pragma unroll
  for (int s = 0; s < P + 1; ++s)
#pragma unroll
    for (int d = 0; d < W; ++d) acc[s][d] = 0.0;

  const int Elo = max(0, tile.z0 - P), Ehi = min(nel2 - 1, tile.z1 - 1);

  // point data of element row e2 (all NQ Gauss lines) into buffer `buf`
  auto phase_a = [&](int e2, int buf) __attribute__((always_inline)) {
    for (int t = tid; t < nq1 * NQ; t += C::BLOCK) {
      const int k2 = t / nq1, l = t - k2 * nq1;
      const int g[2] = {E1a * NQ + l, e2 * NQ + k2};
      double v[C::NC];
      point_data<2, FORM>(kp, b, g, v);
#pragma unroll
      for (int c = 0; c < C::NC; ++c) Cs[buf][c][k2][l] = v[c];
    }
  };

  // the ring entry is selected by comparison with a slot that is a
  // compile-time constant after inlining, so acc stays in registers
  auto write_row = [&](int i2, int slot) __attribute__((always_inline)) {
    if (active && i2 >= tile.z0 && i2 < tile.z1) {
      const size_t idx = size_t(i1) + size_t(kp.m[0]) * i2;
#pragma unroll
      for (int dd = 0; dd < W; ++dd) {
        double v = 0.0;
#pragma unroll
        for (int r = 0; r <= P; ++r)
          if (r == slot) v = acc[r][dd];
        out[size_t(d1 + W * dd) * kp.ld + idx] = static_cast<OutT>(v);
      }
    }
  };

  if (Elo <= Ehi) phase_a(Elo, 0);
  __syncthreads();

  for (int e0 = Elo; e0 <= Ehi; e0 += P + 1) {
    static_for<0, P + 1>([&](auto ph) __attribute__((always_inline)) {
      constexpr int PH = decltype(ph)::value;
      const int e2 = e0 + PH;
      if (e2 > Ehi) return;
      const int buf = (e2 - Elo) & 1;
      if (e2 < Ehi) phase_a(e2 + 1, buf ^ 1);
      if (active) {
#pragma unroll 1
        for (int k2 = 0; k2 < NQ; ++k2) {
          const int g2 = e2 * NQ + k2;
          double Y0 = 0.0, Y1 = 0.0, Y2 = 0.0, Y3 = 0.0;
#pragma unroll
          for (int a = 0; a <= P; ++a) {
            const int e1 = i1 - a;
            const int bb = j1 - e1;
            if (e1 < 0 || e1 >= nel1 || bb < 0 || bb > P) continue;
            const int le = (e1 - E1a) * NQ;
#pragma unroll
            for (int k1 = 0; k1 < NQ; ++k1) {
              const int l1 = le + k1;
              const double vi = T1v[a][l1], vj = T1v[bb][l1];
              if constexpr (FORM == IGS_MASS) {
                Y0 += vi * vj * Cs[buf][0][k2][l1];
              } else {
                const double di = T1d[a][l1], dj = T1d[bb][l1];
                Y0 += di * dj * Cs[buf][0][k2][l1];  // (1,1): K11, dd
                Y1 += di * vj * Cs[buf][1][k2][l1];  // (1,2): K12, dv
                Y2 += vi * dj * Cs[buf][1][k2][l1];  // (2,1): K12, vd
                Y3 += vi * vj * Cs[buf][2][k2][l1];  // (2,2): K22, vv
              }
            }
          }
          const double* v2p = kp.t[1].bv + size_t(g2) * (P + 1);
          const double* d2p = kp.t[1].bd + size_t(g2) * (P + 1);
          double v2[P + 1], dv2[P + 1];
#pragma unroll
          for (int a = 0; a <= P; ++a) {
            v2[a] = v2p[a];
            dv2[a] = d2p[a];
          }
#pragma unroll
          for (int b2 = 0; b2 <= P; ++b2) {
            double U, V;
            if constexpr (FORM == IGS_MASS) {
              U = v2[b2] * Y0;
              V = 0.0;
            } else {
              U = v2[b2] * Y0 + dv2[b2] * Y1;
              V = v2[b2] * Y2 + dv2[b2] * Y3;
            }
#pragma unroll
            for (int a2 = 0; a2 <= P; ++a2) {
              if constexpr (FORM == IGS_MASS)
                acc[(PH + a2) % (P + 1)][b2 - a2 + P] += v2[a2] * U;
              else
                acc[(PH + a2) % (P + 1)][b2 - a2 + P] += v2[a2] * U + dv2[a2] * V;
            }
          }
        }
      }
      if (e2 < nel2 - 1) {
        write_row(e2, PH);
#pragma unroll
        for (int d = 0; d < W; ++d) acc[PH][d] = 0.0;
      } else {
#pragma unroll
        for (int a = 0; a <= P; ++a) {
          write_row(e2 + a, (PH + a) % (P + 1));
#pragma unroll
          for (int d = 0; d < W; ++d) acc[(PH + a) % (P + 1)][d] = 0.0;
        }
      }
      __syncthreads();
    });
  }
}

// ------------------------------------------------------------- load vector --

template <int ND>
__device__ __forceinline__ double source_at(const KProblem& kp, const int* g, int src, double c) {
  double xi[ND], w = 1.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    xi[d] = kp.t[d].x[g[d]];
    w *= kp.t[d].w[g[d]];
  }
  double J[ND][ND];
  jacobian<ND>(kp, g, xi, J);
  double det;
  if constexpr (ND == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  } else {
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  }
  if (!(det > 0.0)) atomicOr(kp.flag, 1);
  double f = c;
  if (src == 1) {
    double F[ND];
    phys_point<ND>(kp, g, xi, F);
#pragma unroll
    for (int d = 0; d < ND; ++d) f *= sinpi(F[d]);
  }
  return w * fabs(det) * f;
}

template <int P>
struct R3 {
  static constexpr int NQ = P + 1, TX = 16, TY = 16;
  static constexpr int NQ1 = (TX + P) * NQ, NQ2 = (TY + P) * NQ;
  static constexpr int BLOCK = TX * TY;
};

template <int P>
__global__ void __launch_bounds__(R3<P>::BLOCK)
    rhs3d_kernel(KProblem kp, const QTile* __restrict__ tiles, int src, double c, double* __restrict__ f) {
  using C = R3<P>;
  constexpr int NQ = C::NQ, TX = C::TX, NQ1 = C::NQ1, NQ2 = C::NQ2;
  __shared__ double Fs[NQ1][NQ2];
  __shared__ double Ys[TX][NQ2];
  __shared__ double T1v[P + 1][NQ1], T2v[P + 1][NQ2];
  const QTile tile = tiles[blockIdx.x];
  const int b = blockIdx.y;
  double* out = f + size_t(b) * kp.N;
  const int tid = threadIdx.x;
  const int nel1 = kp.nelem[0], nel2 = kp.nelem[1], nel3 = kp.nelem[2];
  const int E1a = max(0, tile.i1 - P), E1b = min(nel1 - 1, tile.i1 + tile.nx - 1);
  const int E2a = max(0, tile.i2 - P), E2b = min(nel2 - 1, tile.i2 + tile.ny - 1);
  const int nq1 = (E1b - E1a + 1) * NQ, nq2 = (E2b - E2a + 1) * NQ;
  for (int t = tid; t < nq1 * (P + 1); t += C::BLOCK) T1v[t % (P + 1)][t / (P + 1)] = kp.t[0].bv[size_t(E1a) * NQ * (P + 1) + t];
  for (int t = tid; t < nq2 * (P + 1); t += C::BLOCK) T2v[t % (P + 1)][t / (P + 1)] = kp.t[1].bv[size_t(E2a) * NQ * (P + 1) + t];
  const int r1 = tid % TX, r2 = tid / TX;
  const bool active = r1 < tile.nx && r2 < tile.ny;
  const int i1 = tile.i1 + r1, i2 = tile.i2 + r2;
  double acc[P + 1];
#pragma unroll
  for (int s = 0; s <= P; ++s) acc[s] = 0.0;
  const int Elo = max(0, tile.z0 - P), Ehi = min(nel3 - 1, tile.z1 - 1);
  __syncthreads();
  auto write_row = [&](int i3, double v) {
    if (active && i3 >= tile.z0 && i3 < tile.z1) out[size_t(i1) + size_t(kp.m[0]) * (i2 + size_t(kp.m[1]) * i3)] = v;
  };
  for (int e0 = Elo; e0 <= Ehi; e0 += P + 1) {
    static_for<0, P + 1>([&](auto ph) {
      constexpr int PH = decltype(ph)::value;
      const int e3 = e0 + PH;
      if (e3 > Ehi) return;
      for (int k3 = 0; k3 < NQ; ++k3) {
        const int g3 = e3 * NQ + k3;
        for (int t = tid; t < nq1 * nq2; t += C::BLOCK) {
          const int l1 = t / nq2, l2 = t - l1 * nq2;
          const int g[3] = {E1a * NQ + l1, E2a * NQ + l2, g3};
          Fs[l1][l2] = source_at<3>(kp, g, src, c);
        }
        __syncthreads();
        for (int t = tid; t < TX * nq2; t += C::BLOCK) {
          const int l2 = t % nq2, rr1 = t / nq2;
          const int ii1 = tile.i1 + rr1;
          double y = 0.0;
#pragma unroll
          for (int a = 0; a <= P; ++a) {
            const int e1 = ii1 - a;
            if (rr1 >= tile.nx || e1 < 0 || e1 >= nel1) continue;
#pragma unroll
            for (int k1 = 0; k1 < NQ; ++k1) {
              const int l1 = (e1 - E1a) * NQ + k1;
              y += T1v[a][l1] * Fs[l1][l2];
            }
          }
          Ys[rr1][l2] = y;
        }
        __syncthreads();
        if (active) {
          double z = 0.0;
#pragma unroll
          for (int a2 = 0; a2 <= P; ++a2) {
            const int e2 = i2 - a2;
            if (e2 < 0 || e2 >= nel2) continue;
#pragma unroll
            for (int k2 = 0; k2 < NQ; ++k2) {
              const int l2 = (e2 - E2a) * NQ + k2;
              z += T2v[a2][l2] * Ys[r1][l2];
            }
          }
          const double* v3 = kp.t[2].bv + size_t(g3) * (P + 1);
#pragma unroll
          for (int a3 = 0; a3 <= P; ++a3) acc[(PH + a3) % (P + 1)] += v3[a3] * z;
        }
      }
      if (e3 < nel3 - 1) {
        write_row(e3, acc[PH]);
        acc[PH] = 0.0;
      } else {
#pragma unroll
        for (int a = 0; a <= P; ++a) {
          write_row(e3 + a, acc[(PH + a) % (P + 1)]);
          acc[(PH + a) % (P + 1)] = 0.0;
        }
      }
    });
  }
}

template <int P>
struct R2 {
  static constexpr int NQ = P + 1, TX = 256;
  static constexpr int NQ1 = (TX + P) * NQ;
};

template <int P>
__global__ void __launch_bounds__(256)
    rhs2d_kernel(KProblem kp, const QTile* __restrict__ tiles, int src, double c, double* __restrict__ f) {
  using C = R2<P>;
  constexpr int NQ = C::NQ, NQ1 = C::NQ1;
  __shared__ double Fs[NQ1];
  __shared__ double T1v[P + 1][NQ1];
  const QTile tile = tiles[blockIdx.x];
  const int b = blockIdx.y;
  double* out = f + size_t(b) * kp.N;
  const int tid = threadIdx.x;
  const int nel1 = kp.nelem[0], nel2 = kp.nelem[1];
  const int E1a = max(0, tile.i1 - P), E1b = min(nel1 - 1, tile.i1 + tile.nx - 1);
  const int nq1 = (E1b - E1a + 1) * NQ;
  for (int t = tid; t < nq1 * (P + 1); t += 256) T1v[t % (P + 1)][t / (P + 1)] = kp.t[0].bv[size_t(E1a) * NQ * (P + 1) + t];
  const bool active = tid < tile.nx;
  const int i1 = tile.i1 + tid;
  double acc[P + 1];
#pragma unroll
  for (int s = 0; s <= P; ++s) acc[s] = 0.0;
  const int Elo = max(0, tile.z0 - P), Ehi = min(nel2 - 1, tile.z1 - 1);
  __syncthreads();
  auto write_row = [&](int i2, double v) {
    if (active && i2 >= tile.z0 && i2 < tile.z1) out[size_t(i1) + size_t(kp.m[0]) * i2] = v;
  };
  for (int e0 = Elo; e0 <= Ehi; e0 += P + 1) {
    static_for<0, P + 1>([&](auto ph) {
      constexpr int PH = decltype(ph)::value;
      const int e2 = e0 + PH;
      if (e2 > Ehi) return;
      for (int k2 = 0; k2 < NQ; ++k2) {
        const int g2 = e2 * NQ + k2;
        for (int t = tid; t < nq1; t += 256) {
          const int g[2] = {E1a * NQ + t, g2};
          Fs[t] = source_at<2>(kp, g, src, c);
        }
        __syncthreads();
        if (active) {
          double y = 0.0;
#pragma unroll
          for (int a = 0; a <= P; ++a) {
            const int e1 = i1 - a;
            if (e1 < 0 || e1 >= nel1) continue;
#pragma unroll
            for (int k1 = 0; k1 < NQ; ++k1) {
              const int l1 = (e1 - E1a) * NQ + k1;
              y += T1v[a][l1] * Fs[l1];
            }
          }
          const double* v2 = kp.t[1].bv + size_t(g2) * (P + 1);
#pragma unroll
          for (int a2 = 0; a2 <= P; ++a2) acc[(PH + a2) % (P + 1)] += v2[a2] * y;
        }
        __syncthreads();
      }
      if (e2 < nel2 - 1) {
        write_row(e2, acc[PH]);
        acc[PH] = 0.0;
      } else {
#pragma unroll
        for (int a = 0; a <= P; ++a) {
          write_row(e2 + a, acc[(PH + a) % (P + 1)]);
          acc[(PH + a) % (P + 1)] = 0.0;
        }
      }
    });
  }
}

// ------------------------------------------------------------- launchers ---

void quad_tile_shape(int n, int p, int* tx, int* ty) {
  if (n == 2) {
    *tx = p == 4 ? Q2<4, IGS_STIFFNESS>::TX : Q2<1, IGS_STIFFNESS>::TX;
    *ty = 1;
    return;
  }
  switch (p) {
    case 1: *tx = Q3B<1, IGS_STIFFNESS>::TX; *ty = Q3B<1, IGS_STIFFNESS>::TY; break;
    case 2: *tx = Q3B<2, IGS_STIFFNESS>::TX; *ty = Q3B<2, IGS_STIFFNESS>::TY; break;
    case 3: *tx = Q3B<3, IGS_STIFFNESS>::TX; *ty = Q3B<3, IGS_STIFFNESS>::TY; break;
    default: *tx = Q3B<4, IGS_STIFFNESS>::TX; *ty = Q3B<4, IGS_STIFFNESS>::TY; break;
  }
}

void rhs_tile_shape(int n, int* tx, int* ty) {
  *tx = (n == 2) ? 256 : 16;
  *ty = (n == 2) ? 1 : 16;
}

template <int P, int FORM, typename OutT>
static hipError_t launch_quad_t(const KProblem& kp, const QTile* tiles, int ntiles, bool rows, OutT* band,
                                hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  dim3 grid(ntiles, kp.batch);
  const bool vc = kp.coef != IGS_COEF_CONST;
  if (kp.n == 3 && rows) {
    if (vc)
      hipLaunchKernelGGL((quad3d_row_kernel<P, FORM, true, OutT>), grid, dim3(Q3R<P, FORM>::BLOCK), 0, s, kp, tiles,
                         band);
    else
      hipLaunchKernelGGL((quad3d_row_kernel<P, FORM, false, OutT>), grid, dim3(Q3R<P, FORM>::BLOCK), 0, s, kp,
                         tiles, band);
  } else if (kp.n == 3) {
    if (vc)
      hipLaunchKernelGGL((quad3d_tile_kernel<P, FORM, true, OutT>), grid, dim3(Q3B<P, FORM>::BLOCK), 0, s, kp,
                         tiles, band);
    else
      hipLaunchKernelGGL((quad3d_tile_kernel<P, FORM, false, OutT>), grid, dim3(Q3B<P, FORM>::BLOCK), 0, s, kp,
                         tiles, band);
  } else {
    hipLaunchKernelGGL((quad2d_kernel<P, FORM, OutT>), grid, dim3(Q2<P, FORM>::BLOCK), 0, s, kp, tiles, band);
  }
  return hipGetLastError();
}

template <int P, typename OutT>
static hipError_t launch_quad_p(const KProblem& kp, int form, const QTile* tiles, int ntiles, bool rows, OutT* band,
                                hipStream_t s) {
  return form == IGS_MASS ? launch_quad_t<P, IGS_MASS, OutT>(kp, tiles, ntiles, rows, band, s)
                          : launch_quad_t<P, IGS_STIFFNESS, OutT>(kp, tiles, ntiles, rows, band, s);
}

// rows = false: tiles of quad_tile_shape; rows = true: single-row tiles (nx = ny = 1, z1 = z0 + 1)
template <typename OutT>
hipError_t launch_quad(const KProblem& kp, int form, const QTile* tiles, int ntiles, bool rows, OutT* band,
                       hipStream_t s) {
  switch (kp.p) {
    case 1: return launch_quad_p<1, OutT>(kp, form, tiles, ntiles, rows, band, s);
    case 2: return launch_quad_p<2, OutT>(kp, form, tiles, ntiles, rows, band, s);
    case 3: return launch_quad_p<3, OutT>(kp, form, tiles, ntiles, rows, band, s);
    default: return launch_quad_p<4, OutT>(kp, form, tiles, ntiles, rows, band, s);
  }
}

template hipError_t launch_quad<double>(const KProblem&, int, const QTile*, int, bool, double*, hipStream_t);
template hipError_t launch_quad<float>(const KProblem&, int, const QTile*, int, bool, float*, hipStream_t);

template <int P>
static hipError_t launch_rhs_p(const KProblem& kp, const QTile* tiles, int ntiles, int src, double c, double* f,
                               hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  dim3 grid(ntiles, kp.batch);
  if (kp.n == 3)
    hipLaunchKernelGGL((rhs3d_kernel<P>), grid, dim3(R3<P>::BLOCK), 0, s, kp, tiles, src, c, f);
  else
    hipLaunchKernelGGL((rhs2d_kernel<P>), grid, dim3(256), 0, s, kp, tiles, src, c, f);
  return hipGetLastError();
}

hipError_t launch_rhs(const KProblem& kp, const QTile* tiles, int ntiles, int src, double c, double* f,
                      hipStream_t s) {
  switch (kp.p) {
    case 1: return launch_rhs_p<1>(kp, tiles, ntiles, src, c, f, s);
    case 2: return launch_rhs_p<2>(kp, tiles, ntiles, src, c, f, s);
    case 3: return launch_rhs_p<3>(kp, tiles, ntiles, src, c, f, s);
    default: return launch_rhs_p<4>(kp, tiles, ntiles, src, c, f, s);
  }
}

}  // namespace igs
