// Internal declarations shared by the host planner, the HIP kernels and the
// C-ABI layer of libigs.  Nothing here is part of the public ABI (include/igs.h).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "igs.h"

namespace igs {

constexpr int kMaxP = 4;
constexpr int kMaxQ = 5;

// Device-resident 1-D tables for one direction.  Quadrature point g = e*nq + k
// (element e, Gauss point k); the p+1 functions alive on element e are e..e+p
// and "local index a" means function e+a.
struct Tab1D {
  const double* x;     // [Q]       parametric coordinate
  const double* w;     // [Q]       Gauss weight * h/2
  const double* bv;    // [Q][p+1]  b_{e+a}(x_g)
  const double* bd;    // [Q][p+1]  b'_{e+a}(x_g)
  const double* bpr;   // [Q][p+1][p+1][4] products of functions e+a, e+b:
                       //   b_a b_b, b_a b'_b, b'_a b_b, b'_a b'_b
  const double* trig;  // [Q][4]    sin(pi x), pi cos(pi x), sin(2 pi x), 2 pi cos(2 pi x)
  const double* cb;    // [Q][cdeg+1] coefficient-spline basis values (spline kinds)
  const int* cf;       // [Q]       first coefficient-spline function alive at x_g
};

// Problem description as the kernels see it (passed by value).
struct KProblem {
  int n, p, nq;
  int nelem[3], m[3];
  int64_t N, ld;
  int S;                 // (2p+1)^n
  int batch;
  int geom;
  double ga;
  int coef;
  double c0, camp;
  int cdeg;
  int cn[3];
  int64_t cstride;       // control values per problem
  const double* cc;      // control values [batch][cstride]
  Tab1D t[3];
  int* flag;             // device error word: bit 0 = det J <= 0
  // 3-D tile kernels with transpose != 0 also store every entry A_ij whose
  // partner j lies in the box [tr_lo, tr_hi]^3 as A_ji into row j (slot -delta):
  // the exact entries the analysis-domain rows take from rows outside it
  int transpose;
  int tr_lo[3], tr_hi[3];
};

// One tile of rows for the quadrature kernels.
//   3D: rows i1 in [i1, i1+nx), i2 in [i2, i2+ny), i3 in [z0, z1)
//   2D: rows i1 in [i1, i1+nx), i2 in [z0, z1) (i2, ny unused)
struct QTile {
  int i1, i2, nx, ny, z0, z1;
};

// Interpolation plan (surrogate) as the kernels see it.
template <typename T>
struct KInterp {
  int q;
  int Sd[3];             // samples per direction
  int lo[3], hi[3];      // analysis-domain index range per direction
  const int* samp[3];    // [Sd]  sample fine indices
  const double* ginv[3]; // [Sd][Sd] inverse collocation matrices (row-major)
  const int* ef[3];      // [m]   first spline function alive at fine index
  const T* eb[3];        // [m][q+1] spline values at fine index
  int nup;               // number of interpolated (upper) slots
  const int* upslot;     // [nup] band slot of each interpolated delta
  int nc[3];             // max coefficient span of a fill box, per direction
  int flo[3], fhi[3];    // coefficient range of the spline part per direction;
                         // outside it ginv is the identity (face/edge layers)
};

// Interpolation with a domain per stencil function (per-delta surrogate).
// Per direction d and offset e = delta_d + p, the stencil function's domain is
// the index range [lo, hi] where row i and partner i + delta_d index cardinal
// B-splines; its samples are a subset of the direction's common sample
// indices U (the analysis-domain lattice plus the two transition bands).
constexpr int kMaxW = 9;  // 2p + 1 offsets per direction, p <= 4
struct KInterpPD {
  int q, p, W, smax, nup, form;
  int m[3];
  int S[3][kMaxW];                  // samples of offset e (first = lo, last = hi)
  int lo[3][kMaxW], hi[3][kMaxW];   // domain index range of offset e
  int nu[3];                        // size of U per direction
  const int* U[3];                  // [nu] common sample indices
  const int* pos[3];                // [W][smax] position in U of sample k of offset e
  const double* ginv[3];            // [W][smax][smax] inverse collocation matrices
  const int* ef[3];                 // [W][m] first spline coefficient alive at index i
  const double* eb[3];              // [W][q+1][m] spline values at index i
};

// ---------------------------------------------------------------- host plan

struct Dims {
  int n, p, nq, W, S;
  int nelem[3], m[3];
  int64_t N, ld;
  int batch;
  // 2-D surrogate plans: 1 when the pencils are too long for the 2-D fill
  // with register-held weights but its LDS footprint fits (set by the plan;
  // make_dims leaves it 0)
  int wide2d;
};

igs_status make_dims(const igs_problem* pb, Dims* d);

struct HostTables {
  // per direction, flattened as in Tab1D
  std::vector<double> x[3], w[3], bv[3], bd[3], bpr[3], trig[3], cb[3];
  std::vector<int> cf[3];
};

void build_tables(const igs_problem* pb, const Dims& d, HostTables* t);

struct HostInterp {
  int q;
  std::vector<int> samp[3];
  std::vector<double> ginv[3];
  std::vector<int> ef[3];
  std::vector<double> eb[3];
  std::vector<int> upslot;
  int nc[3];
  int lo[3], hi[3];      // rows the fill evaluates per direction (the analysis
                         // range, or the whole index range for face/edge)
  int flo[3], fhi[3];    // spline part of the coefficient range (see KInterp)
};

// samples per direction; IGS_ERR_SAMPLES when the lattice is too small
igs_status sample_lattice(int m, int p, int M, std::vector<int>* s);
igs_status build_interp(const Dims& d, int form, int M, int q, int boxlen[3], HostInterp* hi);
// Face/edge stencil functions (Sec. 3.6): per direction the sample set is the
// 4p boundary layers plus the lattice, in index order; the interpolation is
// the degree-q spline on the lattice part and the identity on the layers, and
// the fill covers every index.  samp[d] then lists every quadrature index.
igs_status build_interp_fe(const Dims& d, int form, int M, int q, int boxlen[3], HostInterp* hi);

struct HostInterpPD {
  int q, p, W, smax;
  std::vector<int> U[3];
  int S[3][kMaxW], lo[3][kMaxW], hi[3][kMaxW];
  std::vector<int> pos[3];      // [W][smax]
  std::vector<double> ginv[3];  // [W][smax][smax]
  std::vector<int> ef[3];       // [W][m]
  std::vector<double> eb[3];    // [W][q+1][m]
  std::vector<int> upslot;
};
// Per-delta surrogate (Sec. 4 remark): per direction the common sample set U
// and, per offset, its samples, inverse collocation matrix and evaluation
// tables.  IGS_ERR_SAMPLES when an offset has fewer than q+1 samples.
igs_status build_interp_pd(const Dims& d, int form, int M, int q, HostInterpPD* hi);
// Rows outside the box [c, m_d - c - 1]^n as tiles streamed along the last
// direction (groups[0]: rows of the box's pencils outside it in i1, groups[1]:
// the other pencils), long tiles first.
std::vector<QTile> tiles_shell(const Dims& d, int c, int tx, int ty, int zchunk, int groups[2]);

// Tile lists.
std::vector<QTile> tiles_all(const Dims& d, int tx, int ty, int zchunk);
// groups[0..2] = tile counts of the rows of the analysis-domain pencils
// (pencils along i1) outside the domain in i1, the rows of the other pencils,
// and the sample rows (in that order in the list)
std::vector<QTile> tiles_surrogate(const Dims& d, const std::vector<int> samp[3], int tx, int ty, int zchunk,
                                   int groups[3]);

// Face/edge surrogate: the quadrature rows of the tensor sample set; groups[0]
// tiles of quad_tile_shape (runs of the set), groups[2] single-row tiles
// (3-D rows with an isolated i1), groups[1] = 0.
std::vector<QTile> tiles_fe(const Dims& d, const std::vector<int> samp[3], int tx, int ty, int zchunk,
                            int groups[3]);

// Caller-provided device memory that arenas carve their pieces from instead
// of allocating (the allocation-free entry point): every arena attached to a
// pool takes the next 256-byte aligned range, and fails with
// IGS_ERR_SCRATCH when the pool is exhausted.
struct ScratchPool {
  char* base = nullptr;
  size_t cap = 0, used = 0;
};

// Device scratch arena: one stream-ordered allocation carved into pieces.
// put() reserves a piece and stages host data for it; flush() sends every
// staged piece with a single host-to-device copy (the pieces are contiguous,
// scratch pieces between them receive zeros before any kernel touches them).
struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0;
  hipStream_t stream = nullptr;
  bool persistent = false;  // plain hipMalloc/hipFree (outlives the stream it was made on)
  ScratchPool* pool = nullptr;  // when set: carve from the pool, never allocate or free
  std::vector<char> stage;
  size_t dlo = ~size_t(0), dhi = 0;
  igs_status alloc(size_t bytes, hipStream_t s);
  template <typename T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return reinterpret_cast<T*>(base + off);
  }
  template <typename T>
  const T* put(const T* data, size_t count) {
    T* p = take<T>(count);
    const size_t off = reinterpret_cast<char*>(p) - base, bytes = count * sizeof(T);
    if (stage.size() < off + bytes) stage.resize(size);
    if (bytes) std::memcpy(stage.data() + off, data, bytes);
    dlo = std::min(dlo, off);
    dhi = std::max(dhi, off + bytes);
    return p;
  }
  igs_status flush();
  void release();
  ~Arena() { release(); }
};

inline size_t padded(size_t bytes) { return (bytes + 255) & ~size_t(255); }

// Uploads host tables into an arena and fills the kernel view.
struct DeviceTables {
  KProblem kp;
};

}  // namespace igs
