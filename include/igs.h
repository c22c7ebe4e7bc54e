/*
 * igs.h -- C ABI of the surrogate-matrix isogeometric assembly library
 * (libigs.so, HIP kernels for gfx950).
 *
 * The method: Drzisga, Keith & Wohlmuth, "The surrogate matrix methodology:
 * Low-cost assembly for isogeometric analysis".  Section references below are
 * to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Discretisation (Sec. 2.2): single patch, parametric domain (0,1)^n,
 *   n in {2,3}; tensor-product B-splines of uniform degree p on open uniform
 *   knot vectors with nelem[d] elements in direction d; m[d] = nelem[d] + p
 *   functions per direction; N = prod m[d] dofs per problem.
 * - Dof index (Sec. 2.2, colexicographic): i = i1 + m1*(i2 + m2*i3), 0-based.
 * - Stencils (Sec. 3.2): row i couples to j = i + delta, delta in [-p,p]^n;
 *   S = (2p+1)^n slots per row; slot s = sum_d (delta_d + p)(2p+1)^(d-1),
 *   delta_1 fastest, so slots are ordered like the colex offset of delta and
 *   the centre slot (S-1)/2 is the diagonal.  "Upper" slots are s > (S-1)/2
 *   (j > i in the dof order, Sec. 5.2).
 * - Band layout (stencil-major): band[b][s][k], b < batch, s < S, k < ld,
 *   where ld is the smallest multiple of 64 greater than N (igs_band_layout).  Entry
 *   band[b][s][i] = A_{i, i+delta_s}; it is 0 when i+delta_s leaves the index
 *   box.  Padding k in [N, ld) is written as 0.
 * - Vectors are [batch][N], contiguous.
 * - Band pointers passed to igs_apply and igs_solve_cg are aligned to 16
 *   bytes (FP64) or 8 bytes (FP32), as every device allocation is: their
 *   kernels read two consecutive rows of a slot with one load.  Others are
 *   rejected with IGS_ERR_ARG.
 * - Device memory: every pointer marked "device" must be device memory (or
 *   host-coherent memory visible to the GPU) owned by the caller.  The library
 *   keeps no pointer after a call returns and holds no global mutable state
 *   besides the opt-in, thread-local profiling record (igs_profile_enable)
 *   and the static scratch array of igs_assemble_noalloc;
 *   scratch memory is taken stream-ordered from the default memory pool and
 *   returned before the call returns.  Plans (igs_plan_*) are the exception:
 *   they own device memory from igs_plan_create to igs_plan_destroy.
 * - stream: a hipStream_t passed as void* (NULL = the null stream).
 * - Errors: every entry point returns an igs_status.  Argument errors are
 *   detected on the host before any GPU work is queued.  Assembly entry points
 *   synchronise `stream` before returning so that a geometry map that folds
 *   (det J <= 0 at a quadrature point) is reported as IGS_ERR_GEOMETRY; the
 *   band contents are then unspecified.
 */
#ifndef IGS_H
#define IGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum igs_status {
  IGS_OK = 0,
  IGS_ERR_ARG = -1,         /* null pointer, bad enum, bad size */
  IGS_ERR_UNSUPPORTED = -2, /* valid input outside what the library implements */
  IGS_ERR_KNOTS = -3,       /* a supplied knot vector is not open uniform */
  IGS_ERR_SAMPLES = -4,     /* fewer than q+1 samples, or no analysis-domain rows */
  IGS_ERR_GEOMETRY = -5,    /* det J <= 0 at a quadrature point */
  IGS_ERR_HIP = -6,         /* a HIP runtime call failed */
  IGS_ERR_NOMEM = -7,       /* scratch allocation failed */
  IGS_ERR_SCRATCH = -8,     /* igs_assemble_noalloc: the problem needs more
                               scratch than IGS_NOALLOC_SCRATCH_BYTES */
  IGS_NOT_CONVERGED = 1,    /* solver stopped at maxit */
  IGS_BREAKDOWN = 2         /* CG: p^T A p <= 0 or a non-finite value */
} igs_status;

typedef enum igs_form { IGS_STIFFNESS = 0, IGS_MASS = 1 } igs_form;
typedef enum igs_dtype { IGS_F64 = 0, IGS_F32 = 1 } igs_dtype;

/* Geometry map F: (0,1)^n -> R^n (Sec. 2.1 single patch; the paper builds F
 * from NURBS, here it is analytic).
 *   IDENTITY: F(xi) = xi.
 *   SINE (amplitude a):
 *     n=2: F = (xi1 + a sin(pi xi1) sin(2 pi xi2), xi2 + a sin(2 pi xi1) sin(pi xi2))
 *     n=3: F = xi + a (s(pi xi1)s(2pi xi2)s(pi xi3), s(2pi xi1)s(pi xi2)s(pi xi3),
 *                      s(pi xi1)s(pi xi2)s(2pi xi3)),  s = sin
 *   POLY2 (amplitude a): F_r = xi_r + a (r+1) prod_d xi_d (1 - xi_d), r 0-based;
 *     every component lies in Q_2 (used for the mass reproduction property,
 *     Corollary MassMatrixReproduction). */
typedef enum igs_geom_kind { IGS_GEOM_IDENTITY = 0, IGS_GEOM_SINE = 1, IGS_GEOM_POLY2 = 2 } igs_geom_kind;

typedef struct igs_geometry {
  int32_t kind;  /* igs_geom_kind */
  double a;      /* amplitude */
} igs_geometry;

/* Diffusion coefficient kappa of the stiffness form a(u,v) = int kappa grad u . grad v
 * (Sec. 3.2 eq. BilinearFormPoissonTensor with K scaled by kappa).
 *   CONST:      kappa = c0
 *   SINE3:      kappa = c0 + amp sin(2pi x1) cos(2pi x2) [sin(2pi x3)], x = F(xi)
 *   SPLINE:     kappa = g(xi) = sum_k c_k N_k(xi)
 *   EXP_SPLINE: kappa = exp(g(xi))
 * g is a tensor B-spline of degree `degree` on open uniform knots over the
 * parametric domain with ncoef[d] functions in direction d; its control values
 * `coef` are device memory, [batch][prod ncoef], colex (k1 fastest).  The mass
 * form ignores kappa. */
typedef enum igs_coef_kind {
  IGS_COEF_CONST = 0, IGS_COEF_SINE3 = 1, IGS_COEF_SPLINE = 2, IGS_COEF_EXP_SPLINE = 3
} igs_coef_kind;

typedef struct igs_coef {
  int32_t kind;        /* igs_coef_kind */
  double c0, amp;
  int32_t degree;      /* spline kinds: 1..5 */
  int32_t ncoef[3];    /* spline kinds: functions per direction, degree < ncoef[d] <= 64 */
  const double* coef;  /* spline kinds: device, [batch][prod ncoef] */
} igs_coef;

/* The problem (Sec. 2): knots, degree, geometry, coefficient. */
typedef struct igs_problem {
  int32_t n;                 /* 2 or 3 */
  int32_t p;                 /* 1..4 */
  int32_t nelem[3];          /* elements per direction (entries >= n ignored) */
  int32_t nquad;             /* Gauss points per direction per element; 0 or p+1 */
  int32_t batch;             /* >= 1 independent problems (differ only in coef) */
  const double* knots[3];    /* host, optional: NULL = open uniform; else m+p+1
                                values that must form the open uniform vector */
  igs_geometry geom;
  igs_coef coef;
} igs_problem;

/* Sizes of the band for a problem (host-only, no GPU call). */
typedef struct igs_layout {
  int32_t m[3];        /* functions per direction (1 for unused directions) */
  int32_t slots;       /* S = (2p+1)^n */
  int32_t upper;       /* (S-1)/2 upper slots */
  int64_t N;           /* dofs per problem */
  int64_t ld;          /* slot stride of the band: smallest multiple of 64 > N */
  int64_t band_elems;  /* batch * S * ld */
} igs_layout;

/* Sampling of the surrogate (host-only): sample lattice and row classes. */
typedef struct igs_surrogate_info {
  int32_t samples[3];        /* samples per direction */
  int32_t interior[3];       /* analysis-domain indices per direction, m - 4p */
  int64_t sample_rows;       /* prod samples */
  int64_t boundary_rows;     /* rows outside the analysis domain */
  int64_t quadrature_rows;   /* boundary_rows + sample_rows */
} igs_surrogate_info;

/* Face/edge surrogate sampling (host-only, igs_surrogate_fe_layout). */
typedef struct igs_fe_info {
  int32_t samples[3];        /* per direction: the 4p boundary layers plus the
                                lattice samples (1 for unused directions) */
  int64_t classes;           /* row classes with a stencil-function family:
                                (4p+1)^n - (4p)^n */
  int64_t corner_rows;       /* (4p)^n rows with no free direction (exact) */
  int64_t quadrature_rows;   /* prod samples[d]: every row assembled by quadrature */
} igs_fe_info;

/* Per-delta surrogate sampling (host-only, igs_surrogate_pd_layout). */
typedef struct igs_pd_info {
  int32_t samples[3];        /* per direction: the common sample indices, the
                                lattice plus the 2p transition-band indices
                                [p, 2p) and [m-2p, m-p) (1 if unused) */
  int32_t max_samples[3];    /* largest sample count of one offset */
  int64_t noncardinal_rows;  /* N - prod (m_d - 2p): rows of non-cardinal functions */
  int64_t quadrature_rows;   /* noncardinal_rows + prod samples[d] */
} igs_pd_info;

typedef struct igs_cg_info {
  int32_t iterations;        /* total CG iterations (inner FP32 ones in mixed mode) */
  int32_t outer_iterations;  /* with an FP32 band: FP64 residual replacements;
                                FP64 only: 1 unless the true-residual check
                                restarts CG */
  int32_t status;            /* igs_status of the solve */
  double relres;             /* max over batch of ||f_I - A_II u_I||_2 / ||f_I||_2, FP64 */
} igs_cg_info;

/* ---------------------------------------------------------------- queries */

/* Band sizes.  IGS_ERR_ARG for invalid problems.  Host only. */
igs_status igs_band_layout(const igs_problem* pb, igs_layout* out);

/* Validate a problem (and, for M >= 1, the sampling M, q).  Host only. */
igs_status igs_validate(const igs_problem* pb, int32_t M, int32_t q);

/* Sample lattice (Sec. 6): in each direction start at the first analysis-domain
 * index 2p, take every M-th index and append the last one, m-2p-1, if M does
 * not land on it.  `indices` (host, optional) receives the concatenated sample
 * indices per direction.  Host only. */
igs_status igs_surrogate_layout(const igs_problem* pb, int32_t M, int32_t q, igs_surrogate_info* out,
                                int32_t* indices, int32_t capacity);

/* Sampling of the face/edge surrogate (igs_assemble_surrogate_fe).  Host only. */
igs_status igs_surrogate_fe_layout(const igs_problem* pb, int32_t M, int32_t q, igs_fe_info* out);

/* Sampling of the per-delta surrogate (igs_assemble_surrogate_pd).  Host only. */
igs_status igs_surrogate_pd_layout(const igs_problem* pb, int32_t M, int32_t q, igs_pd_info* out);

/* Mesh-dependent sampling length (Sec. 7.3.3): M(h) = max{1, floor(c h^e)}
 * with h = 1/nelem and e = (p - q + beta)/(q + 1), so that H = M h obeys
 * H^(q+1) <= c^(q+1) h^(p+1+beta) and, for beta > 0, the consistency error
 * falls faster than the discretisation error under refinement.  c >= 0 is
 * calibrated per problem; the paper uses beta = 1/2.  Evaluated in FP64 as
 * c * nelem^(-e), scaled by (1 + 1e-12) before the floor so that a value that
 * is an integer in exact arithmetic is not rounded down; clamped to 2^30.
 * Returns M >= 1, or IGS_ERR_ARG for nelem < 1, p < 1, q < 1, or c or beta
 * negative or not finite.  Host only. */
int32_t igs_sampling_length(int32_t nelem, int32_t p, int32_t q, double c, double beta);

const char* igs_status_string(int32_t status);
const char* igs_version(void);

/* -------------------------------------------------------------- assembly */

/* Full assembly: every row by Gauss quadrature with nquad^n points per element
 * (Sec. 3.2, eqs. ChangeOfVars and StencilFunction evaluated row by row).
 * form: IGS_STIFFNESS (kappa-weighted, pulled back by K = |det J| J^-1 J^-T,
 * eq. BilinearFormPoissonTensor) or IGS_MASS (int B_i B_j |det J|).
 * dtype: storage type of `band` (device, igs_layout.band_elems elements).
 * Arithmetic is FP64; IGS_F32 rounds on store.  Synchronous on return. */
igs_status igs_assemble_exact(const igs_problem* pb, int32_t form, int32_t dtype, void* band, void* stream);

/* Surrogate assembly (Secs. 4, 5, 6).  Rows outside the analysis domain
 * [2p, m-2p-1]^n and the rows of the sample lattice (igs_surrogate_layout) are
 * assembled by quadrature; for every upper stencil delta the sample values are
 * interpolated by the tensor-product degree-q spline whose knots are the
 * samples (odd q: not-a-knot interior knots s_{(q+1)/2}..s_{S-1-(q+1)/2};
 * even q: midpoints), and
 *   stiffness, eq. 5.1c: upper entries with i, j in the analysis domain are
 *     Phi~_delta(i); lower ones copy the transposed upper entry; other
 *     off-diagonal entries are the exact A_ij (copied from row j's
 *     quadrature); the diagonal of analysis-domain rows is -sum_{k!=i} A~_ik;
 *   mass, eq. 5.1b: as above with the diagonal interpolated too.
 * M = 1 reproduces igs_assemble_exact to rounding.  q in 1..5.
 * dtype IGS_F32 is the precision form: quadrature in FP64 rounded on store,
 * interpolation evaluated in FP32 from FP64-fitted coefficients, FP32
 * diagonal sums.  Synchronous on return.
 * Limits: in 2D, pencils of more than 8192 functions in direction 1, or of
 * 4097..8192 when 2 S1 + m1 values (S1 samples in direction 1) exceed 160 KB
 * of LDS, take a chunked fill whose per-chunk tables must fit in LDS; when
 * they do not (small M on such meshes) the call returns IGS_ERR_UNSUPPORTED. */
igs_status igs_assemble_surrogate(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype,
                                  void* band, void* stream);

/* Surrogate assembly with face- and edge-based stencil functions (Sec. 3.6:
 * besides the stencil functions of the analysis domain, a family for each face
 * and edge layer, exploiting the translation invariance left parallel to it).
 * Row classes: in direction d an index is free in [2p, m_d-2p-1] and
 * otherwise one of the 4p boundary layers; a row's class fixes its layers.
 * Every class with a free direction has, for each upper stencil delta (and
 * delta = 0 for mass), its own stencil function of the free coordinates,
 * sampled on the same lattice as the analysis domain (igs_surrogate_layout)
 * at the class's layers and interpolated by the degree-q tensor spline along
 * the free directions only.  Rows with no free direction (corners, (4p)^n of
 * them) keep their quadrature.  Entries, eq. 5.1c extended to the classes:
 * for i < j the class of i decides (its interpolant at i, exact for a corner
 * row); A~_ji = A~_ij; entries whose partner leaves the index box are 0; the
 * stiffness diagonal is -sum_{k!=i} A~_ik in every row, the mass diagonal is
 * interpolated (exact on corners).  Quadrature runs only on the rows of the
 * tensor product of the per-direction sets layers + lattice
 * (igs_surrogate_fe_layout: 28^3 = 21,952 rows at p = 3, 128^3, M = 8, against
 * 567,028 for igs_assemble_surrogate).  M = 1 reproduces igs_assemble_exact to
 * rounding.  Same arguments, dtype semantics, errors and synchronisation as
 * igs_assemble_surrogate. */
igs_status igs_assemble_surrogate_fe(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype,
                                     void* band, void* stream);

/* Allocation-free assembly, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  M = 0: as igs_assemble_exact; M >= 1: as
 * igs_assemble_surrogate with sampling step M and degree q.  Same arguments,
 * validation, results and errors as those calls, and synchronous on return
 * like them; the caller still passes the band (device, igs_layout.band_elems
 * elements of dtype).  The scratch the kernels use (the 1-D tables, tile and
 * chunk lists, interpolation tables, spline coefficients and the error word)
 * lives in one static device array of IGS_NOALLOC_SCRATCH_BYTES per GPU,
 * held from the first call on that GPU until the process ends; the call makes
 * no hipMalloc, hipMallocAsync or hipFree.  A problem whose scratch exceeds
 * the array returns IGS_ERR_SCRATCH before any GPU work is queued (the 3-D
 * p = 3, 128^3 surrogate with M = 8 needs about 20 MB).  Calls share their
 * GPU's array: calls that overlap in time on one GPU (other host threads,
 * other streams) race and must be serialised by the caller.  Host-side set-up
 * uses ordinary host memory.  IGS_ERR_HIP if the array's device address cannot
 * be obtained. */
#define IGS_NOALLOC_SCRATCH_BYTES (32u << 20)
igs_status igs_assemble_noalloc(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype, void* band,
                                void* stream);

/* Surrogate assembly with a domain per stencil function (Sec. 4: the results
 * hold with the analysis domain replaced by each stencil function's own
 * domain, given an interpolation operator per offset; entries as in Sec. 5).
 * Function i is cardinal when its support spans p+1 uniform knot intervals,
 * i_d in [p, m_d-p-1].  The domain of Phi_delta is the box of rows i with i
 * and i + delta cardinal: per direction [p + max(0,-delta_d),
 * m_d-p-1 - max(0,delta_d)].  Phi_delta (upper delta, and delta = 0 for mass)
 * is sampled on the tensor product of its per-direction samples -- the
 * analysis-domain lattice (igs_surrogate_layout) plus every transition-band
 * index [p, 2p) and [m_d-2p, m_d-p) inside its domain -- and interpolated by
 * the degree-q not-a-knot tensor spline.  Entries: Phi~_delta(i) for upper
 * delta when i and i + delta are cardinal; A~_ji = A~_ij (eq. 5.1b); every
 * other entry exact (a non-cardinal function is involved), 0 outside the index
 * box; stiffness diagonal of cardinal rows -sum_{k!=i} A~_ik (eq. 5.1c), mass
 * diagonal of cardinal rows Phi~_0(i); rows of non-cardinal functions exact.
 * Quadrature runs on the non-cardinal rows and the tensor product of the
 * per-direction sample sets (igs_surrogate_pd_layout: 294,966 + 22^3 rows at
 * p = 3, 128^3, M = 8, against 567,028 for igs_assemble_surrogate).  M = 1
 * reproduces igs_assemble_exact to rounding.  Same arguments, dtype semantics,
 * errors and synchronisation as igs_assemble_surrogate; IGS_ERR_UNSUPPORTED
 * when an offset has more than 2048 samples in a direction. */
igs_status igs_assemble_surrogate_pd(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype,
                                     void* band, void* stream);

/* ---------------------------------------------------------------- plans */

/* A plan keeps what an assembly needs besides the band: the 1-D tables, tile
 * and chunk lists, interpolation tables and coefficient scratch, in device
 * memory owned by the plan.  It is for callers that assemble the same problem
 * repeatedly (an optimisation loop over the coefficient, repeated timing): the
 * host-side setup and the geometry check are paid once.
 *
 * igs_plan_create: M = 0 plans the full assembly (as igs_assemble_exact),
 *   M >= 1 the surrogate assembly with sampling step M and degree q (as
 *   igs_assemble_surrogate).  Same validation and errors as those calls;
 *   synchronises `stream`; *out is NULL on error.  The problem's coefficient
 *   pointer is remembered, the struct itself is not.
 * igs_plan_execute: queues the assembly into `band` (device, the plan's dtype,
 *   igs_layout.band_elems elements) on `stream`.  coef (device, optional)
 *   replaces the spline control values of a SPLINE/EXP_SPLINE problem
 *   ([batch][prod ncoef]); NULL keeps the creation pointer.  The first
 *   execution synchronises `stream` and reports a folding map as
 *   IGS_ERR_GEOMETRY (so does every later execution of that plan); later
 *   executions return once queued.  Executions of one plan must not overlap in
 *   time (they share its scratch): run them on one stream or synchronise.
 * igs_plan_destroy: waits for the last stream the plan ran on, then frees it;
 *   NULL is a no-op. */
typedef struct igs_plan_s* igs_plan;
igs_status igs_plan_create(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype, void* stream,
                           igs_plan* out);
/* igs_plan_create_pd: as igs_plan_create for the per-delta surrogate
 * (igs_assemble_surrogate_pd); M >= 1. */
igs_status igs_plan_create_pd(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype, void* stream,
                              igs_plan* out);
/* igs_plan_create_fe: as igs_plan_create for the face/edge surrogate
 * (igs_assemble_surrogate_fe); M >= 1. */
igs_status igs_plan_create_fe(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype, void* stream,
                              igs_plan* out);
igs_status igs_plan_execute(igs_plan plan, const double* coef, void* band, void* stream);

/* Matrix-free surrogate operator (Sec. 1 names the surrogate's cheap
 * matrix-free application as the goal; remark after eq. 5.1c).  A plan from
 * igs_plan_create_mf (3-D, FP64; same validation as igs_plan_create with
 * M >= 1) executes only what the operator needs: the sample rows, the tensor
 * spline coefficients of every upper stencil function (kept in the plan) and
 * the exact rows outside the analysis domain, written into `band` (the full
 * igs_layout band; its analysis-domain rows are neither written nor read).
 * igs_apply_mf: y = A~ x for the surrogate of eq. 5.1c (5.1b for mass) -- the
 *   analysis-domain rows evaluate Phi~_delta from the coefficients on the fly
 *   (their copied exact entries and the rows outside the domain come from
 *   `band`, which must hold the plan's last execution); dirichlet as in
 *   igs_apply.  x, y: device [batch][N] FP64.  Asynchronous.  2-D plans
 *   (at creation) and meshes whose analysis-domain pencils are too short for
 *   the chunked evaluation (a 768-row chunk touching more than 256 / (S1)
 *   pencils, e.g. 18-row pencils with 6 samples) return IGS_ERR_UNSUPPORTED.
 * igs_solve_cg_mf: FP64 CG with that operator, arguments and stopping rule
 *   as igs_solve_cg without an FP32 band (x0 = u on entry).  Synchronous. */
igs_status igs_plan_create_mf(const igs_problem* pb, int32_t form, int32_t M, int32_t q, void* stream, igs_plan* out);
igs_status igs_apply_mf(igs_plan plan, const double* band, const double* x, double* y, int32_t dirichlet,
                        void* stream);
igs_status igs_solve_cg_mf(igs_plan plan, const double* band, const double* f, double* u, double rtol, int32_t maxit,
                           igs_cg_info* info, void* stream);
igs_status igs_plan_destroy(igs_plan plan);

/* Load vector F(B_i) = int_Omega f B_i dx (Sec. 7, eq. PoissonWeakForm) by
 * the same quadrature; source 0: f = c, source 1: f = c prod_d sin(pi x_d),
 * x = F(xi).  f: device [batch][N] FP64.  Synchronous on return. */
igs_status igs_assemble_rhs(const igs_problem* pb, int32_t source, double c, double* f, void* stream);

/* Asynchronous assembly: the same work as igs_assemble_exact (M = 0) or
 * igs_assemble_surrogate (M >= 1, degree q), and as igs_assemble_rhs, queued
 * on `stream` without waiting for it.  Same arguments, validation and host-side
 * errors (argument and validation errors before any GPU work is queued,
 * IGS_ERR_UNSUPPORTED from the plan before any kernel); the call's device scratch is
 * freed in stream order, so `pb` and host memory may be reused on return, while
 * device inputs (spline coefficients) must stay valid until the stream has run
 * the call.  The device-side error of these calls -- a geometry map whose
 * Jacobian determinant is not positive at some quadrature point (Sec. 3.2,
 * eq. ChangeOfVars needs an invertible map) -- cannot be known on return: each
 * call records it in a status word of (current device, stream), made on the
 * first asynchronous call on that stream (IGS_ERR_HIP if it cannot be made).
 * igs_check(stream) waits for the stream, returns IGS_ERR_GEOMETRY if any
 * asynchronous call queued on it since the last check recorded the error (the
 * band or load vector of that call is then undefined), clears the word, and
 * otherwise returns IGS_OK (also for a stream no asynchronous call has used).
 * Synchronous calls report only their own errors and leave the word alone.
 * Words are kept until the process ends and are keyed by the stream handle:
 * check a stream before destroying it, or a new stream that receives the same
 * handle inherits its record.  Host threads that queue and check on one
 * stream concurrently race. */
igs_status igs_assemble_async(const igs_problem* pb, int32_t form, int32_t M, int32_t q, int32_t dtype, void* band,
                              void* stream);
igs_status igs_assemble_rhs_async(const igs_problem* pb, int32_t source, double c, double* f, void* stream);
igs_status igs_check(void* stream);

/* ---------------------------------------------------------------- solve */

/* y = A x with the band of `dtype` (x, y of the same type, device [batch][N]).
 * dirichlet != 0 applies the Dirichlet restriction of Sec. 6 (remark on
 * boundary conditions, eq. BlockSystem): x is read as 0 and y is written 0 on
 * dofs with some i_d in {0, m_d-1}.  FP32 bands accumulate in FP32.
 * Asynchronous. */
igs_status igs_apply(const igs_problem* pb, int32_t dtype, const void* band, const void* x, void* y,
                     int32_t dirichlet, void* stream);

/* Conjugate gradients for A_II u_I = f_I with homogeneous Dirichlet dofs
 * (Sec. 6, eq. BlockSystem with u_D = 0), per problem of the batch.
 * band64: device FP64 band (required).  band32: optional device FP32 band of
 * the same matrix; when given, CG iterates on A32 with FP32 vectors while the
 * solution accumulates in FP64, and the FP32 recursive residual is replaced by
 * the FP64 residual f - A64 u (FP64 band) whenever it has fallen tenfold since
 * the last replacement or claims convergence: FP64 iterative refinement whose
 * FP32 correction solves keep their search direction.
 * f: device [batch][N]; u: device [batch][N], in: initial guess (Dirichlet
 * entries ignored), out: solution with u_D = 0.  Stops when the FP64 residual
 * satisfies ||f_I - A_II u_I||_2 <= rtol ||f_I||_2 for every problem, or after
 * maxit CG iterations (IGS_NOT_CONVERGED).  info (host) receives counts and
 * the final FP64 relative residual.  Synchronous on return. */
igs_status igs_solve_cg(const igs_problem* pb, const double* band64, const float* band32, const double* f,
                        double* u, double rtol, int32_t maxit, igs_cg_info* info, void* stream);

/* -------------------------------------------------------------- adjoint */

/* Vector-Jacobian product of y = A~(c) x (surrogate with M, q; M = 0 means
 * exact assembly), for spline coefficients (IGS_COEF_SPLINE/EXP_SPLINE):
 *   xbar = A~^T ybar = A~ ybar         (device [batch][N], optional)
 *   cbar = d(ybar^T A~(c) x)/dc         (device [batch][prod ncoef], optional)
 * A~ is linear in the quadrature entries, so cbar pushes the weights
 * ybar_i x_j through the transpose of the surrogate construction onto the
 * quadrature rows and contracts them with dA_ij/dc_k = int dkappa/dc_k
 * grad B_i^T K grad B_j, recomputing Jacobians at the quadrature points.
 * band64 (device) must hold A~(c) when xbar is requested.  Every n and p of
 * the assembly (an element's (p+1)^n x (p+1)^n weight matrix is held in
 * LDS; for n = 3, p = 4 with its contraction tables made one derivative
 * pattern at a time).  Synchronous on return. */
igs_status igs_apply_vjp(const igs_problem* pb, int32_t M, int32_t q, const double* band64, const double* x,
                         const double* ybar, double* xbar, double* cbar, void* stream);

/* Gradient of the compliance J = f^T u, A~(c) u = f (u_D = 0):
 * dJ/dc = -u^T (dA~/dc) u (self-adjoint, no second solve).  u: device
 * [batch][N]; cbar: device [batch][prod ncoef].  Synchronous on return. */
igs_status igs_compliance_grad(const igs_problem* pb, int32_t M, int32_t q, const double* u, double* cbar,
                               void* stream);

/* ------------------------------------------------------------ profiling */

/* Opt-in phase timing (for benchmarks).  When enabled on the calling host
 * thread, every entry point brackets each kernel launch with HIP events on
 * its stream and accumulates per phase (kernel name) the number of launches
 * and their summed GPU duration.  The record is thread-local and is the only
 * state the library keeps between calls; igs_profile_read returns it and
 * clears it.  Reading synchronises the events it reports.  Disabled by
 * default; enabling costs two event records per launch. */
#define IGS_PROFILE_MAX_PHASES 24

typedef struct igs_profile_phase {
  char name[32];
  int32_t launches;
  double ms;                 /* summed duration of the launches */
} igs_profile_phase;

typedef struct igs_profile {
  int32_t nphase;
  igs_profile_phase phase[IGS_PROFILE_MAX_PHASES];
} igs_profile;

igs_status igs_profile_enable(int32_t on);
igs_status igs_profile_read(igs_profile* out);

#ifdef __cplusplus
}
#endif

#endif /* IGS_H */
