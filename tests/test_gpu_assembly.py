"""GPU parity: exact and surrogate band rows from the HIP kernels against the
FP64 CPU oracle, element by element, 1e-12 relative in the max norm (FP64).
Small problems are compared in full (several tiles, ragged tails); the
workload sizes are compared on sampled rows."""
import numpy as np
import pytest

from gpu_util import gather_rows, rel_maxnorm
from paper_1904_06971_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


@pytest.fixture(scope="module")
def igs():
    import torch

    assert torch.cuda.is_available()
    from paper_1904_06971_amd import igs as m

    m.lib()
    return m


def _full(igs, band, prob, b=0):
    return igs.band_rows(band, prob, b)


EXACT_CASES = [
    (W.problem(2, 1, 70), 0), (W.problem(2, 2, 33), 0), (W.problem(2, 3, (67, 21)), 0), (W.problem(2, 4, 29), 0),
    (W.problem(2, 2, 33), 1), (W.problem(2, 3, 40, geom="identity"), 1),
    (W.problem(2, 3, 26, coef="sine3", camp=0.5), 0), (W.problem(2, 2, 20, geom="poly2", ga=0.3), 0),
    (W.problem(3, 1, (19, 9, 7)), 0), (W.problem(3, 2, (11, 9, 8)), 0), (W.problem(3, 3, (10, 9, 11)), 0),
    (W.problem(3, 4, (9, 7, 8)), 0), (W.problem(3, 3, (10, 9, 11)), 1), (W.problem(3, 4, 8), 1),
    (W.problem(3, 3, 9, coef="sine3", camp=0.5), 0), (W.problem(3, 2, 9, geom="poly2", ga=0.2), 1),
]


@pytest.mark.parametrize("prob,form", EXACT_CASES)
def test_exact_small(igs, oracle, prob, form):
    _, N, _ = oracle.dims(prob)
    band = igs.assemble_exact(prob, form)
    ref = oracle.exact_rows(prob, form, np.arange(N))
    assert rel_maxnorm(_full(igs, band, prob), ref) < TOL64
    lay = igs.layout(prob)
    if lay.ld > N:
        assert float(band[:, :, N:].abs().max()) == 0.0


def test_exact_batched_spline(igs, oracle):
    rng = np.random.default_rng(0)
    cc = rng.normal(0, 0.5, (3, 36))
    prob = W.problem(2, 3, 30, coef="exp_spline", cdeg=3, cn=(6, 6), cc=cc, batch=3)
    band = igs.assemble_exact(prob, 0)
    _, N, _ = oracle.dims(prob)
    for b in range(3):
        ref = oracle.exact_rows(prob, 0, np.arange(N), b=b)
        assert rel_maxnorm(_full(igs, band, prob, b), ref) < TOL64


def test_exact_fp32_storage(igs, oracle):
    import torch

    prob = W.problem(3, 3, 12)
    _, N, _ = oracle.dims(prob)
    band = igs.assemble_exact(prob, 0, dtype=torch.float32)
    ref = oracle.exact_rows(prob, 0, np.arange(N))
    err = rel_maxnorm(_full(igs, band, prob), ref)
    assert err < 1e-7


SUR_CASES = [
    (W.problem(2, 2, 32), 0, 4, 3), (W.problem(2, 3, 70), 0, 5, 3), (W.problem(2, 2, 50), 1, 4, 3),
    (W.problem(2, 2, 45), 0, 3, 2), (W.problem(2, 3, 90, coef="sine3", camp=0.5), 0, 8, 5),
    (W.problem(2, 1, 66), 0, 4, 1), (W.problem(2, 4, 80), 0, 6, 4),
    (W.problem(3, 2, 22), 0, 4, 3), (W.problem(3, 3, (26, 24, 25)), 0, 4, 3), (W.problem(3, 3, 26), 1, 4, 3),
    (W.problem(3, 4, 30), 0, 5, 3), (W.problem(3, 2, 20, coef="sine3", camp=0.5), 0, 3, 2),
]


@pytest.mark.parametrize("prob,form,M,q", SUR_CASES)
def test_surrogate_small(igs, oracle, prob, form, M, q):
    _, N, _ = oracle.dims(prob)
    band = igs.assemble_surrogate(prob, form, M=M, q=q)
    ref = oracle.surrogate_rows(prob, form, M, q)
    assert rel_maxnorm(_full(igs, band, prob), ref) < TOL64


@pytest.mark.parametrize("ne,c", [(96, 0.75), (96, 3.0), (200, 0.75), (200, 3.0)])
def test_surrogate_mesh_dependent_q5(igs, oracle, ne, c):
    """2D p = 2, q = 5 with the mesh-dependent sampling length M(h) (beta = 1/2)
    of the paper's timing study: the library's M equals the oracle's and the
    band matches the oracle's surrogate."""
    M = oracle.sampling_length(ne, 2, 5, c, 0.5)
    assert igs.sampling_length(ne, 2, 5, c, 0.5) == M
    prob = W.problem(2, 2, ne)
    print(f"nelem {ne} c {c}: M = {M}")
    band = igs.assemble_surrogate(prob, 0, M=M, q=5)
    ref = oracle.surrogate_rows(prob, 0, M, 5)
    assert rel_maxnorm(_full(igs, band, prob), ref) < TOL64


@pytest.mark.parametrize("prob,form", [(W.problem(2, 3, 30), 0), (W.problem(3, 2, 14), 0), (W.problem(3, 2, 14), 1)])
def test_surrogate_m1_equals_exact(igs, oracle, prob, form):
    a = igs.band_rows(igs.assemble_exact(prob, form), prob)
    t = igs.band_rows(igs.assemble_surrogate(prob, form, M=1, q=3), prob)
    assert rel_maxnorm(t, a) < 1e-13


@pytest.mark.parametrize("prob,form,M,q", [
    (W.problem(2, 2, 37), 0, 4, 3), (W.problem(2, 3, (70, 41)), 1, 5, 5), (W.problem(2, 2, 140), 0, 3, 5),
    (W.problem(3, 2, 14), 0, 3, 3), (W.problem(3, 3, 20), 1, 4, 3),
])
def test_surrogate_writes_every_word(igs, oracle, prob, form, M, q):
    """Into a band filled with NaN first, with a plan executed twice: every
    row equals the oracle's and the padding columns are zero.  In 2D the rows
    outside the analysis domain come from the quadrature launch that runs
    before the fill (which stores only domain rows), and the fill zeroes the
    padding; the sample grids take the one-launch fit up to 1024 values and the
    two passes above (140^2 elements, M = 3: 45 x 45 samples)."""
    import torch

    _, N, _ = oracle.dims(prob)
    band = igs.empty_band(prob, torch.float64)
    band.fill_(float("nan"))
    pl = igs.Plan(prob, form, M=M, q=q)
    pl.execute(out=band)
    band.fill_(float("nan"))
    pl.execute(out=band)
    pl.close()
    ref = oracle.surrogate_rows(prob, form, M, q)
    assert rel_maxnorm(_full(igs, band, prob), ref) < TOL64
    if igs.layout(prob).ld > N:
        assert float(band[:, :, N:].abs().max()) == 0.0


def test_surrogate_structure(igs, oracle):
    """Bitwise symmetry of interpolated pairs and zero row sums (eq. 5.1c)."""
    prob = W.problem(3, 3, 30)
    band = igs.assemble_surrogate(prob, 0, M=4, q=3)
    R = _full(igs, band, prob)
    A = oracle.to_csr(prob, R)
    d = abs(A - A.T)
    assert d.max() <= 1e-15 * abs(A).max()
    assert np.abs(np.asarray(A.sum(axis=1))).max() < 1e-13 * abs(A).max()


def test_surrogate_fp32(igs, oracle):
    import torch

    prob = W.problem(3, 3, 28)
    band = igs.assemble_surrogate(prob, 0, M=4, q=3, dtype=torch.float32)
    ref = oracle.surrogate_rows(prob, 0, 4, 3)
    got = _full(igs, band, prob)
    assert rel_maxnorm(got, ref) < 2e-6


@pytest.mark.parametrize("prob,form,M,q", [
    (W.problem(2, 3, (70, 41)), 0, 5, 5), (W.problem(2, 2, (37, 66)), 1, 4, 2),
    (W.problem(2, 4, (60, 47), coef="sine3", camp=0.5), 0, 6, 3), (W.problem(2, 1, (300, 23)), 0, 7, 1),
    # m1 = 4096, the widest pencil of the per-pencil 2D fill (1024 threads x 4 rows)
    (W.problem(2, 1, (4095, 8)), 0, 2, 1),
])
def test_surrogate_2d_rectangular(igs, oracle, prob, form, M, q):
    """2D fill on meshes with m1 != m2 (pencils of one direction, lattices of
    the other), stiffness and mass, even and odd q."""
    band = igs.assemble_surrogate(prob, form, M=M, q=q)
    ref = oracle.surrogate_rows(prob, form, M, q)
    assert rel_maxnorm(_full(igs, band, prob), ref) < TOL64


@pytest.mark.parametrize("prob,form,M,q", [
    (W.problem(3, 1, (200, 5, 5)), 0, 1, 1), (W.problem(3, 1, (5, 200, 5)), 1, 1, 1),
    (W.problem(3, 1, (5, 5, 200)), 0, 1, 1), (W.problem(2, 2, 230), 0, 1, 5), (W.problem(2, 2, (60, 230)), 1, 1, 3),
])
def test_surrogate_fit_tiled(igs, oracle, prob, form, M, q):
    """At least 192 samples in a direction: the fit runs as tiled products
    (each direction long in turn in 3D; 2D stiffness and mass)."""
    band = igs.assemble_surrogate(prob, form, M=M, q=q)
    ref = oracle.surrogate_rows(prob, form, M, q)
    assert rel_maxnorm(_full(igs, band, prob), ref) < TOL64


def test_surrogate_fit_tiled_fp32(igs, oracle):
    """The FP32 form of the tiled fit (FP32 sample rows gathered into the FP64
    products): 2D p = 2, 230^2 elements, M = 1, q = 5 (226 samples per
    direction), at FP32 resolution."""
    import torch

    prob = W.problem(2, 2, 230)
    band = igs.assemble_surrogate(prob, 0, M=1, q=5, dtype=torch.float32)
    ref = oracle.surrogate_rows(prob, 0, 1, 5)
    assert rel_maxnorm(_full(igs, band, prob), ref) < 2e-6


def test_surrogate_fit_tiled_batch(igs, oracle):
    """Tiled fit over a batch of two coefficient fields (2D, 197 x 197 samples)."""
    rng = np.random.default_rng(41)
    cc = rng.normal(0, 0.4, (2, 25))
    prob = W.problem(2, 1, 200, coef="exp_spline", cdeg=2, cn=(5, 5), cc=cc, batch=2)
    band = igs.assemble_surrogate(prob, 0, M=1, q=3)
    for b in range(2):
        ref = oracle.surrogate_rows(prob, 0, 1, 3, b=b)
        assert rel_maxnorm(igs.band_rows(band, prob, b), ref) < TOL64


@pytest.mark.parametrize("prob,form,M,q,f32", [
    (W.problem(2, 1, (4200, 8)), 0, 2, 1, False), (W.problem(2, 1, (4200, 8)), 0, 16, 1, False),
    (W.problem(2, 2, (4300, 12)), 1, 2, 3, False), (W.problem(2, 1, (4200, 8)), 0, 2, 1, True),
    # m1 = 8192, the widest pencil of the reloaded-weight fill (1024 threads x 8 rows)
    (W.problem(2, 1, (8191, 5)), 0, 4, 1, False),
])
def test_surrogate_2d_wide(igs, oracle, prob, form, M, q, f32):
    """Pencils of 4097 to 8192 functions in direction 1: the 2D fill with the
    direction-1 weights reloaded per delta (eight rows per thread), stiffness
    and mass, FP64 and FP32 storage."""
    import torch

    band = igs.assemble_surrogate(prob, form, M=M, q=q, dtype=torch.float32 if f32 else torch.float64)
    ref = oracle.surrogate_rows(prob, form, M, q)
    assert rel_maxnorm(_full(igs, band, prob), ref) < (2e-6 if f32 else TOL64)


def test_surrogate_2d_too_wide(igs):
    """Past 8192 functions in direction 1 (or when the 2D fill's pencil and
    coefficient lines exceed LDS) the chunked fill takes over, whose per-chunk
    tables outgrow LDS at small sampling steps: a clean IGS_ERR_UNSUPPORTED
    from the plan, before any kernel runs."""
    prob = W.problem(2, 1, (8300, 8))
    with pytest.raises(igs.IGSError) as e:
        igs.assemble_surrogate(prob, 0, M=2, q=1)
    assert e.value.status == -2


@pytest.mark.parametrize("form", [0, 1])
def test_surrogate_2d_fp32(igs, oracle, form):
    """2D precision form (FP32 fill from FP64-fitted coefficients)."""
    import torch

    prob = W.problem(2, 3, (90, 77))
    band = igs.assemble_surrogate(prob, form, M=6, q=3, dtype=torch.float32)
    ref = oracle.surrogate_rows(prob, form, 6, 3)
    assert rel_maxnorm(_full(igs, band, prob), ref) < 2e-6


def test_geometry_fold_reported(igs):
    """A sine map with amplitude 0.5 folds (det J < 0 somewhere)."""
    prob = W.problem(2, 2, 16, ga=0.5)
    with pytest.raises(igs.IGSError) as e:
        igs.assemble_exact(prob, 0)
    assert e.value.status == -5


def test_async_calls_and_check(igs):
    """igs_assemble_async and igs_assemble_rhs_async queue the kernels of the
    synchronous calls (bitwise equal results).  A folding geometry returns
    IGS_OK at call time; igs_check on the same stream reports
    IGS_ERR_GEOMETRY once and clears it, and a check on another stream does
    not see it."""
    import torch

    prob = W.problem(2, 2, 32)
    for M in (0, 4):
        ref = igs.assemble_exact(prob, 0) if M == 0 else igs.assemble_surrogate(prob, 0, M=M, q=3)
        out = igs.assemble_async(prob, 0, M=M, q=3)
        igs.check()
        assert torch.equal(out, ref)
    ref = igs.assemble_rhs(prob, 1, 2.0)
    out = igs.assemble_rhs_async(prob, 1, 2.0)
    igs.check()
    assert torch.equal(out, ref)

    bad = W.problem(2, 2, 16, ga=0.5)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        igs.assemble_async(bad, 0)
        igs.assemble_rhs_async(bad, 0, 1.0)
        igs.assemble_async(prob, 0, M=4, q=3)
    igs.check()  # the current (default) stream has no error recorded
    with torch.cuda.stream(side):
        with pytest.raises(igs.IGSError) as e:
            igs.check()
        assert e.value.status == -5
        igs.check()  # cleared by the previous check
        out = igs.assemble_async(prob, 1, M=4, q=3)
        igs.check()
    assert torch.equal(out, igs.assemble_surrogate(prob, 1, M=4, q=3))


# ------------------------------------------------------------------ plans ---
@pytest.mark.parametrize("prob,form,M,q", [(W.problem(3, 3, (26, 24, 25)), 0, 4, 3), (W.problem(2, 2, 32), 1, 4, 3),
                                           (W.problem(3, 2, 12), 0, 0, 0)])
def test_plan_matches_one_shot(igs, prob, form, M, q):
    """A kept plan runs the same kernels: bitwise equal to the one-shot call,
    on its first (synchronising) and later (queue-only) executions."""
    import torch

    ref = igs.assemble_surrogate(prob, form, M=M, q=q) if M else igs.assemble_exact(prob, form)
    plan = igs.Plan(prob, form, M=M, q=q)
    for _ in range(3):
        band = plan.execute()
        torch.cuda.synchronize()
        assert torch.equal(band, ref)
    plan.close()


def test_plan_coefficient_swap(igs, oracle):
    """Executing a plan with new spline control values equals the oracle for
    those values (the batched exp-spline coefficient of the adjoint workload)."""
    rng = np.random.default_rng(4)
    cc0 = rng.normal(0, 0.5, (2, 36))
    cc1 = rng.normal(0, 0.5, (2, 36))
    prob0 = W.problem(2, 3, 30, coef="exp_spline", cdeg=3, cn=(6, 6), cc=cc0, batch=2)
    prob1 = W.problem(2, 3, 30, coef="exp_spline", cdeg=3, cn=(6, 6), cc=cc1, batch=2)
    import torch

    plan = igs.Plan(prob0, 0, M=4, q=3)
    band = plan.execute(coef=torch.as_tensor(cc1, device="cuda"))
    _, N, _ = oracle.dims(prob1)
    for b in range(2):
        ref = oracle.surrogate_rows(prob1, 0, 4, 3, b=b)
        assert rel_maxnorm(_full(igs, band, prob1, b), ref) < TOL64
    band = plan.execute()  # creation coefficients again
    ref = oracle.surrogate_rows(prob0, 0, 4, 3, b=1)
    assert rel_maxnorm(_full(igs, band, prob0, 1), ref) < TOL64
    plan.close()


def test_plan_geometry_fold(igs):
    prob = W.problem(2, 2, 16, ga=0.5)
    plan = igs.Plan(prob, 0, M=0, q=0)
    for _ in range(2):
        with pytest.raises(igs.IGSError) as e:
            plan.execute()
        assert e.value.status == -5
    plan.close()


# ------------------------------------------------------------ full sizes ---
def _sampled(oracle, prob, M, seed, count=4096):
    _, N, _ = oracle.dims(prob)
    m = oracle.dims(prob)[0]
    samp = [oracle.lattice(m[d], prob["p"], M) for d in range(prob["n"])]
    g = np.meshgrid(*samp[::-1], indexing="ij")
    srows = oracle.flat_index(prob, np.stack([x.ravel() for x in g[::-1]], axis=1))
    rnd = W.random_rows(N, count, seed)
    return np.unique(np.concatenate([srows, rnd]))


@pytest.mark.parametrize("M", [4, 8, 16])
def test_c2_surrogate_sampled(igs, oracle, M):
    prob = W.c2_poisson3d()
    rows = _sampled(oracle, prob, M, 20 + M, 1500)
    for form in (0, 1):
        band = igs.assemble_surrogate(prob, form, M=M, q=3)
        ref = oracle.Surrogate(prob, form, M, 3).rows(rows)
        assert rel_maxnorm(gather_rows(band, rows), ref) < TOL64
        del band


def test_c2_exact_sampled(igs, oracle):
    prob = W.c2_poisson3d()
    _, N, _ = oracle.dims(prob)
    rows = W.random_rows(N, 3000, 7)
    for form in (0, 1):
        band = igs.assemble_exact(prob, form)
        ref = oracle.exact_rows(prob, form, rows)
        assert rel_maxnorm(gather_rows(band, rows), ref) < TOL64
        del band


def test_c4_surrogate_and_exact_sampled(igs, oracle):
    prob = W.c4_precision3d()
    rows = _sampled(oracle, prob, 8, 4, 2048)
    band = igs.assemble_surrogate(prob, 0, M=8, q=3)
    ref = oracle.Surrogate(prob, 0, 8, 3).rows(rows)
    err = rel_maxnorm(gather_rows(band, rows), ref)
    print(f"3D p=3 128^3 surrogate M=8 q=3, {len(rows)} rows: max rel error {err:.2e}")
    assert err < TOL64
    del band
    band = igs.assemble_exact(prob, 0)
    _, N, _ = oracle.dims(prob)
    rr = W.random_rows(N, 1500, 5)
    err = rel_maxnorm(gather_rows(band, rr), oracle.exact_rows(prob, 0, rr))
    print(f"3D p=3 128^3 exact, {len(rr)} rows: max rel error {err:.2e}")
    assert err < TOL64


def test_c4_surrogate_fp32_sampled(igs, oracle):
    """Precision form: FP32 storage of the 3D p=3 128^3 surrogate (fill in FP32
    with FP32 accumulation) against the FP64 oracle on sampled rows."""
    import torch

    prob = W.c4_precision3d()
    rows = _sampled(oracle, prob, 8, 6, 2048)
    band = igs.assemble_surrogate(prob, 0, M=8, q=3, dtype=torch.float32)
    err = rel_maxnorm(gather_rows(band, rows).astype(np.float64), oracle.Surrogate(prob, 0, 8, 3).rows(rows))
    print(f"3D p=3 128^3 surrogate in FP32 storage, {len(rows)} rows: max rel error {err:.2e}")
    assert err < 2e-6


def test_c3_surrogate_sampled(igs, oracle):
    """p = 4 variable coefficient: all sample rows plus 4096 seeded random rows."""
    prob = W.c3_varcoef3d()
    _, N, _ = oracle.dims(prob)
    m = oracle.dims(prob)[0]
    rnd = np.random.default_rng(3).integers(0, N, 4096)
    band = igs.assemble_surrogate(prob, 0, M=8, q=3)
    sur = oracle.Surrogate(prob, 0, 8, 3)
    rows = np.unique(np.concatenate([sur.sample_rows, rnd]))
    err = rel_maxnorm(gather_rows(band, rows), sur.rows(rows))
    print(f"3D p=4 128^3 variable coefficient surrogate, {len(rows)} rows: max rel error {err:.2e}")
    assert err < TOL64


# ------------------------------------------------- more surrogate cases ---
def test_surrogate_batched_spline_3d(igs, oracle):
    """3D surrogate of a batch of two exp-spline coefficient fields: the fill,
    copy and quadrature kernels index the batch through the grid."""
    rng = np.random.default_rng(11)
    cc = rng.normal(0, 0.3, (2, 5 * 5 * 5))
    prob = W.problem(3, 2, (18, 16, 17), coef="exp_spline", cdeg=2, cn=(5, 5, 5), cc=cc, batch=2)
    band = igs.assemble_surrogate(prob, 0, M=4, q=3)
    for b in range(2):
        ref = oracle.surrogate_rows(prob, 0, 4, 3, b=b)
        assert rel_maxnorm(_full(igs, band, prob, b), ref) < TOL64


@pytest.mark.parametrize("prob,form,M,q", [(W.problem(2, 3, 70), 0, 5, 3), (W.problem(3, 3, 24), 1, 4, 3),
                                           (W.problem(2, 2, 50), 1, 4, 3)])
def test_surrogate_fp32_more(igs, oracle, prob, form, M, q):
    """FP32 storage (fill in FP32 with FP32 accumulation) in 2D and for the
    mass form, against the FP64 oracle at FP32 resolution."""
    import torch

    band = igs.assemble_surrogate(prob, form, M=M, q=q, dtype=torch.float32)
    ref = oracle.surrogate_rows(prob, form, M, q)
    assert rel_maxnorm(_full(igs, band, prob), ref) < 2e-6


@pytest.mark.parametrize("prob,M,q", [(W.problem(3, 2, 19), 5, 3), (W.problem(2, 3, 40), 11, 3),
                                      (W.problem(3, 1, 14), 10, 1)])
def test_surrogate_few_samples(igs, oracle, prob, M, q):
    """Sampling steps that leave exactly q+1 samples in a direction (the
    smallest lattice the interpolant accepts), with a shorter last interval."""
    m, N, _ = oracle.dims(prob)
    assert min(len(oracle.lattice(m[d], prob["p"], M)) for d in range(prob["n"])) == q + 1
    band = igs.assemble_surrogate(prob, 0, M=M, q=q)
    ref = oracle.surrogate_rows(prob, 0, M, q)
    assert rel_maxnorm(_full(igs, band, prob), ref) < TOL64
