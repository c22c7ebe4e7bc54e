"""GPU parity of the surrogate with a domain per stencil function
(igs_assemble_surrogate_pd, Sec. 4 remark) against the oracle's SurrogatePD,
element by element, 1e-12 relative in the max norm (FP64): small 2D and 3D
problems in full (several tiles, ragged tails, rectangular meshes, both forms,
q = 1..5, p = 1..4), M = 1 against the full assembly, the structure of eqs.
5.1b/5.1c (bitwise symmetry, zero row sums), the FP32 storage form, batched
spline coefficients, plans, and the 3D p = 3 128^3 workload on sampled rows."""
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


def _rows(oracle, prob, M, seed, count=2500):
    """All rows of a small problem; else a seeded subset: rows of the
    transition bands (cardinal rows with a non-cardinal partner), non-cardinal
    rows, sample rows and random rows."""
    m, N, _ = oracle.dims(prob)
    if N <= 8000:
        return np.arange(N)
    rng = np.random.default_rng(seed)
    p = prob["p"]
    idx = oracle.multi_index(prob, np.arange(N))
    card = oracle.cardinal_mask(prob, idx)
    band = card & np.any((idx < 2 * p) | (idx > np.array(m) - 2 * p - 1), axis=1)
    quad = np.nonzero(oracle.quadrature_rows_pd(prob, M) & card)[0]
    return np.unique(np.concatenate([rng.choice(np.nonzero(band)[0], count // 2), rng.choice(quad, 400),
                                     rng.choice(np.nonzero(~card)[0], 400), rng.integers(0, N, count // 2)]))


PD_CASES = [
    (W.problem(2, 2, 32), 0, 4, 3), (W.problem(2, 3, (70, 41)), 0, 5, 3), (W.problem(2, 2, 50), 1, 4, 3),
    (W.problem(2, 2, 45), 0, 3, 2), (W.problem(2, 3, 90, coef="sine3", camp=0.5), 0, 8, 5),
    (W.problem(2, 1, 66), 0, 4, 1), (W.problem(2, 4, 80), 0, 6, 4), (W.problem(2, 2, 20, geom="poly2", ga=0.3), 1, 3, 3),
    (W.problem(3, 2, 22), 0, 4, 3), (W.problem(3, 3, (26, 24, 25)), 0, 4, 3), (W.problem(3, 3, 26), 1, 4, 3),
    (W.problem(3, 4, (17, 16, 17)), 0, 2, 1), (W.problem(3, 2, 20, coef="sine3", camp=0.5), 0, 3, 2),
    (W.problem(3, 1, (17, 13, 15)), 1, 3, 1), (W.problem(3, 3, 22), 0, 3, 4),
]


@pytest.mark.parametrize("prob,form,M,q", PD_CASES)
def test_pd_small(igs, oracle, prob, form, M, q):
    _, N, _ = oracle.dims(prob)
    print(f"per-delta n={prob['n']} p={prob['p']} nelem={prob['nelem']} form={form} M={M} q={q}", flush=True)
    band = igs.assemble_surrogate_pd(prob, form, M=M, q=q)
    rows = _rows(oracle, prob, M, N % 97)
    got = gather_rows(band, rows)
    print(f"  GPU done; oracle on {len(rows)} of {N} rows ...", flush=True)
    ref = oracle.SurrogatePD(prob, form, M, q).rows(rows)
    assert rel_maxnorm(got, ref) < TOL64
    lay = igs.layout(prob)
    if lay.ld > N:
        assert float(band[:, :, N:].abs().max()) == 0.0


@pytest.mark.parametrize("prob,form", [(W.problem(2, 3, 30), 0), (W.problem(3, 2, 14), 0), (W.problem(3, 2, 14), 1)])
def test_pd_m1_equals_exact(igs, oracle, prob, form):
    a = igs.band_rows(igs.assemble_exact(prob, form), prob)
    t = igs.band_rows(igs.assemble_surrogate_pd(prob, form, M=1, q=3), prob)
    assert rel_maxnorm(t, a) < 1e-13


@pytest.mark.parametrize("prob", [W.problem(3, 3, 22), W.problem(2, 3, (61, 47))])
def test_pd_structure(igs, oracle, prob):
    """Symmetry: bitwise for every pair with a cardinal row (an interpolated
    entry and its mirror come from the same evaluation; an exact entry and its
    mirror from one quadrature row, in 3-D by its transposed store), to
    rounding for pairs of non-cardinal rows (two quadrature rows, as in the
    full assembly); zero row sums; exact rows of non-cardinal functions."""
    m, N, S = oracle.dims(prob)
    band = igs.assemble_surrogate_pd(prob, 0, M=4, q=3)
    R = igs.band_rows(band, prob)
    print("  GPU done; oracle ...", flush=True)
    A = oracle.to_csr(prob, R)
    idx = oracle.multi_index(prob, np.arange(N))
    card = oracle.cardinal_mask(prob, idx)
    D = abs(A - A.T).tocoo()
    withcard = card[D.row] | card[D.col]
    if prob["n"] == 3:
        assert D.data[withcard].max(initial=0.0) == 0.0
    assert D.max() <= 1e-15 * abs(A).max()
    assert np.abs(np.asarray(A.sum(axis=1))).max() < 1e-13 * abs(A).max()
    nc = np.nonzero(~card)[0]
    assert rel_maxnorm(R[nc], oracle.exact_rows(prob, 0, nc)) < TOL64


def test_pd_fp32(igs, oracle):
    import torch

    prob = W.problem(3, 3, 20)
    band = igs.assemble_surrogate_pd(prob, 0, M=4, q=3, dtype=torch.float32)
    rows = _rows(oracle, prob, 4, 5)
    print("  GPU done; oracle ...", flush=True)
    ref = oracle.SurrogatePD(prob, 0, 4, 3).rows(rows)
    assert rel_maxnorm(gather_rows(band, rows).astype(np.float64), ref) < 2e-6
    prob = W.problem(2, 2, 40)
    band = igs.assemble_surrogate_pd(prob, 1, M=4, q=3, dtype=torch.float32)
    ref = oracle.SurrogatePD(prob, 1, 4, 3).rows(np.arange(oracle.dims(prob)[1]))
    assert rel_maxnorm(igs.band_rows(band, prob).astype(np.float64), ref) < 2e-6


def test_pd_batched_spline(igs, oracle):
    rng = np.random.default_rng(13)
    cc = rng.normal(0, 0.5, (3, 125))
    prob = W.problem(3, 2, 16, coef="exp_spline", cdeg=3, cn=(5, 5, 5), cc=cc, batch=3)
    band = igs.assemble_surrogate_pd(prob, 0, M=3, q=3)
    for b in range(3):
        print(f"  oracle problem {b} ...", flush=True)
        ref = oracle.SurrogatePD(prob, 0, 3, 3, b=b).rows(np.arange(oracle.dims(prob)[1]))
        assert rel_maxnorm(igs.band_rows(band, prob, b), ref) < TOL64


def test_pd_plan_matches_one_shot(igs):
    prob = W.problem(3, 3, 20, coef="sine3", camp=0.5)
    a = igs.assemble_surrogate_pd(prob, 0, M=4, q=3)
    pl = igs.Plan(prob, 0, M=4, q=3, per_delta=True)
    b = pl.execute()
    c = pl.execute()
    pl.close()
    assert float((a - b).abs().max()) == 0.0 and float((b - c).abs().max()) == 0.0


def test_pd_c4_sampled(igs, oracle):
    """3D p=3 128^3, M = 8, q = 3: transition-band rows, sample rows,
    non-cardinal rows and random rows of the per-delta surrogate."""
    prob = W.c4_precision3d()
    m, N, _ = oracle.dims(prob)
    info = igs.surrogate_pd_layout(prob, 8, 3)
    assert info.quadrature_rows == int(oracle.quadrature_rows_pd(prob, 8).sum())
    rows = _rows(oracle, prob, 8, 23, count=3000)
    band = igs.assemble_surrogate_pd(prob, 0, M=8, q=3)
    got = gather_rows(band, rows)
    del band
    print(f"  GPU done; oracle fit and rows ({len(rows)}) ...", flush=True)
    err = rel_maxnorm(got, oracle.SurrogatePD(prob, 0, 8, 3).rows(rows))
    print(f"3D p=3 128^3 per-delta surrogate M=8 q=3, {len(rows)} rows: max rel error {err:.2e}")
    assert err < TOL64
