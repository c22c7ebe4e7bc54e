"""Pins for the oracle's surrogate construction (Secs. 4-6):

* M = 1 samples every analysis-domain row, so A~ = A (Sec. 6);
* polynomial reproduction: identity map with kappa in Q_q gives A~ = A
  (Remark PolynomialReproduction, Prop. PolynomialReproduction); a Q_2 map
  with q >= np-1 gives M~ = M (Corollary MassMatrixReproduction);
* the entry error decays like H^{q+1} = (M h)^{q+1} at fixed h
  (Thm. RegularityOfStencilFunctions with Lemma SplineBAE);
* sample rows keep their exact upper entries; A~ is symmetric; stiffness
  rows sum to zero (eq. 5.1c); mass diagonal is interpolated (eq. 5.1b).
"""
import numpy as np
import pytest

from paper_1904_06971_amd import workloads as W


def _dense(oracle, prob, rows):
    return oracle.to_csr(prob, rows).toarray()


@pytest.mark.parametrize("prob,form", [
    (W.problem(2, 2, 20), 0), (W.problem(2, 3, 22, coef="sine3", camp=0.5), 0), (W.problem(2, 2, 20), 1),
    (W.problem(3, 2, 12), 0), (W.problem(3, 2, 12), 1),
])
def test_m1_equals_exact(oracle, prob, form):
    _, N, _ = oracle.dims(prob)
    A = oracle.exact_rows(prob, form, np.arange(N))
    At = oracle.surrogate_rows(prob, form, 1, 3)
    assert np.abs(A - At).max() < 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("n,p,ne,q,deg", [(2, 2, 24, 3, 3), (2, 3, 26, 3, 2), (2, 2, 34, 5, 5), (3, 2, 20, 3, 3)])
@pytest.mark.parametrize("M", [2, 3, 5])
def test_reproduction_polynomial_coefficient(oracle, n, p, ne, q, deg, M):
    """Identity map, kappa = g with g a single-element degree-`deg` spline (a Q_deg
    polynomial, deg <= q): every stencil function lies in Q_q and is reproduced."""
    rng = np.random.default_rng(deg)
    cc = 1.5 + 0.3 * rng.standard_normal((deg + 1) ** n)
    prob = W.problem(n, p, ne, geom="identity", coef="spline", cdeg=deg, cn=(deg + 1,) * n, cc=cc)
    _, N, _ = oracle.dims(prob)
    A = oracle.exact_rows(prob, 0, np.arange(N))
    sur = oracle.Surrogate(prob, 0, M, q)
    At = sur.rows(np.arange(N))
    assert np.abs(A - At).max() < 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("M", [2, 4, 6])
def test_mass_reproduction_q2_map(oracle, M):
    """Q_2 geometry map, p = 2, n = 2, q = 3 >= np - 1: M~ = M."""
    prob = W.problem(2, 2, 26, geom="poly2", ga=0.3)
    _, N, _ = oracle.dims(prob)
    Mm = oracle.exact_rows(prob, 1, np.arange(N))
    Mt = oracle.surrogate_rows(prob, 1, M, 3)
    assert np.abs(Mm - Mt).max() < 1e-13 * np.abs(Mm).max()
    # and it is not trivially so for the stiffness (rational integrand)
    A = oracle.exact_rows(prob, 0, np.arange(N))
    At = oracle.surrogate_rows(prob, 0, M, 3)
    assert np.abs(A - At).max() > 1e-10 * np.abs(A).max()


@pytest.mark.slow
@pytest.mark.parametrize("q,rate", [(1, 2.0), (3, 4.0)])
def test_entry_error_rate(oracle, q, rate):
    """||A - A~||_max ~ H^{q+1} at fixed h; fitted on M = 4 -> 8."""
    prob = W.problem(2, 2, 250)
    m, N, _ = oracle.dims(prob)
    idx = oracle.multi_index(prob, np.arange(N))
    rows = np.nonzero(oracle.interior_mask(prob, idx))[0][::7]
    A = oracle.exact_rows(prob, 0, rows)
    errs = []
    for M in (4, 8, 16):
        At = oracle.Surrogate(prob, 0, M, q).rows(rows)
        off = np.ones(A.shape[1], dtype=bool)
        off[A.shape[1] // 2] = False
        errs.append(np.abs(A - At)[:, off].max())
    slope = np.log2(errs[1] / errs[0])
    assert abs(slope - rate) < 0.5, (errs, slope)
    assert errs[2] > errs[1] > errs[0]


@pytest.mark.slow
@pytest.mark.parametrize("form,q,rate", [(0, 3, 4.0), (1, 3, 4.0), (0, 1, 2.0)])
def test_entry_error_rate_3d(oracle, form, q, rate):
    """The same rate in 3D (Thm. RegularityOfStencilFunctions holds in any
    dimension): stiffness and mass on the 3D sine map, p = 2, 44^3 elements,
    off-diagonal entries of every 23rd analysis-domain row, M = 4 -> 8."""
    prob = W.problem(3, 2, 44)
    m, N, _ = oracle.dims(prob)
    idx = oracle.multi_index(prob, np.arange(N))
    rows = np.nonzero(oracle.interior_mask(prob, idx))[0][::23]
    A = oracle.exact_rows(prob, form, rows)
    off = np.ones(A.shape[1], dtype=bool)
    off[A.shape[1] // 2] = False
    errs = [np.abs(A - oracle.Surrogate(prob, form, M, q).rows(rows))[:, off].max() for M in (4, 8, 16)]
    slope = np.log2(errs[1] / errs[0])
    assert abs(slope - rate) < 0.5, (errs, slope)
    assert errs[2] > errs[1] > errs[0]


@pytest.mark.parametrize("form", [0, 1])
def test_structure(oracle, form):
    prob = W.problem(2, 3, 30, coef="sine3", camp=0.5)
    m, N, S = oracle.dims(prob)
    sur = oracle.Surrogate(prob, form, 4, 3)
    R = sur.rows(np.arange(N))
    A = _dense(oracle, prob, R)
    sc = np.abs(A).max()
    assert np.abs(A - A.T).max() < 1e-14 * sc * 10
    if form == 0:
        assert np.abs(A.sum(axis=1)).max() < 1e-13 * sc
    # sample rows: upper entries are the exact ones (interpolation property)
    E = oracle.exact_rows(prob, form, sur.sample_rows)
    Rs = R[np.searchsorted(np.arange(N), sur.sample_rows)]
    upper = np.arange(S) > (S - 1) // 2
    assert np.abs(E[:, upper] - Rs[:, upper]).max() < 1e-13 * sc
    # rows outside the analysis domain are exact
    idx = oracle.multi_index(prob, np.arange(N))
    out = ~oracle.interior_mask(prob, idx)
    assert np.array_equal(R[out], oracle.exact_rows(prob, form, np.nonzero(out)[0]))
    # an interpolated row differs from the exact one
    assert np.abs(R - oracle.exact_rows(prob, form, np.arange(N))).max() > 1e-9 * sc


def test_rows_subset_consistent(oracle):
    """Evaluating a subset of rows gives the same numbers as the full band."""
    prob = W.problem(3, 2, 16)
    _, N, _ = oracle.dims(prob)
    sur = oracle.Surrogate(prob, 0, 4, 3)
    rows = W.random_rows(N, 300, 11)
    full = sur.rows(np.arange(N))
    assert np.abs(sur.rows(rows) - full[rows]).max() < 1e-15 * np.abs(full).max() * 10


def test_too_few_samples_rejected(oracle):
    prob = W.problem(2, 2, 14)       # L = m - 4p = 8 analysis rows per direction
    with pytest.raises(ValueError):
        oracle.Surrogate(prob, 0, 4, 3)  # samples 4, 8, 11 -> S = 3 < q + 1
