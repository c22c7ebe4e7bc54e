"""Pins for the oracle's surrogate with a domain per stencil function (Sec. 4,
the remark after the analysis domain; entries as in Sec. 5):

* the index range of each stencil function's domain matches the cardinal
  B-splines of the open knot vector (brute force over the knots), and the
  intersection over all offsets is the analysis domain, whose centre points
  start at (3p+1)/(2(m-p)) as the paper's closed form states;
* M = 1 samples every cardinal row, so A~ = A;
* polynomial reproduction: identity map with kappa in Q_q gives A~ = A
  (Remark PolynomialReproduction), a Q_2 map with q >= np - 1 gives M~ = M
  (Corollary MassMatrixReproduction);
* the entry error decays like H^{q+1} (Thm. RegularityOfStencilFunctions);
* structure: symmetric, stiffness rows sum to zero (eq. 5.1c), rows of
  non-cardinal functions and entries with a non-cardinal partner are exact;
* the quadrature rows are the non-cardinal rows plus the sample product.
"""
import numpy as np
import pytest

from paper_1904_06971_amd import workloads as W


def _open_knots(nelem, p):
    return np.concatenate([np.zeros(p), np.linspace(0.0, 1.0, nelem + 1), np.ones(p)])


@pytest.mark.parametrize("nelem,p", [(12, 1), (15, 2), (20, 3), (23, 4)])
def test_delta_ranges_are_cardinal_pairs(oracle, nelem, p):
    """Brute force over the knot vector: function i is cardinal when its p+2
    knots are distinct; the domain of offset dd is the set of rows i with i and
    i + dd cardinal; their intersection is [2p, m-2p-1], whose first centre
    (3p+1)/2 h is the paper's lower bound (3p+1)/(2(m-p))."""
    t = _open_knots(nelem, p)
    m = nelem + p
    card = np.array([np.all(np.diff(t[i:i + p + 2]) > 0) for i in range(m)])
    lo, hi = oracle.cardinal_range(m, p)
    assert np.array_equal(np.nonzero(card)[0], np.arange(lo, hi + 1))
    inter = np.ones(m, dtype=bool)
    for dd in range(-p, p + 1):
        want = np.array([card[i] and 0 <= i + dd < m and card[i + dd] for i in range(m)])
        a, b = oracle.delta_range(m, p, dd)
        assert np.array_equal(np.nonzero(want)[0], np.arange(a, b + 1))
        inter &= want
    rows = np.nonzero(inter)[0]
    assert rows[0] == 2 * p and rows[-1] == m - 2 * p - 1
    h = 1.0 / nelem
    centre = 0.5 * (t[rows[0]] + t[rows[0] + p + 1])
    assert abs(centre - (3 * p + 1) / (2 * (m - p))) < 1e-14 and abs(centre - (3 * p + 1) / 2 * h) < 1e-14


def test_lattice_pd_contains_analysis_lattice(oracle):
    m, p, M = 40, 3, 5
    base = oracle.lattice(m, p, M)
    U = oracle.sample_union_pd(m, p, M)
    assert np.array_equal(U, np.unique(np.concatenate([np.arange(p, 2 * p), base, np.arange(m - 2 * p, m - p)])))
    for dd in range(-p, p + 1):
        s = oracle.lattice_pd(m, p, M, dd)
        lo, hi = oracle.delta_range(m, p, dd)
        assert s[0] == lo and s[-1] == hi and np.all(np.diff(s) > 0) and np.all(np.isin(base, s))


@pytest.mark.parametrize("prob,form", [
    (W.problem(2, 2, 20), 0), (W.problem(2, 3, 22, coef="sine3", camp=0.5), 0), (W.problem(2, 2, 20), 1),
    (W.problem(3, 2, 12), 0), (W.problem(3, 2, 12), 1),
])
def test_m1_equals_exact(oracle, prob, form):
    _, N, _ = oracle.dims(prob)
    A = oracle.exact_rows(prob, form, np.arange(N))
    At = oracle.surrogate_pd_rows(prob, form, 1, 3)
    assert np.abs(A - At).max() < 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("n,p,ne,q,deg", [(2, 2, 24, 3, 3), (2, 3, 26, 3, 2), (2, 2, 34, 5, 5), (3, 2, 20, 3, 3)])
@pytest.mark.parametrize("M", [2, 3, 5])
def test_reproduction_polynomial_coefficient(oracle, n, p, ne, q, deg, M):
    """Identity map, kappa a Q_deg polynomial (deg <= q): every stencil function
    lies in Q_q on its own domain and is reproduced."""
    rng = np.random.default_rng(deg + 7)
    cc = 1.5 + 0.3 * rng.standard_normal((deg + 1) ** n)
    prob = W.problem(n, p, ne, geom="identity", coef="spline", cdeg=deg, cn=(deg + 1,) * n, cc=cc)
    _, N, _ = oracle.dims(prob)
    A = oracle.exact_rows(prob, 0, np.arange(N))
    At = oracle.SurrogatePD(prob, 0, M, q).rows(np.arange(N))
    assert np.abs(A - At).max() < 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("M", [2, 4, 6])
def test_mass_reproduction_q2_map(oracle, M):
    """Q_2 geometry map, p = 2, n = 2, q = 3 >= np - 1: M~ = M, while the
    stiffness (a rational integrand) is not reproduced."""
    prob = W.problem(2, 2, 26, geom="poly2", ga=0.3)
    _, N, _ = oracle.dims(prob)
    Mm = oracle.exact_rows(prob, 1, np.arange(N))
    assert np.abs(Mm - oracle.surrogate_pd_rows(prob, 1, M, 3)).max() < 1e-13 * np.abs(Mm).max()
    A = oracle.exact_rows(prob, 0, np.arange(N))
    assert np.abs(A - oracle.surrogate_pd_rows(prob, 0, M, 3)).max() > 1e-10 * np.abs(A).max()


@pytest.mark.slow
@pytest.mark.parametrize("q,rate", [(1, 2.0), (3, 4.0)])
def test_entry_error_rate(oracle, q, rate):
    """||A - A~||_max ~ H^{q+1} at fixed h over cardinal rows (the transition
    bands included); fitted on M = 4 -> 8."""
    prob = W.problem(2, 2, 250)
    _, N, _ = oracle.dims(prob)
    idx = oracle.multi_index(prob, np.arange(N))
    rows = np.nonzero(oracle.cardinal_mask(prob, idx))[0][::7]
    A = oracle.exact_rows(prob, 0, rows)
    off = np.ones(A.shape[1], dtype=bool)
    off[A.shape[1] // 2] = False
    errs = [np.abs(A - oracle.SurrogatePD(prob, 0, M, q).rows(rows))[:, off].max() for M in (4, 8, 16)]
    slope = np.log2(errs[1] / errs[0])
    assert abs(slope - rate) < 0.5, (errs, slope)
    assert errs[2] > errs[1] > errs[0]


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("prob", [W.problem(2, 3, 30, coef="sine3", camp=0.5), W.problem(3, 2, 14)])
def test_structure(oracle, prob, form):
    m, N, S = oracle.dims(prob)
    sur = oracle.SurrogatePD(prob, form, 4, 3)
    R = sur.rows(np.arange(N))
    A = oracle.to_csr(prob, R).toarray()
    sc = np.abs(A).max()
    assert np.abs(A - A.T).max() < 1e-14 * sc * 10
    if form == 0:
        assert np.abs(A.sum(axis=1)).max() < 1e-13 * sc
    E = oracle.exact_rows(prob, form, np.arange(N))
    idx = oracle.multi_index(prob, np.arange(N))
    card = oracle.cardinal_mask(prob, idx)
    # rows of non-cardinal functions are exact
    assert np.array_equal(R[~card], E[~card])
    # entries with a non-cardinal partner are exact
    off = oracle.stencil_offsets(prob)
    mvec = np.array(m)
    for s in range(S):
        if s == (S - 1) // 2:
            continue
        j = idx + off[s]
        inbox = np.all((j >= 0) & (j < mvec), axis=1)
        jc = oracle.cardinal_mask(prob, np.where(inbox[:, None], j, 0))
        sel = card & inbox & ~jc
        assert np.array_equal(R[sel, s], E[sel, s])
    # sample rows keep their exact upper entries wherever they are interpolated
    rows = sur.sample_rows
    Rs, Es = R[rows], E[rows]
    upper = np.arange(S) > (S - 1) // 2
    assert np.abs(Rs[:, upper] - Es[:, upper]).max() < 1e-13 * sc
    # an interpolated entry differs from the exact one
    assert np.abs(R - E).max() > 1e-9 * sc


def test_quadrature_rows(oracle):
    """Non-cardinal rows plus the tensor product of the sample unions; fewer
    than the analysis-domain surrogate's quadrature rows."""
    prob = W.problem(3, 3, 40)
    m, N, _ = oracle.dims(prob)
    p, M = 3, 6
    qr = oracle.quadrature_rows_pd(prob, M)
    U = [oracle.sample_union_pd(m[d], p, M) for d in range(3)]
    nc = N - np.prod([m[d] - 2 * p for d in range(3)])
    assert qr.sum() == nc + np.prod([len(u) for u in U])
    assert qr.sum() < oracle.quadrature_rows(prob, M).sum()


def test_rows_subset_consistent(oracle):
    prob = W.problem(3, 2, 16)
    _, N, _ = oracle.dims(prob)
    sur = oracle.SurrogatePD(prob, 0, 4, 3)
    rows = W.random_rows(N, 300, 11)
    full = sur.rows(np.arange(N))
    assert np.abs(sur.rows(rows) - full[rows]).max() < 1e-15 * np.abs(full).max() * 10
