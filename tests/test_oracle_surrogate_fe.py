"""Pins for the oracle's face/edge surrogate (Sec. 3.6: stencil functions that
exploit the translation invariance left parallel to faces and edges; the
reading is stated in oracle.SurrogateFE):

* M = 1 samples every row of every class, so A~ = A (as for Sec. 6's M = 1);
* polynomial reproduction: identity map with kappa in Q_q makes every class's
  stencil function a Q_q polynomial of its free coordinates (the free
  directions enter through translates only), so A~ = A for every M, boundary
  rows included (Remark PolynomialReproduction, extended to the classes);
* the entry error decays like H^{q+1} at fixed h on the boundary rows too
  (Thm. RegularityOfStencilFunctions along the free directions);
* symmetry and zero stiffness row sums by construction (eq. 5.1c extended);
  sample rows of every class keep their exact upper entries; corner rows
  keep exact upper entries;
* interior rows whose whole stencil stays in the analysis domain equal the
  analysis-domain surrogate's rows (both use the same interior interpolant).
"""
import numpy as np
import pytest

from paper_1904_06971_amd import workloads as W


def _dense(oracle, prob, rows):
    return oracle.to_csr(prob, rows).toarray()


@pytest.mark.parametrize("prob,form", [
    (W.problem(2, 2, 20), 0), (W.problem(2, 3, 22, coef="sine3", camp=0.5), 0), (W.problem(2, 2, 20), 1),
    (W.problem(2, 1, (15, 19)), 0), (W.problem(3, 1, 9), 0), (W.problem(3, 2, 11), 1),
])
def test_fe_m1_equals_exact(oracle, prob, form):
    _, N, _ = oracle.dims(prob)
    A = oracle.exact_rows(prob, form, np.arange(N))
    At = oracle.surrogate_fe_rows(prob, form, 1, 3 if min(prob["nelem"]) > 12 else 1)
    assert np.abs(A - At).max() < 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("n,p,ne,q,deg,M", [(2, 2, 24, 3, 3, 2), (2, 2, 24, 3, 3, 5), (2, 3, 26, 3, 2, 3),
                                            (2, 2, 34, 5, 5, 4), (2, 1, 30, 2, 2, 3), (3, 2, 20, 3, 3, 3),
                                            (3, 1, 16, 2, 2, 4)])
def test_fe_reproduction_polynomial_coefficient(oracle, n, p, ne, q, deg, M):
    """Identity map, kappa a Q_deg polynomial (deg <= q): every row, boundary
    layers included, is reproduced for every sampling step."""
    rng = np.random.default_rng(deg + 10 * n)
    cc = 1.5 + 0.3 * rng.standard_normal((deg + 1) ** n)
    prob = W.problem(n, p, ne, geom="identity", coef="spline", cdeg=deg, cn=(deg + 1,) * n, cc=cc)
    _, N, _ = oracle.dims(prob)
    A = oracle.exact_rows(prob, 0, np.arange(N))
    At = oracle.surrogate_fe_rows(prob, 0, M, q)
    assert np.abs(A - At).max() < 1e-12 * np.abs(A).max()
    # the mass form on the identity map has constant stencil functions
    Mm = oracle.exact_rows(prob, 1, np.arange(N))
    assert np.abs(Mm - oracle.surrogate_fe_rows(prob, 1, M, q)).max() < 1e-12 * np.abs(Mm).max()


@pytest.mark.slow
@pytest.mark.parametrize("q,rate", [(1, 2.0), (3, 4.0)])
def test_fe_entry_error_rate(oracle, q, rate):
    """||A - A~||_max ~ H^{q+1} at fixed h, over the boundary-layer rows alone
    (the rows the face/edge functions add) and over all rows; M = 4 -> 8."""
    prob = W.problem(2, 2, 200)
    m, N, S = oracle.dims(prob)
    rows = np.arange(N)[::5]
    idx = oracle.multi_index(prob, rows)
    bnd = np.any(oracle.row_class(prob, idx) >= 0, axis=1)
    A = oracle.exact_rows(prob, 0, rows)
    off = np.ones(S, dtype=bool)
    off[S // 2] = False
    errs, errb = [], []
    for M in (4, 8, 16):
        e = np.abs(A - oracle.SurrogateFE(prob, 0, M, q).rows(rows))[:, off]
        errs.append(e.max())
        errb.append(e[bnd].max())
    for er in (errs, errb):
        slope = np.log2(er[1] / er[0])
        assert abs(slope - rate) < 0.5, (er, slope)
        assert er[2] > er[1] > er[0]


@pytest.mark.parametrize("prob,form,M,q", [(W.problem(2, 3, 30, coef="sine3", camp=0.5), 0, 4, 3),
                                           (W.problem(2, 2, (27, 33)), 1, 3, 2),
                                           (W.problem(3, 2, 18), 0, 3, 3), (W.problem(3, 1, 14), 1, 4, 1)])
def test_fe_structure(oracle, prob, form, M, q):
    m, N, S = oracle.dims(prob)
    sur = oracle.SurrogateFE(prob, form, M, q)
    R = sur.rows(np.arange(N))
    A = _dense(oracle, prob, R)
    sc = np.abs(A).max()
    assert np.abs(A - A.T).max() <= 1e-15 * sc
    if form == 0:
        assert np.abs(A.sum(axis=1)).max() < 1e-13 * sc
    E = oracle.exact_rows(prob, form, np.arange(N))
    upper = np.arange(S) > (S - 1) // 2
    # sample rows of every class: upper entries equal the exact ones
    assert np.abs(E[sur.sample_rows][:, upper] - R[sur.sample_rows][:, upper]).max() < 1e-13 * sc
    # corner rows: upper entries exact (bitwise, own quadrature)
    idx = oracle.multi_index(prob, np.arange(N))
    corner = np.all(oracle.row_class(prob, idx) >= 0, axis=1)
    assert corner.sum() == (4 * prob["p"]) ** prob["n"]
    assert np.array_equal(R[corner][:, upper], E[corner][:, upper])
    # a boundary-layer row off the sample lattice is interpolated, not exact
    bnd = ~corner & ~oracle.interior_mask(prob, idx)
    assert np.abs(R[bnd] - E[bnd]).max() > 1e-9 * sc
    # the quadrature rows are the sample rows of every class plus the corners
    quad = oracle.quadrature_rows_fe(prob, M)
    assert quad.sum() == len(np.unique(sur.sample_rows)) + corner.sum()
    assert quad.sum() < oracle.quadrature_rows(prob, M).sum()


@pytest.mark.parametrize("prob,form", [(W.problem(2, 3, 40, coef="sine3", camp=0.5), 0), (W.problem(3, 2, 20), 1)])
def test_fe_interior_rows_match_domain_surrogate(oracle, prob, form):
    """Rows whose whole stencil lies in the analysis domain use only the
    interior interpolant in both constructions."""
    m, N, S = oracle.dims(prob)
    idx = oracle.multi_index(prob, np.arange(N))
    p = prob["p"]
    deep = np.ones(N, dtype=bool)
    for d in range(prob["n"]):
        deep &= (idx[:, d] >= 3 * p) & (idx[:, d] <= m[d] - 3 * p - 1)
    rows = np.nonzero(deep)[0]
    a = oracle.SurrogateFE(prob, form, 4, 3).rows(rows)
    b = oracle.Surrogate(prob, form, 4, 3).rows(rows)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()


def test_fe_too_few_samples_rejected(oracle):
    with pytest.raises(ValueError):
        oracle.SurrogateFE(W.problem(2, 2, 14), 0, 4, 3)
