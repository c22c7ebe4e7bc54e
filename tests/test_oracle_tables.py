"""Pins for the oracle's 1-D building blocks against independent libraries:
Gauss-Legendre (numpy), B-spline values/derivatives (scipy BSpline) and the
interpolating spline of the surrogate (scipy make_interp_spline and
RectBivariateSpline, the tool the paper's 2D implementation used, Sec. 6)."""
import numpy as np
import pytest
from scipy.interpolate import BSpline, RectBivariateSpline, make_interp_spline


@pytest.mark.parametrize("nq", range(1, 9))
def test_gauss_matches_numpy(oracle, nq):
    x, w = oracle.gauss(nq)
    xr, wr = np.polynomial.legendre.leggauss(nq)
    assert np.max(np.abs(x - xr)) < 1e-15
    assert np.max(np.abs(w - wr)) < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_basis_matches_scipy(oracle, p):
    ne = 7
    t = np.concatenate([np.zeros(p), np.linspace(0, 1, ne + 1), np.ones(p)])
    rng = np.random.default_rng(p)
    xs = rng.uniform(0, 1, 40)
    for k in range(ne + p):
        c = np.zeros(ne + p)
        c[k] = 1.0
        s = BSpline(t, c, p)
        ds = s.derivative()
        for x in xs:
            v, d = oracle.basis(ne, p, k, x)
            assert abs(v - s(x)) < 1e-14
            assert abs(d - ds(x)) < 1e-12


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("m,p,M", [(40, 2, 4), (67, 3, 8), (52, 3, 5), (35, 2, 3)])
def test_interpolant_matches_make_interp_spline(oracle, q, m, p, M):
    s = oracle.lattice(m, p, M)
    if len(s) < q + 1:
        pytest.skip("too few samples")
    rng = np.random.default_rng(m + q)
    v = rng.standard_normal(len(s))
    t = oracle.interp_knots(s, q)
    G = oracle.bspline_matrix(t, q, s)
    c = np.linalg.solve(G, v)
    x = np.arange(s[0], s[-1] + 1, dtype=float)
    mine = oracle.bspline_matrix(t, q, x) @ c
    ref = make_interp_spline(s.astype(float), v, k=q)
    assert np.max(np.abs(mine - ref(x))) < 1e-12 * max(1.0, np.max(np.abs(v)))
    # interpolation property at the samples
    assert np.max(np.abs(G @ c - v)) < 1e-12


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_tensor_interpolant_matches_rect_bivariate_spline(oracle, q):
    """The 2D implementation of the paper interpolates with RectBivariateSpline
    (s = 0); the oracle's tensor-product interpolant must coincide with it."""
    s1 = oracle.lattice(47, 2, 4)
    s2 = oracle.lattice(39, 2, 3)
    rng = np.random.default_rng(q)
    V = rng.standard_normal((len(s1), len(s2)))
    rbs = RectBivariateSpline(s1.astype(float), s2.astype(float), V, kx=q, ky=q, s=0)
    t1, t2 = oracle.interp_knots(s1, q), oracle.interp_knots(s2, q)
    C = np.linalg.solve(oracle.bspline_matrix(t1, q, s1), V)
    C = np.linalg.solve(oracle.bspline_matrix(t2, q, s2), C.T).T
    x1 = np.arange(s1[0], s1[-1] + 1, dtype=float)
    x2 = np.arange(s2[0], s2[-1] + 1, dtype=float)
    mine = oracle.bspline_matrix(t1, q, x1) @ C @ oracle.bspline_matrix(t2, q, x2).T
    assert np.max(np.abs(mine - rbs(x1, x2))) < 1e-12


def test_lattice_end_rule(oracle):
    # m = 131, p = 3: analysis indices 6..124, every 8th plus the last (Sec. 6)
    s = oracle.lattice(131, 3, 8)
    assert s[0] == 6 and s[-1] == 124 and len(s) == 16
    assert np.all(np.diff(s)[:-1] == 8) and np.diff(s)[-1] == 6
    s = oracle.lattice(67, 3, 4)       # 6..60, (60-6)/4 not integer
    assert len(s) == 15 and s[-1] == 60
    s = oracle.lattice(20, 2, 1)       # M = 1 samples every analysis index
    assert np.array_equal(s, np.arange(4, 16))


def _golden():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")) as fh:
        return json.load(fh)


def test_knot_vector_example(oracle):
    """The paper's p = 2 example: 21 functions, all but four translates of one."""
    g = _golden()["open_knot_example"]
    p, ne = g["p"], g["intervals"]
    assert ne + p == g["functions"]
    h = 1.0 / ne
    xs = np.random.default_rng(0).uniform(-1.5 * h, 1.5 * h, 50)
    ref_k = p                                  # first cardinal function (0-based)
    centre = lambda k: (k + 1 - (p + 1) / 2) * h  # x~ of function k (0-based k)
    translates = 0
    for k in range(ne + p):
        ok = True
        for x in xs:
            a, _ = oracle.basis(ne, p, k, centre(k) + x)
            b, _ = oracle.basis(ne, p, ref_k, centre(ref_k) + x)
            if abs(a - b) > 1e-14:
                ok = False
        translates += ok
    assert ne + p - translates == g["non_translates"]


def test_analysis_domain_formula(oracle):
    """Rows whose centre lies in the paper's analysis-domain interval are exactly
    the indices [2p, m-2p-1] the oracle treats as interior."""
    for m, p in _golden()["analysis_domain"]["cases"]:
        h = 1.0 / (m - p)
        lo = (3 * p + 1) / (2 * (m - p))
        ks = [k for k in range(p + 1, m - p + 1) if lo - 1e-12 <= (k - (p + 1) / 2) * h <= 1 - lo + 1e-12]
        ks0 = np.array(ks) - 1
        prob = {"n": 2, "p": p, "nelem": (m - p, m - p)}
        idx = np.stack([np.arange(m), np.full(m, m // 2)], axis=1)
        inner = np.nonzero(oracle.interior_mask(prob, idx))[0]
        assert np.array_equal(inner, ks0)
        assert ks0[0] == 2 * p and ks0[-1] == m - 2 * p - 1


def test_stencil_counts(oracle):
    for n, p, S, half in _golden()["stencil_counts"]["cases"]:
        prob = {"n": n, "p": p, "nelem": (10,) * n}
        off = oracle.stencil_offsets(prob)
        assert len(off) == S and len({tuple(o) for o in off}) == S
        colex = [sum(int(o[d]) * 100 ** d for d in range(n)) for o in off]
        assert sum(c >= 0 for c in colex) == half        # upper incl. diagonal
        assert np.all(np.diff(colex) > 0)                # slot order = colex order of delta
