"""Pins for the oracle's exact assembly (row-wise quadrature of the pulled-back
forms, Sec. 3.2 eq. BilinearFormPoissonTensor, and the mass form):

* closed-form cardinal stencils on the identity map from exact rational
  arithmetic (the autocorrelation of a degree-p cardinal B-spline is the
  degree-2p+1 cardinal B-spline, Sec. 2.2 on cardinal B-splines);
* symmetry, zero stiffness row sums (partition of unity, Sec. 5.3), mass row
  sums equal to the integral of B_i;
* linear functions in the kernel of the identity-map stiffness;
* agreement with a brute-force element-by-element assembler.
"""
from fractions import Fraction
from math import comb, factorial

import numpy as np
import pytest

from brute_force import assemble_dense
from paper_1904_06971_amd import workloads as W


def _card(r, x, deriv=0):
    """Cardinal B-spline of degree r (support [0, r+1]) or its deriv-th
    derivative at rational x, exactly."""
    tot = Fraction(0)
    for j in range(r + 2):
        y = Fraction(x) - j
        if y > 0:
            e = r - deriv
            coef = Fraction(factorial(r), factorial(e)) if deriv else 1
            tot += (-1) ** j * comb(r + 1, j) * coef * y ** e
    return tot / factorial(r)


def gram_tables(p):
    """G[k] = int b(x) b(x-k), S[k] = int b'(x) b'(x-k) for the unit-spacing
    cardinal B-spline b of degree p: G[k] = M_{2p+1}(p+1+k), S[k] = -M''_{2p+1}(p+1+k)."""
    G = [_card(2 * p + 1, p + 1 + k) for k in range(p + 1)]
    S = [-_card(2 * p + 1, p + 1 + k, deriv=2) for k in range(p + 1)]
    return G, S


def test_gram_tables_printed_values():
    G, S = gram_tables(2)
    assert G == [Fraction(11, 20), Fraction(13, 60), Fraction(1, 120)]
    assert S == [Fraction(1), Fraction(-1, 3), Fraction(-1, 6)]
    G, S = gram_tables(3)
    assert G == [Fraction(151, 315), Fraction(397, 1680), Fraction(1, 42), Fraction(1, 5040)]
    assert S == [Fraction(2, 3), Fraction(-1, 8), Fraction(-1, 5), Fraction(-1, 120)]


@pytest.mark.parametrize("n,p,ne", [(2, 1, 9), (2, 2, 10), (2, 3, 12), (2, 4, 14), (3, 2, 8), (3, 3, 10), (3, 4, 13)])
def test_identity_map_closed_form(oracle, n, p, ne):
    prob = W.problem(n, p, ne, geom="identity")
    m, N, S = oracle.dims(prob)
    G, Sg = gram_tables(p)
    h = 1.0 / ne
    centre = np.array([m[d] // 2 for d in range(n)])   # every function i+delta is cardinal
    assert np.all(centre - p >= p) and np.all(centre + p <= np.array(m) - p - 1)
    row = oracle.flat_index(prob, centre[None, :])
    A = oracle.exact_rows(prob, 0, row)[0]
    Mm = oracle.exact_rows(prob, 1, row)[0]
    off = oracle.stencil_offsets(prob)
    for s in range(S):
        d = np.abs(off[s])
        a_ref = sum(float(Sg[d[k]]) * np.prod([float(G[d[e]]) for e in range(n) if e != k]) for k in range(n))
        a_ref *= h ** (n - 2)
        m_ref = h ** n * np.prod([float(G[d[e]]) for e in range(n)])
        assert abs(A[s] - a_ref) < 1e-13 * max(1.0, abs(a_ref)) * 10
        assert abs(Mm[s] - m_ref) < 1e-15 + 1e-13 * abs(m_ref)
    # worked values
    if n == 2 and p == 2:
        assert abs(A[S // 2] - 1.1) < 1e-14 and abs(A[S // 2 + 1] - 1.0 / 30) < 1e-15
    if n == 3 and p == 3:
        assert abs(A[S // 2] - 45602 / 99225 * h) < 1e-14
        assert abs(Mm[S // 2] - 3442951 / 31255875 * h ** 3) < 1e-17


def _full(oracle, prob, form):
    _, N, _ = oracle.dims(prob)
    return oracle.to_csr(prob, oracle.exact_rows(prob, form, np.arange(N))).toarray()


@pytest.mark.parametrize("prob", [
    W.problem(2, 2, 12), W.problem(2, 3, 11, coef="sine3", camp=0.5),
    W.problem(3, 2, 6), W.problem(3, 3, 7, coef="sine3", camp=0.5),
    W.problem(2, 3, 10, coef="exp_spline", cdeg=3, cn=(6, 5), cc=np.random.default_rng(1).normal(0, .5, 30)),
])
def test_symmetry_and_row_sums(oracle, prob):
    A = _full(oracle, prob, 0)
    scale = np.abs(A).max()
    assert np.abs(A - A.T).max() < 1e-14 * scale * 10
    assert np.abs(A.sum(axis=1)).max() < 1e-13 * scale
    Mm = _full(oracle, prob, 1)
    assert np.abs(Mm - Mm.T).max() < 1e-15 * np.abs(Mm).max() * 10
    # total mass = |Omega| = 1: both sine maps send the unit cube onto itself
    assert abs(Mm.sum() - 1.0) < 2e-6


@pytest.mark.parametrize("n,p,ne", [(2, 2, 9), (2, 3, 8), (3, 2, 5)])
def test_mass_row_sums_identity(oracle, n, p, ne):
    """Identity map: sum_j M_ij = int B_i = prod_d (xi_{i_d+p+1} - xi_{i_d})/(p+1)."""
    prob = W.problem(n, p, ne, geom="identity")
    m, N, _ = oracle.dims(prob)
    Mm = _full(oracle, prob, 1)
    t = np.concatenate([np.zeros(p), np.linspace(0, 1, ne + 1), np.ones(p)])
    span = (t[p + 1:] - t[:-p - 1]) / (p + 1)
    idx = oracle.multi_index(prob, np.arange(N))
    ref = np.prod([span[idx[:, d]] for d in range(n)], axis=0)
    assert np.abs(Mm.sum(axis=1) - ref).max() < 1e-15
    assert abs(Mm.sum() - 1.0) < 1e-14


@pytest.mark.parametrize("n,p,ne", [(2, 2, 10), (2, 4, 9), (3, 3, 6)])
def test_linear_functions_in_kernel_identity(oracle, n, p, ne):
    """x_d = sum_i gamma_{i_d} B_i (Greville abscissae), so (A g)_i = int d_d B_i = 0
    for every row whose function vanishes on the boundary in direction d."""
    prob = W.problem(n, p, ne, geom="identity")
    m, N, _ = oracle.dims(prob)
    A = _full(oracle, prob, 0)
    t = np.concatenate([np.zeros(p), np.linspace(0, 1, ne + 1), np.ones(p)])
    grev = np.array([t[k + 1:k + p + 1].mean() for k in range(ne + p)])
    idx = oracle.multi_index(prob, np.arange(N))
    for d in range(n):
        g = grev[idx[:, d]]
        r = A @ g
        inner = (idx[:, d] > 0) & (idx[:, d] < m[d] - 1)
        assert np.abs(r[inner]).max() < 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("prob,form", [
    (W.problem(2, 1, 5), 0), (W.problem(2, 2, 4), 0), (W.problem(2, 3, 5, coef="sine3", camp=0.5), 0),
    (W.problem(2, 2, 5), 1), (W.problem(3, 2, 3), 0), (W.problem(3, 1, 3, coef="sine3", camp=0.5), 0),
    (W.problem(3, 2, 3), 1),
    (W.problem(2, 3, 5, coef="exp_spline", cdeg=3, cn=(5, 6), cc=np.random.default_rng(7).normal(0, .5, 30)), 0),
    (W.problem(2, 2, 4, coef="spline", cdeg=2, cn=(3, 3), cc=np.arange(9.0) + 1.0), 0),
    (W.problem(2, 2, 5, geom="poly2", ga=0.3), 0), (W.problem(2, 3, 4, geom="poly2", ga=0.3), 1),
    (W.problem(3, 2, 3, geom="poly2", ga=0.2), 0), (W.problem(3, 2, 3, geom="poly2", ga=0.2), 1),
    (W.problem(2, 2, 4, geom="poly2", ga=0.3, coef="sine3", camp=0.5), 0),
])
def test_rows_match_brute_force(oracle, prob, form):
    ref = assemble_dense(prob, form)
    A = _full(oracle, prob, form)
    assert np.abs(A - ref).max() < 1e-14 * max(1.0, np.abs(ref).max()) * 10


@pytest.mark.parametrize("prob", [W.problem(2, 2, 7, geom="poly2", ga=0.3), W.problem(2, 3, 6, geom="poly2", ga=0.3),
                                  W.problem(3, 3, 4, geom="poly2", ga=0.2)])
def test_poly2_total_mass(oracle, prob):
    """The Q_2 map fixes the boundary of the unit box (a factor xi_d (1 - xi_d)
    vanishes there) and folds nowhere at these amplitudes, so it maps the box
    onto itself and sum_ij M_ij = int det J = |Omega| = 1 (partition of unity,
    Sec. 2.2).  Every entry of J has degree <= 2 in each variable, so det J
    has degree <= 2n in each variable (4 in 2D, 6 in 3D), which (p+1)-point
    Gauss integrates exactly for p >= 2 (2D) and p >= 3 (3D): the sum is 1 to
    rounding, not just to quadrature accuracy."""
    Mm = _full(oracle, prob, 1)
    assert abs(Mm.sum() - 1.0) < 1e-13
    A = _full(oracle, prob, 0)
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
    assert np.abs(A.sum(axis=1)).max() < 1e-13 * np.abs(A).max()


def test_rhs_identity_constant(oracle):
    """f = 1 on the identity map: F(B_i) = int B_i."""
    p, ne = 3, 9
    prob = W.problem(2, p, ne, geom="identity")
    m, N, _ = oracle.dims(prob)
    f = oracle.rhs(prob, 0, 1.0)
    t = np.concatenate([np.zeros(p), np.linspace(0, 1, ne + 1), np.ones(p)])
    span = (t[p + 1:] - t[:-p - 1]) / (p + 1)
    idx = oracle.multi_index(prob, np.arange(N))
    assert np.abs(f - span[idx[:, 0]] * span[idx[:, 1]]).max() < 1e-15


def test_rhs_matches_mass_times_interpolant(oracle):
    """For f = const on any map, F(B_i) = c sum_j M_ij (partition of unity)."""
    prob = W.problem(2, 3, 9)
    m, N, _ = oracle.dims(prob)
    Mm = _full(oracle, prob, 1)
    f = oracle.rhs(prob, 0, 2.5)
    assert np.abs(f - 2.5 * Mm.sum(axis=1)).max() < 1e-15
