"""Pins for the oracle's solve and gradient:

* CG on the Dirichlet-reduced system (Sec. 6, eq. BlockSystem) against a
  direct sparse solve;
* L2 error of the discrete solution against the manufactured one decays like
  h^{p+1} (Thm. APrioriBounds) for the exact and surrogate matrices;
* the compliance gradient -u^T (dA~/dc) u against central differences of the
  quadratic form and of the solved compliance.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from paper_1904_06971_amd import workloads as W


def _system(oracle, prob, band):
    A = oracle.to_csr(prob, band)
    I = ~oracle.dirichlet_mask(prob)
    return A[I][:, I].tocsc(), I


def test_cg_matches_direct(oracle):
    prob = W.c1_poisson2d(32)
    _, N, _ = oracle.dims(prob)
    band = oracle.surrogate_rows(prob, 0, 4, 3)
    f = oracle.rhs(prob, 1, 2 * math.pi ** 2)
    u, it, res = oracle.cg(prob, band, f, rtol=1e-12)
    AII, I = _system(oracle, prob, band)
    ud = spla.spsolve(AII, f[I])
    assert res <= 1e-12 and it > 10
    assert np.abs(u[I] - ud).max() < 1e-9 * np.abs(ud).max()
    assert np.all(u[~I] == 0.0)


def test_l2_convergence(oracle):
    """u = sin(pi x) sin(pi y) on the sine-mapped square: rate ~ h^{p+1} = h^3."""
    errs = {"exact": [], "surrogate": []}
    for ne in (16, 32, 64):
        prob = W.c1_poisson2d(ne)
        _, N, _ = oracle.dims(prob)
        f = oracle.rhs(prob, 1, 2 * math.pi ** 2)
        for kind in errs:
            if kind == "exact":
                band = oracle.exact_rows(prob, 0, np.arange(N))
            else:
                band = oracle.surrogate_rows(prob, 0, 2, 3)
            AII, I = _system(oracle, prob, band)
            u = np.zeros(N)
            u[I] = spla.spsolve(AII, f[I])
            errs[kind].append(oracle.l2_error(prob, u, lambda x: np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])))
    for kind, e in errs.items():
        rate = math.log2(e[1] / e[2])
        assert 2.5 < rate < 3.6, (kind, e)
    assert errs["surrogate"][-1] < 1.5 * errs["exact"][-1]


def _small_adjoint_problem(cc):
    return W.problem(2, 3, 28, coef="exp_spline", cdeg=3, cn=(6, 6), cc=cc)


def test_quadratic_form_gradient_fd(oracle):
    """d/dc_k (u^T A~(c) u) at fixed u, central differences with step 1e-6,
    differences of the matrices formed entrywise before contracting."""
    rng = np.random.default_rng(3)
    cc = rng.normal(0, 0.5, 36)
    prob = _small_adjoint_problem(cc)
    _, N, _ = oracle.dims(prob)
    u = rng.standard_normal(N)
    ks = [0, 7, 14, 21, 35]
    g = -oracle.compliance_grad(prob, 4, 3, u, ks)      # = +u^T dA~ u
    for t, k in enumerate(ks):
        cp, cm = cc.copy(), cc.copy()
        cp[k] += 1e-6
        cm[k] -= 1e-6
        Ap = oracle.surrogate_rows(_small_adjoint_problem(cp), 0, 4, 3)
        Am = oracle.surrogate_rows(_small_adjoint_problem(cm), 0, 4, 3)
        fd = oracle.quadratic_form(prob, (Ap - Am) / 2e-6, u)
        assert abs(fd - g[t]) < 1e-6 * max(abs(g).max(), 1e-30)


def test_compliance_gradient_fd(oracle):
    rng = np.random.default_rng(4)
    cc = rng.normal(0, 0.5, 36)
    prob = _small_adjoint_problem(cc)
    _, N, _ = oracle.dims(prob)
    f = oracle.rhs(prob, 0, 1.0)

    def compliance(c):
        pr = _small_adjoint_problem(c)
        band = oracle.surrogate_rows(pr, 0, 4, 3)
        AII, I = _system(oracle, pr, band)
        u = np.zeros(N)
        u[I] = spla.spsolve(AII, f[I])
        return float(f @ u), u

    J0, u = compliance(cc)
    ks = [3, 10, 22, 30]
    g = oracle.compliance_grad(prob, 4, 3, u, ks)
    fds = []
    for k in ks:
        cp, cm = cc.copy(), cc.copy()
        cp[k] += 1e-6
        cm[k] -= 1e-6
        fds.append((compliance(cp)[0] - compliance(cm)[0]) / 2e-6)
    fds = np.array(fds)
    assert np.abs(fds - g).max() < 1e-6 * np.abs(g).max()
