"""Brute-force dense assembly on tiny meshes: a textbook element loop with
local (p+1)^n x (p+1)^n matrices scattered into a dense N x N matrix.

Independent of the oracle's row assembler: B-splines come from
scipy.interpolate.BSpline, Gauss points from numpy's leggauss, the geometry
maps and coefficients are transcribed here from the workload statements.
"""
import math

import numpy as np
from scipy.interpolate import BSpline


def _knots(ne, p):
    return np.concatenate([np.zeros(p), np.linspace(0.0, 1.0, ne + 1), np.ones(p)])


def _basis_1d(ne, p, x):
    """values and derivatives of all m = ne+p functions at points x -> [len(x), m]"""
    t = _knots(ne, p)
    m = ne + p
    V = np.zeros((len(x), m))
    D = np.zeros((len(x), m))
    for k in range(m):
        c = np.zeros(m)
        c[k] = 1.0
        s = BSpline(t, c, p, extrapolate=False)
        V[:, k] = np.nan_to_num(s(x))
        D[:, k] = np.nan_to_num(s.derivative()(x))
    return V, D


def sine_map(xi, a):
    """F and J = dF/dxi of the sine maps of the workloads (2D and 3D)."""
    n = len(xi)
    pi = math.pi
    s1 = [math.sin(pi * v) for v in xi]
    c1 = [pi * math.cos(pi * v) for v in xi]
    s2 = [math.sin(2 * pi * v) for v in xi]
    c2 = [2 * pi * math.cos(2 * pi * v) for v in xi]
    J = np.eye(n)
    F = np.array(xi, dtype=float)
    if n == 2:
        F[0] += a * s1[0] * s2[1]
        F[1] += a * s2[0] * s1[1]
        J[0] += a * np.array([c1[0] * s2[1], s1[0] * c2[1]])
        J[1] += a * np.array([c2[0] * s1[1], s2[0] * c1[1]])
    else:
        F[0] += a * s1[0] * s2[1] * s1[2]
        F[1] += a * s2[0] * s1[1] * s1[2]
        F[2] += a * s1[0] * s1[1] * s2[2]
        J[0] += a * np.array([c1[0] * s2[1] * s1[2], s1[0] * c2[1] * s1[2], s1[0] * s2[1] * c1[2]])
        J[1] += a * np.array([c2[0] * s1[1] * s1[2], s2[0] * c1[1] * s1[2], s2[0] * s1[1] * c1[2]])
        J[2] += a * np.array([c1[0] * s1[1] * s2[2], s1[0] * c1[1] * s2[2], s1[0] * s1[1] * c2[2]])
    return F, J


def poly2_map(xi, a):
    """F and J of the Q_2 map F_r = xi_r + a (r+1) prod_d xi_d (1 - xi_d)
    (r 0-based).  J is not transcribed: it comes from complex-step
    differentiation of F, dF/dxi_c = Im F(xi + i t e_c) / t, which is exact
    to rounding for a polynomial map and shares no formula with the oracle's
    hand-written Jacobian."""
    n = len(xi)

    def F(z):
        prod = 1.0 + 0.0j
        for d in range(n):
            prod *= z[d] * (1.0 - z[d])
        return np.array([z[r] + a * (r + 1) * prod for r in range(n)])

    x0 = np.array(xi, dtype=complex)
    t = 1e-30
    J = np.zeros((n, n))
    for c in range(n):
        z = x0.copy()
        z[c] += 1j * t
        J[:, c] = F(z).imag / t
    return F(x0).real, J


def coefficient(prob, xi, F):
    kind = prob["coef"]
    if kind == "const":
        return prob["c0"]
    if kind == "sine3":
        v = math.sin(2 * math.pi * F[0]) * math.cos(2 * math.pi * F[1])
        if len(F) == 3:
            v *= math.sin(2 * math.pi * F[2])
        return prob["c0"] + prob["camp"] * v
    deg, cn = prob["cdeg"], prob["cn"]
    n = len(xi)
    vals = []
    for d in range(n):
        V, _ = _basis_1d(cn[d] - deg, deg, np.array([xi[d]]))
        vals.append(V[0])
    cc = np.asarray(prob["cc"]).reshape(prob["batch"], *cn[::-1])[0]
    if n == 2:
        g = vals[1] @ cc @ vals[0]
    else:
        g = np.einsum("kji,k,j,i->", cc, vals[2], vals[1], vals[0])
    return g if kind == "spline" else math.exp(g)


def assemble_dense(prob, form):
    """Dense stiffness (form 0) or mass (form 1) matrix, colex dof ordering."""
    n, p = prob["n"], prob["p"]
    ne = prob["nelem"]
    m = [ne[d] + p for d in range(n)]
    N = int(np.prod(m))
    nq = prob.get("nq", 0) or p + 1
    gx, gw = np.polynomial.legendre.leggauss(nq)
    A = np.zeros((N, N))
    for e in np.ndindex(*[ne[d] for d in range(n)][::-1]):
        e = e[::-1]                                     # e[0] = direction 1
        pts, wts, V, D = [], [], [], []
        for d in range(n):
            h = 1.0 / ne[d]
            x = e[d] * h + 0.5 * h * (gx + 1.0)
            vv, dd = _basis_1d(ne[d], p, x)
            pts.append(x)
            wts.append(0.5 * h * gw)
            V.append(vv[:, e[d]:e[d] + p + 1])
            D.append(dd[:, e[d]:e[d] + p + 1])
        loc = [list(range(e[d], e[d] + p + 1)) for d in range(n)]
        glob = []
        for a in np.ndindex(*[p + 1] * n):
            a = a[::-1]
            gi, stride = 0, 1
            for d in range(n):
                gi += loc[d][a[d]] * stride
                stride *= m[d]
            glob.append((a, gi))
        nl = len(glob)
        Ke = np.zeros((nl, nl))
        for k in np.ndindex(*[nq] * n):
            xi = [pts[d][k[d]] for d in range(n)]
            w = np.prod([wts[d][k[d]] for d in range(n)])
            if prob["geom"] == "identity":
                F, J = np.array(xi), np.eye(n)
            elif prob["geom"] == "poly2":
                F, J = poly2_map(xi, prob["ga"])
            else:
                F, J = sine_map(xi, prob["ga"])
            det = np.linalg.det(J)
            Jinv = np.linalg.inv(J)
            grads = np.zeros((nl, n))
            vals = np.zeros(nl)
            for t, (a, _) in enumerate(glob):
                vals[t] = np.prod([V[d][k[d], a[d]] for d in range(n)])
                for c in range(n):
                    grads[t, c] = np.prod([(D if d == c else V)[d][k[d], a[d]] for d in range(n)])
            if form == 0:
                K = coefficient(prob, xi, F) * abs(det) * Jinv @ Jinv.T
                Ke += w * grads @ K @ grads.T
            else:
                Ke += w * abs(det) * np.outer(vals, vals)
        ids = [g for _, g in glob]
        A[np.ix_(ids, ids)] += Ke
    return A
