"""Seeded synthetic workloads: problem descriptions and random inputs.

This module holds no arithmetic of the method.  It only states the problems
(degree, mesh, geometry map, coefficient, sampling) and draws the seeded random
inputs (coefficient nets, row samples, vectors) that the GPU path and the
CPU oracle both consume.

Problem description (a plain dict):
  n            dimension (2 or 3)
  p            spline degree (maximally smooth, open uniform knots)
  nelem        elements per direction (tuple of n ints)
  nq           Gauss points per direction per element (0 means p+1)
  geom, ga     geometry map: "identity", "sine" (amplitude ga), "poly2"
  coef         diffusion coefficient: "const" (c0), "sine3" (c0 + camp*...),
               "spline" (g), "exp_spline" (exp g); spline degree cdeg with cn
               functions per direction and control values cc [batch, prod cn]
  batch        number of independent problems (they differ only in cc)
"""
from __future__ import annotations

import numpy as np


def problem(n, p, nelem, geom="sine", ga=0.05, coef="const", c0=1.0, camp=0.0, cdeg=0, cn=None, cc=None,
            batch=1, nq=0):
    if isinstance(nelem, int):
        nelem = (nelem,) * n
    return {"n": n, "p": p, "nelem": tuple(int(e) for e in nelem), "nq": nq, "geom": geom, "ga": ga,
            "coef": coef, "c0": c0, "camp": camp, "cdeg": cdeg, "cn": tuple(cn) if cn else (0,) * n,
            "cc": None if cc is None else np.ascontiguousarray(np.asarray(cc, dtype=np.float64).reshape(batch, -1)),
            "batch": batch}


def coef_net(b, shape=(16, 16), sigma=0.5):
    """Control values of g for problem b of the differentiation workload: N(0, sigma^2)."""
    return np.random.default_rng(5000 + b).normal(0.0, sigma, shape)


def fd_indices(b, ncoef=256, count=16):
    """Coefficients checked by central differences for problem b."""
    return np.random.default_rng(5100 + b).choice(ncoef, count, replace=False)


def random_rows(N, count, seed):
    return np.random.default_rng(seed).integers(0, N, count)


def random_vector(N, seed, batch=1):
    return np.random.default_rng(seed).standard_normal((batch, N))


# The five workloads.  Sizes are the full ones; tests shrink nelem.
def c1_poisson2d(nelem=32):
    """2D Poisson, p=2, sine map a=0.05, kappa=1; surrogate M=4, q=3;
    f = 2 pi^2 sin(pi x) sin(pi y) (u = sin(pi x) sin(pi y))."""
    return problem(2, 2, nelem, geom="sine", ga=0.05)


def c2_poisson3d(nelem=64):
    """3D stiffness + mass, p=3, sine map, kappa=1; M in {4, 8, 16}, q=3."""
    return problem(3, 3, nelem, geom="sine", ga=0.05)


def c3_varcoef3d(nelem=128):
    """3D p=4 stiffness, kappa = 1 + 0.5 sin(2 pi x1) cos(2 pi x2) sin(2 pi x3); M=8, q=3."""
    return problem(3, 4, nelem, geom="sine", ga=0.05, coef="sine3", c0=1.0, camp=0.5)


def c4_precision3d(nelem=128):
    """3D p=3 Poisson, kappa=1, M=8, q=3; f = 3 pi^2 prod sin(pi x_d)."""
    return problem(3, 3, nelem, geom="sine", ga=0.05)


def c5_adjoint2d(nelem=256, batch=8, cn=16):
    """Batch of 2D p=3 Poisson problems, kappa = exp(g), g cubic B-spline on a
    cn x cn net, seeded N(0, 0.5^2); f = 1; M=8, q=3; loss = f^T u."""
    cc = np.stack([coef_net(b, (cn, cn)).ravel() for b in range(batch)])
    return problem(2, 3, nelem, geom="sine", ga=0.05, coef="exp_spline", cdeg=3, cn=(cn, cn), cc=cc, batch=batch)


# RHS sources: (kind, constant)
SRC_CONST, SRC_SINE = 0, 1
