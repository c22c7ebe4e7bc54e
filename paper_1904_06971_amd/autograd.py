"""torch.autograd wrappers over the C ABI (forward and backward both run in
the HIP kernels of libigs).

ApplyA:     y = A~(c) x, gradients w.r.t. x and the coefficient-spline
            control values c (igs_apply_vjp).
Compliance: J = f^T u with A~(c) u = f (homogeneous Dirichlet), gradient
            dJ/dc = -u^T (dA~/dc) u (igs_compliance_grad) and dJ/df = 2u.
M = 0 uses exact assembly, M >= 1 the surrogate with sampling M, degree q.
"""
from __future__ import annotations

import torch

from . import igs


def _with_coef(prob, cc):
    p = dict(prob)
    p["cc"] = cc.detach().to(torch.float64).contiguous()
    return p


def _assemble(p, M, q):
    if M and M >= 1:
        return igs.assemble_surrogate(p, igs.STIFFNESS, M, q)
    return igs.assemble_exact(p, igs.STIFFNESS)


class ApplyA(torch.autograd.Function):
    """y = A~(c) x for a batch of problems; x, y: [batch, N]; c: [batch, ncoef]."""

    @staticmethod
    def forward(ctx, x, cc, prob, M=8, q=3):
        p = _with_coef(prob, cc)
        band = _assemble(p, M, q)
        y = igs.apply(p, band, x.contiguous())
        ctx.save_for_backward(x)
        ctx.band, ctx.prob, ctx.M, ctx.q = band, p, M, q
        return y

    @staticmethod
    def backward(ctx, ybar):
        (x,) = ctx.saved_tensors
        want_x, want_c = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (want_x or want_c):
            return None, None, None, None, None
        xbar, cbar = igs.apply_vjp(ctx.prob, ctx.M or 0, ctx.q, ctx.band, x, ybar.contiguous(), want_x=want_x,
                                   want_c=want_c)
        return xbar, cbar, None, None, None


class Compliance(torch.autograd.Function):
    """J[b] = f[b]^T u[b], A~(c[b]) u[b] = f[b]; returns J [batch]."""

    @staticmethod
    def forward(ctx, cc, f, prob, M=8, q=3, rtol=1e-10, maxit=100000):
        p = _with_coef(prob, cc)
        band = _assemble(p, M, q)
        u, info = igs.solve_cg(p, band, f.contiguous(), rtol=rtol, maxit=maxit)
        ctx.save_for_backward(u)
        ctx.prob, ctx.M, ctx.q, ctx.info = p, M, q, info
        return (f * u).sum(dim=1)

    @staticmethod
    def backward(ctx, Jbar):
        (u,) = ctx.saved_tensors
        cbar = fbar = None
        if ctx.needs_input_grad[0]:
            cbar = igs.compliance_grad(ctx.prob, ctx.M or 0, ctx.q, u) * Jbar[:, None]
        if ctx.needs_input_grad[1]:
            fbar = 2.0 * u * Jbar[:, None]
        return cbar, fbar, None, None, None, None, None


def apply_a(x, cc, prob, M=8, q=3):
    return ApplyA.apply(x, cc, prob, M, q)


def compliance(cc, f, prob, M=8, q=3, rtol=1e-10):
    return Compliance.apply(cc, f, prob, M, q, rtol)
