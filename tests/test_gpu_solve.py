"""GPU parity for the load vector, SpMV and CG against the oracle."""
import math

import numpy as np
import pytest

from gpu_util import rel_maxnorm
from paper_1904_06971_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def igs():
    import torch

    assert torch.cuda.is_available()
    from paper_1904_06971_amd import igs as m

    m.lib()
    return m


@pytest.mark.parametrize("prob,src,c", [(W.c1_poisson2d(), 1, 2 * math.pi ** 2), (W.problem(2, 3, 57), 0, 1.0),
                                        (W.problem(3, 3, (14, 11, 12)), 1, 3 * math.pi ** 2),
                                        (W.problem(3, 2, 13, geom="identity"), 0, 2.0), (W.problem(3, 4, 9), 1, 1.0)])
def test_rhs(igs, oracle, prob, src, c):
    f = igs.assemble_rhs(prob, src, c)
    ref = oracle.rhs(prob, src, c)
    assert rel_maxnorm(f[0].cpu().numpy(), ref) < 1e-13


# every degree in 2D and 3D; N odd or not a multiple of 4 in several cases (the
# kernels give each thread 2 (FP64) or 4 (FP32) consecutive rows)
@pytest.mark.parametrize("prob", [W.problem(2, 3, 41), W.problem(3, 3, (20, 19, 21)), W.problem(3, 2, 17),
                                  W.problem(2, 1, 50), W.problem(3, 4, 9), W.problem(3, 1, (30, 7, 9)),
                                  W.problem(2, 2, 37), W.problem(2, 4, (23, 30))])
@pytest.mark.parametrize("dirichlet", [False, True])
def test_apply(igs, oracle, prob, dirichlet):
    import torch

    _, N, _ = oracle.dims(prob)
    band = igs.assemble_exact(prob, 0)
    rows = igs.band_rows(band, prob)
    x = W.random_vector(N, 9)
    y = igs.apply(prob, band, torch.as_tensor(x, device="cuda"), dirichlet=dirichlet)
    ref = oracle.apply(prob, rows, x[0], dirichlet=dirichlet)
    assert rel_maxnorm(y[0].cpu().numpy(), ref) < 1e-13
    b32 = band.float()
    y32 = igs.apply(prob, b32, torch.as_tensor(x, device="cuda", dtype=torch.float32), dirichlet=dirichlet)
    assert rel_maxnorm(y32[0].double().cpu().numpy(), ref) < 1e-5


def test_apply_batched(igs, oracle):
    """A batch of problems with different coefficient fields: each problem's
    slice of the band applies to its own slice of x."""
    import torch

    prob = W.c5_adjoint2d(nelem=21, batch=3, cn=8)
    _, N, _ = oracle.dims(prob)
    band = igs.assemble_exact(prob, 0)
    x = np.concatenate([W.random_vector(N, 20 + b) for b in range(3)])
    y = igs.apply(prob, band, torch.as_tensor(x, device="cuda"))
    y32 = igs.apply(prob, band.float(), torch.as_tensor(x, device="cuda", dtype=torch.float32))
    for b in range(3):
        ref = oracle.apply(prob, igs.band_rows(band, prob, b), x[b])
        assert rel_maxnorm(y[b].cpu().numpy(), ref) < 1e-13
        assert rel_maxnorm(y32[b].double().cpu().numpy(), ref) < 1e-5


def test_cg_c1(igs, oracle):
    prob = W.c1_poisson2d()
    band = igs.assemble_surrogate(prob, 0, M=4, q=3)
    f = igs.assemble_rhs(prob, 1, 2 * math.pi ** 2)
    u, info = igs.solve_cg(prob, band, f, rtol=1e-10)
    assert info["status"] == 0 and info["relres"] <= 1e-10
    rows = igs.band_rows(band, prob)
    uref, it, _ = oracle.cg(prob, rows, f[0].cpu().numpy(), rtol=1e-13)
    assert rel_maxnorm(u[0].cpu().numpy(), uref) < 1e-8
    # L2 error against the manufactured solution (loose, depends on h)
    err = oracle.l2_error(prob, u[0].cpu().numpy(), lambda x: np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]))
    assert err < 2e-4


def test_cg_mixed_precision(igs, oracle):
    import torch

    prob = W.problem(3, 3, 20)
    b64 = igs.assemble_surrogate(prob, 0, M=4, q=3)
    b32 = igs.assemble_surrogate(prob, 0, M=4, q=3, dtype=torch.float32)
    f = igs.assemble_rhs(prob, 1, 3 * math.pi ** 2)
    u64, i64 = igs.solve_cg(prob, b64, f, rtol=1e-10)
    umx, imx = igs.solve_cg(prob, b64, f, band32=b32, rtol=1e-10)
    assert i64["relres"] <= 1e-10 and imx["relres"] <= 1e-10
    assert imx["outer_iterations"] >= 2
    # both solve the FP64 surrogate system to 1e-10
    rows = igs.band_rows(b64, prob)
    uref, _, _ = oracle.cg(prob, rows, f[0].cpu().numpy(), rtol=1e-13)
    assert rel_maxnorm(u64[0].cpu().numpy(), uref) < 1e-7
    assert rel_maxnorm(umx[0].cpu().numpy(), uref) < 1e-7


def test_cg_batched(igs, oracle):
    prob = W.c5_adjoint2d(nelem=40, batch=3, cn=8)
    band = igs.assemble_surrogate(prob, 0, M=4, q=3)
    f = igs.assemble_rhs(prob, 0, 1.0)
    u, info = igs.solve_cg(prob, band, f, rtol=1e-11)
    assert info["relres"] <= 1e-11
    for b in range(3):
        rows = igs.band_rows(band, prob, b)
        uref, _, _ = oracle.cg(prob, rows, f[b].cpu().numpy(), rtol=1e-13)
        assert rel_maxnorm(u[b].cpu().numpy(), uref) < 1e-8


def test_cg_mixed_batched(igs, oracle):
    """FP32 CG with FP64 residual replacement on a batch: every problem reaches
    the FP64 tolerance and the FP64 solution."""
    import torch

    prob = W.c5_adjoint2d(nelem=40, batch=3, cn=8)
    band = igs.assemble_surrogate(prob, 0, M=4, q=3)
    b32 = igs.assemble_surrogate(prob, 0, M=4, q=3, dtype=torch.float32)
    f = igs.assemble_rhs(prob, 0, 1.0)
    u, info = igs.solve_cg(prob, band, f, band32=b32, rtol=1e-11)
    assert info["status"] == 0 and info["relres"] <= 1e-11
    for b in range(3):
        rows = igs.band_rows(band, prob, b)
        uref, _, _ = oracle.cg(prob, rows, f[b].cpu().numpy(), rtol=1e-13)
        assert rel_maxnorm(u[b].cpu().numpy(), uref) < 1e-8


@pytest.mark.parametrize("mixed", [False, True])
def test_cg_batch_with_finished_problem(igs, oracle, mixed):
    """A batch whose middle problem has f = 0 (finished before the first
    step): its u stays exactly 0 while the fused product and update kernels
    (FP64) or the launch slots (FP32 with FP64 residual replacement) skip it,
    and the other problems reach the FP64 solution."""
    import torch

    prob = W.c5_adjoint2d(nelem=40, batch=3, cn=8)
    band = igs.assemble_surrogate(prob, 0, M=4, q=3)
    b32 = igs.assemble_surrogate(prob, 0, M=4, q=3, dtype=torch.float32) if mixed else None
    f = igs.assemble_rhs(prob, 0, 1.0)
    f[1] = 0.0
    u, info = igs.solve_cg(prob, band, f, band32=b32, rtol=1e-11)
    assert info["status"] == 0 and info["relres"] <= 1e-11
    assert float(u[1].abs().max()) == 0.0
    for b in (0, 2):
        rows = igs.band_rows(band, prob, b)
        uref, _, _ = oracle.cg(prob, rows, f[b].cpu().numpy(), rtol=1e-13)
        assert rel_maxnorm(u[b].cpu().numpy(), uref) < 1e-8


def test_cg_mixed_not_converged(igs):
    import torch

    prob = W.c1_poisson2d()
    band = igs.assemble_exact(prob, 0)
    f = igs.assemble_rhs(prob, 0, 1.0)
    u, info = igs.solve_cg(prob, band, f, band32=band.float(), rtol=1e-10, maxit=3, check=False)
    assert info["status"] == 1 and info["iterations"] <= 3 and info["relres"] > 1e-10


def test_cg_not_converged(igs):
    prob = W.c1_poisson2d()
    band = igs.assemble_exact(prob, 0)
    f = igs.assemble_rhs(prob, 0, 1.0)
    u, info = igs.solve_cg(prob, band, f, rtol=1e-10, maxit=3, check=False)
    assert info["status"] == 1 and info["iterations"] <= 3 + 32


@pytest.mark.parametrize("case", ["fused", "large", "fp32"])
def test_cg_breakdown(igs, case):
    """IGS_BREAKDOWN: CG on a negative definite matrix (the negated mass band)
    meets p^T A p < 0 in its first iteration.  The small 2D problem takes the
    fused scalar kernels, the 3D one (more than 1024 partial sums per problem)
    the separate reduction kernels, the FP32 band the residual-replacement
    loop."""
    import torch

    prob = W.c1_poisson2d() if case != "large" else W.problem(3, 2, 70)
    band = -igs.assemble_exact(prob, 1)
    f = igs.assemble_rhs(prob, 0, 1.0)
    b32 = band.to(torch.float32) if case == "fp32" else None
    u, info = igs.solve_cg(prob, band, f, band32=b32, rtol=1e-10, maxit=1000, check=False)
    assert info["status"] == 2, info
    assert bool(torch.isfinite(u).all())
    with pytest.raises(igs.IGSError, match="BREAKDOWN"):
        igs.solve_cg(prob, band, f, band32=b32, rtol=1e-10, maxit=1000)


def test_cg_large(igs, oracle):
    """A problem with more than 1024 SpMV workgroups per problem (373,248 dofs),
    where the CG scalars are reduced by separate kernels: the returned solution
    meets the tolerance on the FP64 residual recomputed by igs_apply, and agrees
    with the FP32 solve with FP64 residual replacement (other kernels)."""
    import torch

    prob = W.problem(3, 2, 70)
    band = igs.assemble_surrogate(prob, 0, M=8, q=3)
    f = igs.assemble_rhs(prob, 1, 3 * math.pi ** 2)
    u, info = igs.solve_cg(prob, band, f, rtol=1e-10)
    assert info["status"] == 0 and info["relres"] <= 1e-10
    # f restricted to the free dofs (no index on the boundary), minus A_II u_I
    m, N, _ = oracle.dims(prob)
    idx = oracle.multi_index(prob, np.arange(N))
    free = torch.as_tensor(np.all((idx > 0) & (idx < np.asarray(m) - 1), axis=1), device="cuda")[None, :]
    r = torch.where(free, f - igs.apply(prob, band, u, dirichlet=True), torch.zeros_like(f))
    fn = torch.where(free, f, torch.zeros_like(f)).norm()
    assert float(r.norm() / fn) <= 1e-10
    umx, imx = igs.solve_cg(prob, band, f, band32=band.float(), rtol=1e-10)
    assert imx["status"] == 0
    assert float((umx - u).abs().max() / u.abs().max()) < 1e-7
