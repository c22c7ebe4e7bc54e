"""C-ABI checks that need no GPU: the library loads, exports every function
include/igs.h declares, and its host-only queries (band layout, sample
lattice, row classes, argument validation) agree with the oracle's own
planning.  No compute entry point is called with valid arguments here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1904_06971_amd import igs
from paper_1904_06971_amd import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "igs.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:igs_status|int32_t|const char\*)\s+(igs_\w+)\(", txt, flags=re.M)))


def test_exports_every_declared_symbol():
    L = igs.lib()
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(igs.EXPORTS)
    assert "gfx950" in igs.version()


def test_status_strings():
    for st in igs.STATUS:
        assert igs.lib().igs_status_string(st).decode() not in ("", "unknown status")


@pytest.mark.parametrize("prob", [W.c1_poisson2d(), W.c2_poisson3d(), W.c3_varcoef3d(), W.c4_precision3d(),
                                  W.c5_adjoint2d()])
def test_layout_matches_oracle(oracle, prob):
    lay = igs.layout(prob)
    m, N, S = oracle.dims(prob)
    assert tuple(lay.m[:prob["n"]]) == m and lay.N == N and lay.slots == S
    assert lay.ld % 64 == 0 and N < lay.ld <= N + 64
    assert lay.band_elems == prob["batch"] * S * lay.ld
    assert lay.upper == (S - 1) // 2


@pytest.mark.parametrize("prob,M,q", [(W.c1_poisson2d(), 4, 3), (W.c2_poisson3d(), 4, 3), (W.c2_poisson3d(), 8, 3),
                                      (W.c2_poisson3d(), 16, 3), (W.c3_varcoef3d(), 8, 3), (W.c4_precision3d(), 8, 3),
                                      (W.c5_adjoint2d(), 8, 3), (W.problem(2, 2, 40), 1, 5)])
def test_surrogate_layout_matches_oracle(oracle, prob, M, q):
    info, idx = igs.surrogate_layout(prob, M, q)
    m, N, _ = oracle.dims(prob)
    for d in range(prob["n"]):
        assert np.array_equal(idx[d], oracle.lattice(m[d], prob["p"], M))
    quad = oracle.quadrature_rows(prob, M) if N < 400000 else None
    if quad is not None:
        assert info.quadrature_rows == quad.sum()
    inner = np.prod([m[d] - 4 * prob["p"] for d in range(prob["n"])])
    assert info.boundary_rows == N - inner
    assert info.sample_rows == np.prod([len(i) for i in idx])


@pytest.mark.parametrize("prob,M,q", [(W.problem(2, 2, 32), 4, 3), (W.problem(2, 3, (70, 41)), 5, 3),
                                      (W.problem(3, 2, (22, 19, 25)), 4, 2), (W.c4_precision3d(), 8, 3)])
def test_surrogate_fe_layout_matches_oracle(oracle, prob, M, q):
    """Face/edge sampling: per-direction sample sets (4p layers + lattice), the
    class count (4p+1)^n - (4p)^n, and the quadrature row count against the
    oracle's own class enumeration."""
    info = igs.surrogate_fe_layout(prob, M, q)
    m, N, _ = oracle.dims(prob)
    p, n = prob["p"], prob["n"]
    for d in range(n):
        assert info.samples[d] == len(oracle.lattice(m[d], p, M)) + 4 * p
    assert info.classes == len(oracle.layer_classes(prob))
    assert info.corner_rows == (4 * p) ** n
    if N < 400000:
        assert info.quadrature_rows == int(oracle.quadrature_rows_fe(prob, M).sum())
    else:
        assert info.quadrature_rows == np.prod([info.samples[d] for d in range(n)])


@pytest.mark.parametrize("prob,M,q", [(W.problem(2, 2, 30), 4, 3), (W.problem(3, 3, 40), 6, 3),
                                      (W.c4_precision3d(), 8, 3), (W.problem(3, 4, 30), 5, 2)])
def test_surrogate_pd_layout_matches_oracle(oracle, prob, M, q):
    """Per-delta sampling: per-direction common sample sets, the largest
    per-offset sample count, non-cardinal and quadrature row counts against the
    oracle's own definitions."""
    info = igs.surrogate_pd_layout(prob, M, q)
    m, N, _ = oracle.dims(prob)
    p, n = prob["p"], prob["n"]
    for d in range(n):
        assert info.samples[d] == len(oracle.sample_union_pd(m[d], p, M))
        assert info.max_samples[d] == max(len(oracle.lattice_pd(m[d], p, M, dd)) for dd in range(-p, p + 1))
    assert info.noncardinal_rows == N - np.prod([m[d] - 2 * p for d in range(n)])
    if N < 400000:
        assert info.quadrature_rows == int(oracle.quadrature_rows_pd(prob, M).sum())
    else:
        assert info.quadrature_rows == info.noncardinal_rows + np.prod([info.samples[d] for d in range(n)])


def test_published_sizes():
    """Sizes quoted for the workloads: 34^2 = 1156 dofs; 67^3 = 300,763 dofs with
    343-entry stencils; 132^3 with 729-entry stencils; 131^3 ~ 2.25M dofs; 259^2."""
    assert igs.layout(W.c1_poisson2d()).N == 1156
    lay = igs.layout(W.c2_poisson3d())
    assert lay.N == 300763 and lay.slots == 343 and lay.N * lay.slots == 103161709
    lay = igs.layout(W.c3_varcoef3d())
    assert lay.N == 2299968 and lay.slots == 729 and lay.N * lay.slots == 1676676672
    lay = igs.layout(W.c4_precision3d())
    assert lay.N == 2248091 and lay.N * lay.slots == 771095213
    assert igs.layout(W.c5_adjoint2d()).N == 67081


def _status(fn, *args):
    return fn(*args)


@pytest.mark.parametrize("mutate,expected", [
    (lambda pb: setattr(pb, "n", 4), igs.IGS_OK - 1),
    (lambda pb: setattr(pb, "p", 0), -1),
    (lambda pb: setattr(pb, "p", 5), -2),
    (lambda pb: setattr(pb, "batch", 0), -1),
    (lambda pb: setattr(pb, "nquad", 7), -2),
    (lambda pb: setattr(pb, "nquad", -1), -1),
    (lambda pb: pb.nelem.__setitem__(1, 0), -1),
    (lambda pb: setattr(pb.geom, "kind", 9), -1),
    (lambda pb: setattr(pb.coef, "kind", 9), -1),
])
def test_validation_errors(mutate, expected):
    pb = igs.make_problem(W.c1_poisson2d())
    mutate(pb)
    L = igs.lib()
    assert L.igs_validate(ctypes.byref(pb), 0, 0) == expected
    # every compute entry point rejects the same problem before touching the GPU
    dummy = ctypes.c_void_p(16)
    assert L.igs_assemble_exact(ctypes.byref(pb), 0, 0, dummy, None) == expected
    assert L.igs_assemble_surrogate(ctypes.byref(pb), 0, 4, 3, 0, dummy, None) == expected
    assert L.igs_assemble_noalloc(ctypes.byref(pb), 0, 0, 0, 0, dummy, None) == expected
    assert L.igs_assemble_noalloc(ctypes.byref(pb), 0, 4, 3, 0, dummy, None) == expected
    assert L.igs_assemble_surrogate_fe(ctypes.byref(pb), 0, 4, 3, 0, dummy, None) == expected
    assert L.igs_plan_create_fe(ctypes.byref(pb), 0, 4, 3, 0, None, ctypes.byref(ctypes.c_void_p())) == expected
    assert L.igs_assemble_rhs(ctypes.byref(pb), 0, 1.0, dummy, None) == expected
    assert L.igs_assemble_async(ctypes.byref(pb), 0, 0, 0, 0, dummy, None) == expected
    assert L.igs_assemble_async(ctypes.byref(pb), 0, 4, 3, 0, dummy, None) == expected
    assert L.igs_assemble_rhs_async(ctypes.byref(pb), 0, 1.0, dummy, None) == expected
    assert L.igs_apply(ctypes.byref(pb), 0, dummy, dummy, dummy, 0, None) == expected
    h = ctypes.c_void_p(16)
    assert L.igs_plan_create(ctypes.byref(pb), 0, 4, 3, 0, None, ctypes.byref(h)) == expected
    assert h.value is None  # *out cleared on error


def test_sampling_errors():
    L = igs.lib()
    pb = igs.make_problem(W.problem(2, 2, 14))          # 8 analysis rows per direction
    assert L.igs_validate(ctypes.byref(pb), 4, 3) == -4  # 3 samples < q + 1
    assert L.igs_validate(ctypes.byref(pb), 2, 3) == 0
    assert L.igs_validate(ctypes.byref(pb), 0, 3) == -1  # M < 1
    assert L.igs_validate(ctypes.byref(pb), 2, 0) == -1
    assert L.igs_validate(ctypes.byref(pb), 2, 6) == -2  # q > 5
    pb = igs.make_problem(W.problem(2, 3, 5))           # m - 4p < 1: no analysis rows
    assert L.igs_validate(ctypes.byref(pb), 1, 1) == -4
    dummy = ctypes.c_void_p(16)
    assert L.igs_assemble_surrogate(ctypes.byref(pb), 0, 1, 1, 0, dummy, None) == -4
    assert L.igs_assemble_surrogate_fe(ctypes.byref(pb), 0, 1, 1, 0, dummy, None) == -4
    h = ctypes.c_void_p()
    assert L.igs_plan_create(ctypes.byref(pb), 0, 1, 1, 0, None, ctypes.byref(h)) == -4
    pb = igs.make_problem(W.problem(2, 2, 14))
    assert L.igs_plan_create(ctypes.byref(pb), 0, 4, 3, 0, None, ctypes.byref(h)) == -4
    assert L.igs_plan_create(ctypes.byref(pb), 0, 2, 6, 0, None, ctypes.byref(h)) == -2


@pytest.mark.parametrize("p,q", [(2, 5), (1, 3), (3, 5), (2, 4), (4, 3)])
@pytest.mark.parametrize("beta", [0.0, 0.25, 0.5, 1.0])
def test_sampling_length_matches_oracle(oracle, p, q, beta):
    """igs_sampling_length against the oracle's exact rational evaluation, on
    a grid of meshes and calibrations that includes exact-integer cases
    (nelem = 4096 with beta = 1/2, p = 2, q = 5: c * 32)."""
    for nelem in (1, 7, 16, 64, 100, 128, 333, 1000, 1024, 1448, 4096):
        for c in (0.0, 0.25, 0.5, 0.75, 1.0, 2.0, 3.0, 4.0):
            assert igs.sampling_length(nelem, p, q, c, beta) == oracle.sampling_length(nelem, p, q, c, beta), \
                (nelem, c)


def test_sampling_length_rejects():
    L = igs.lib()
    for args in [(0, 2, 5, 1.0, 0.5), (10, 0, 5, 1.0, 0.5), (10, 2, 0, 1.0, 0.5), (10, 2, 5, -1.0, 0.5),
                 (10, 2, 5, 1.0, -0.5), (10, 2, 5, float("nan"), 0.5), (10, 2, 5, 1.0, float("inf"))]:
        assert L.igs_sampling_length(*args) == -1, args


def test_knot_validation():
    prob = W.problem(2, 2, 6)
    good = np.concatenate([np.zeros(2), np.linspace(0, 1, 7), np.ones(2)])
    bad = good.copy()
    bad[4] += 0.01
    L = igs.lib()
    assert L.igs_validate(ctypes.byref(igs.make_problem(prob, knots=[good, good])), 0, 0) == 0
    assert L.igs_validate(ctypes.byref(igs.make_problem(prob, knots=[good, bad])), 0, 0) == -3


def test_null_and_enum_arguments():
    L = igs.lib()
    pb = igs.make_problem(W.c1_poisson2d())
    dummy = ctypes.c_void_p(16)
    assert L.igs_assemble_exact(None, 0, 0, dummy, None) == -1
    assert L.igs_assemble_exact(ctypes.byref(pb), 0, 0, None, None) == -1
    assert L.igs_assemble_exact(ctypes.byref(pb), 2, 0, dummy, None) == -1
    assert L.igs_assemble_exact(ctypes.byref(pb), 0, 5, dummy, None) == -1
    assert L.igs_assemble_noalloc(None, 0, 0, 0, 0, dummy, None) == -1
    assert L.igs_assemble_noalloc(ctypes.byref(pb), 0, 0, 0, 0, None, None) == -1
    assert L.igs_assemble_noalloc(ctypes.byref(pb), 2, 0, 0, 0, dummy, None) == -1
    assert L.igs_assemble_noalloc(ctypes.byref(pb), 0, 0, 0, 5, dummy, None) == -1
    assert L.igs_assemble_noalloc(ctypes.byref(pb), 0, -1, 3, 0, dummy, None) == -1
    assert L.igs_assemble_noalloc(ctypes.byref(pb), 0, 4, 6, 0, dummy, None) == -2
    assert L.igs_assemble_rhs(ctypes.byref(pb), 3, 1.0, dummy, None) == -1
    assert L.igs_assemble_async(None, 0, 0, 0, 0, dummy, None) == -1
    assert L.igs_assemble_async(ctypes.byref(pb), 0, 0, 0, 0, None, None) == -1
    assert L.igs_assemble_async(ctypes.byref(pb), 2, 0, 0, 0, dummy, None) == -1
    assert L.igs_assemble_async(ctypes.byref(pb), 0, 0, 0, 5, dummy, None) == -1
    assert L.igs_assemble_async(ctypes.byref(pb), 0, -1, 3, 0, dummy, None) == -1
    assert L.igs_assemble_async(ctypes.byref(pb), 0, 4, 6, 0, dummy, None) == -2
    assert L.igs_assemble_rhs_async(ctypes.byref(pb), 3, 1.0, dummy, None) == -1
    assert L.igs_assemble_rhs_async(ctypes.byref(pb), 0, 1.0, None, None) == -1
    info = igs.CgInfo()
    assert L.igs_solve_cg(ctypes.byref(pb), dummy, None, dummy, dummy, 0.0, 10, ctypes.byref(info), None) == -1
    h = ctypes.c_void_p()
    assert L.igs_plan_create(None, 0, 4, 3, 0, None, ctypes.byref(h)) == -1
    assert L.igs_plan_create(ctypes.byref(pb), 0, 4, 3, 0, None, None) == -1
    assert L.igs_plan_create(ctypes.byref(pb), 3, 4, 3, 0, None, ctypes.byref(h)) == -1
    assert L.igs_plan_create(ctypes.byref(pb), 0, 4, 3, 7, None, ctypes.byref(h)) == -1
    assert L.igs_plan_create(ctypes.byref(pb), 0, -1, 3, 0, None, ctypes.byref(h)) == -1
    assert L.igs_plan_execute(None, None, dummy, None) == -1
    assert L.igs_plan_destroy(None) == 0
    assert L.igs_solve_cg(ctypes.byref(pb), dummy, None, dummy, dummy, 1e-8, 0, ctypes.byref(info), None) == -1
    assert L.igs_solve_cg(ctypes.byref(pb), None, None, dummy, dummy, 1e-8, 10, ctypes.byref(info), None) == -1
    sp = igs.make_problem(W.c5_adjoint2d())
    sp.coef.coef = None                                # spline coefficient without control values
    assert L.igs_validate(ctypes.byref(sp), 0, 0) == -1


def test_band_alignment_rejected():
    """The SpMV reads a row pair of a slot with one load: a band pointer off
    the 16-byte (FP64) or 8-byte (FP32) grid is an argument error, reported
    before any GPU work."""
    L = igs.lib()
    pb = igs.make_problem(W.c1_poisson2d())
    ok, off8, off4 = ctypes.c_void_p(256), ctypes.c_void_p(264), ctypes.c_void_p(260)
    assert L.igs_apply(ctypes.byref(pb), igs.F64, off8, ok, ok, 0, None) == -1
    assert L.igs_apply(ctypes.byref(pb), igs.F32, off4, ok, ok, 0, None) == -1
    info = igs.CgInfo()
    assert L.igs_solve_cg(ctypes.byref(pb), off8, None, ok, ok, 1e-8, 10, ctypes.byref(info), None) == -1
    assert L.igs_solve_cg(ctypes.byref(pb), ok, off4, ok, ok, 1e-8, 10, ctypes.byref(info), None) == -1


def test_library_resolves_all_symbols():
    """Every symbol the library needs is defined (immediate binding)."""
    ctypes.CDLL(igs.LIB_PATH, mode=os.RTLD_NOW | os.RTLD_LOCAL)
