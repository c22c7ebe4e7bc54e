"""The allocation-free assembly (igs_assemble_noalloc) against the entry points
it stands in for: M = 0 against igs_assemble_exact, M >= 1 against
igs_assemble_surrogate, on the same preallocated bands.  Two calls in a row
per form, the second on a smaller problem, so that the static scratch still
holding the first call's tables cannot leak into the second result; the
smaller results are also checked against the FP64 oracle (1e-12 relative in
the max norm)."""
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


def _pair(igs, prob, form, M, q, dtype):
    """(noalloc band, reference band), both preallocated by the caller."""
    import torch

    tdt = torch.float64 if dtype == igs.F64 else torch.float32
    a = igs.empty_band(prob, tdt)
    b = igs.empty_band(prob, tdt)
    a.fill_(float("nan"))
    torch.cuda.synchronize()
    igs.assemble_noalloc(prob, form, M=M, q=q, dtype=tdt, out=a)
    if M == 0:
        igs.assemble_exact(prob, form, dtype=tdt, out=b)
    else:
        igs.assemble_surrogate(prob, form, M=M, q=q, dtype=tdt, out=b)
    torch.cuda.synchronize()
    return a, b


SEQUENCES = [
    # (problem, form, M, q, dtype): the second entry of each pair is smaller
    [(W.problem(3, 3, (12, 10, 11)), 0, 0, 3, 0), (W.problem(2, 2, 21), 1, 0, 3, 0)],
    [(W.problem(3, 3, 24), 0, 4, 3, 0), (W.problem(3, 2, (15, 13, 14)), 1, 3, 2, 0)],
    [(W.problem(2, 3, 64, coef="sine3", camp=0.5), 0, 8, 3, 0), (W.problem(2, 2, 30), 0, 4, 3, 1)],
]


@pytest.mark.parametrize("seq", SEQUENCES)
def test_noalloc_matches_allocating_calls(igs, oracle, seq):
    for k, (prob, form, M, q, dtype) in enumerate(seq):
        print(f"noalloc case {k}: n={prob['n']} p={prob['p']} nelem={prob['nelem']} form={form} M={M} q={q}",
              flush=True)
        a, b = _pair(igs, prob, form, M, q, dtype)
        lay = igs.layout(prob)
        N = lay.N
        diff = float((a[:, :, :N].double() - b[:, :, :N].double()).abs().max())
        scale = float(b[:, :, :N].double().abs().max())
        assert diff <= 1e-13 * scale, (k, diff)
        assert float(a[:, :, N:].abs().max()) == 0.0
        if k == len(seq) - 1:
            ref = oracle.exact_rows(prob, form, np.arange(N)) if M == 0 else oracle.surrogate_rows(prob, form, M, q)
            tol = 1e-12 if dtype == 0 else 2e-6
            assert rel_maxnorm(igs.band_rows(a, prob), ref) < tol


def test_noalloc_rejects_oversized_scratch(igs):
    """A surrogate whose coefficient scratch exceeds the static array is refused
    before any kernel runs (the band pointer is never touched)."""
    import ctypes

    import torch

    prob = W.problem(3, 3, 64)          # M = 1: 55^3 samples x 172 slots x 3 buffers
    dummy = torch.empty(64, dtype=torch.float64, device="cuda")
    pb = igs.make_problem(prob)
    st = igs.lib().igs_assemble_noalloc(ctypes.byref(pb), 0, 1, 3, 0, ctypes.c_void_p(dummy.data_ptr()),
                                        igs._stream())
    torch.cuda.synchronize()
    assert igs.STATUS[st] == "IGS_ERR_SCRATCH"
    # the array still serves the next call
    a, b = _pair(igs, W.problem(2, 2, 21), 0, 4, 3, 0)
    assert float((a - b).abs().max()) <= 1e-13 * float(b.abs().max())
