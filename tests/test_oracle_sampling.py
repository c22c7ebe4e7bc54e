"""Pins for the oracle's mesh-dependent sampling length (Sec. 7.3.3):
M(h) = max{1, floor(c h^((p-q+beta)/(q+1)))}, h = 1/nelem."""
import math

import pytest


@pytest.mark.parametrize("nelem,p,q,c,beta,want", [
    # h^e = 4096^(5/12) = 2^5 exactly: 0.75 * 32 = 24 (an integer in exact arithmetic)
    (4096, 2, 5, 0.75, 0.5, 24),
    (4096, 2, 5, 0.25, 0.5, 8),
    (4096, 2, 5, 3.0, 0.5, 96),
    # 64^(5/12) = 2^2.5 = 5.657: c = 1 -> 5, c = 3 -> 16.97, c = 4 -> 22.6, c = 0.25 -> 1.41
    (64, 2, 5, 1.0, 0.5, 5),
    (64, 2, 5, 3.0, 0.5, 16),
    (64, 2, 5, 4.0, 0.5, 22),
    (64, 2, 5, 0.25, 0.5, 1),
    # beta = 0, p = 1, q = 3: 256^(2/4) = 16
    (256, 1, 3, 1.0, 0.0, 16),
    (256, 1, 3, 0.5, 0.0, 8),
    # q < p + beta: e > 0, c h^e < 1, so M = 1 (the max{1, .} branch)
    (100, 3, 2, 2.0, 0.5, 1),
    # c = 0 -> 1
    (1000, 2, 5, 0.0, 0.5, 1),
])
def test_sampling_length_values(oracle, nelem, p, q, c, beta, want):
    assert oracle.sampling_length(nelem, p, q, c, beta) == want


@pytest.mark.parametrize("p,q", [(2, 5), (1, 3), (3, 5), (2, 4)])
@pytest.mark.parametrize("c", [0.25, 0.5, 0.75, 1.0, 2.0, 3.0, 4.0])
def test_sampling_length_bound_and_maximality(oracle, p, q, c):
    """The paper's bound H^(q+1) <= c^(q+1) h^(p+1+beta) with H = M h, and M is
    the largest integer with it (checked in floating point away from ties)."""
    beta = 0.5
    for nelem in (16, 40, 100, 333, 1024, 3000):
        h = 1.0 / nelem
        M = oracle.sampling_length(nelem, p, q, c, beta)
        bound = c ** (q + 1) * h ** (p + 1 + beta)
        if M > 1:
            assert (M * h) ** (q + 1) <= bound * (1 + 1e-9)
        nxt = ((M + 1) * h) ** (q + 1)
        if abs(nxt / bound - 1) > 1e-9:
            assert nxt > bound
        # and the plain floating-point formula, where it is not near an integer
        v = c * h ** ((p - q + beta) / (q + 1))
        if abs(v - round(v)) > 1e-9:
            assert M == max(1, math.floor(v))


def test_sampling_length_rejects(oracle):
    for args in [(0, 2, 5, 1.0, 0.5), (10, 0, 5, 1.0, 0.5), (10, 2, 0, 1.0, 0.5), (10, 2, 5, -1.0, 0.5),
                 (10, 2, 5, 1.0, -0.5)]:
        with pytest.raises(ValueError):
            oracle.sampling_length(*args)
