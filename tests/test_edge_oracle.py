"""Pins of the edge-correction oracle (Section 3.2 and Appendix A), CPU only."""
import random

import numpy as np
import pytest

from oracle import edge
from oracle.basis import multiplets, principal


def test_6j_9j_match_sympy():
    from sympy.physics.wigner import wigner_6j, wigner_9j
    rng = random.Random(5)
    for _ in range(300):
        j = [rng.randint(0, 4) for _ in range(6)]
        assert abs(edge.wigner6j(*j) - float(wigner_6j(*j))) < 1e-14
    for _ in range(200):
        j = [rng.randint(0, 3) for _ in range(9)]
        assert abs(edge.wigner9j(*j) - float(wigner_9j(*j))) < 1e-14


def test_9j_with_zero_reduces_to_6j():
    # {a b e; c d e; f f 0} = (-1)^(b+c+e+f) {a b e; d c f} / sqrt((2e+1)(2f+1))
    for a, b, c, d, e, f in [(1, 1, 1, 1, 1, 1), (2, 1, 1, 2, 2, 1), (2, 2, 2, 1, 1, 2), (3, 2, 1, 2, 2, 2)]:
        lhs = edge.wigner9j(a, b, e, c, d, e, f, f, 0)
        rhs = (-1) ** (b + c + e + f) * edge.wigner6j(a, b, e, d, c, f) / np.sqrt((2 * e + 1) * (2 * f + 1))
        assert abs(lhs - rhs) < 1e-14


@pytest.mark.parametrize("N,lmax,parity", [(3, 4, "all"), (4, 2, "all"), (5, 1, "all")])
def test_closed_forms_match_definition(N, lmax, parity):
    """Appendix A closed forms against the definition int P P P (sum over M of
    coupling coefficients times ordinary Gaunt integrals)."""
    lams = multiplets(N, lmax, parity)
    worst = 0.0
    for a in lams:
        for b in lams:
            for c in lams:
                worst = max(worst, abs(edge.gaunt_closed(N, a, b, c) - edge.gaunt_definition(N, a, b, c)))
    assert worst < 1e-13


@pytest.mark.parametrize("N,lmax,parity", [(3, 3, "even"), (4, 2, "all"), (5, 1, "even")])
def test_periodic_window_gives_scaled_identity(N, lmax, parity):
    """Only R_0 nonzero (uniform periodic geometry): M = (4 pi)^{-(N-1)/2} I."""
    n = len(multiplets(N, lmax, parity))
    R = np.zeros((n, 4))
    R[0] = [1.0, 2.5, 7.0, 0.3]
    M = edge.coupling_matrix(N, lmax, R, parity)
    assert np.max(np.abs(M - (4 * np.pi) ** (-(N - 1) / 2) * np.eye(n)[None])) < 1e-15


def test_gaunt_selection_rules():
    """G vanishes unless every direction's (l, l', l'') closes a triangle with an
    even sum (the 3j symbols with zero m), hence also for an odd total sum."""
    N, lmax = 4, 2
    lams = multiplets(N, lmax, "all")
    G = edge.gaunt_tensor(N, lmax, "all")
    for i, a in enumerate(lams):
        for j, b in enumerate(lams):
            for k, c in enumerate(lams):
                la, lb, lc = principal(N, a), principal(N, b), principal(N, c)
                ok = all(abs(x - y) <= z <= x + y and (x + y + z) % 2 == 0 for x, y, z in zip(la, lb, lc))
                if not ok:
                    assert G[i, j, k] == 0.0


@pytest.mark.parametrize("N,lmax", [(3, 3), (4, 2)])
def test_solution_recovers_known_zeta(N, lmax):
    """Closed loop: N'' = R_0 sum_L zeta_L M_{L L''} for a known zeta and a
    non-trivial window; the edge correction returns that zeta."""
    rng = np.random.default_rng(3)
    lams = multiplets(N, lmax)
    n, nB = len(lams), 6
    R = rng.normal(0.0, 0.05, (n, nB))
    R[0] = rng.uniform(1.0, 2.0, nB)
    zeta = rng.normal(size=(n, nB))
    M = edge.coupling_matrix(N, lmax, R)
    Nm = np.einsum("lb,blq->qb", zeta, M) * R[0][None, :]
    Z = edge.edge_correct(N, lmax, Nm, R)
    assert np.max(np.abs(Z - zeta)) < 1e-12
    # lmax_out keeps the lower multiplets in the order of the lmax_out list
    Zo = edge.edge_correct(N, lmax, Nm, R, lmax_out=lmax - 1)
    keep = [lams.index(x) for x in multiplets(N, lmax - 1)]
    assert np.array_equal(Zo, Z[keep])
