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


def test_closed_form_n6_matches_definition():
    """The N = 6 closed form (three 9j symbols, two intermediates) against the
    definition: every triple at lmax = 1 (both parities), and 600 triples at lmax
    = 2 that pass the per-direction triangle rules (the others vanish on both
    sides)."""
    lams = multiplets(6, 1, "all")
    worst, nonzero = 0.0, 0
    for a in lams:
        for b in lams:
            for c in lams:
                g = edge.gaunt_closed(6, a, b, c)
                la, lb, lc = principal(6, a), principal(6, b), principal(6, c)
                if not all(abs(x - y) <= z <= x + y and (x + y + z) % 2 == 0 for x, y, z in zip(la, lb, lc)):
                    assert g == 0.0
                    continue
                d = edge.gaunt_definition(6, a, b, c)
                nonzero += abs(d) > 1e-12
                worst = max(worst, abs(g - d))
    assert nonzero > 1000 and worst < 1e-13
    rng = np.random.default_rng(6)
    lams = multiplets(6, 2, "all")
    n, worst, nonzero = 0, 0.0, 0
    while n < 600:
        a, b, c = (lams[i] for i in rng.integers(0, len(lams), 3))
        la, lb, lc = principal(6, a), principal(6, b), principal(6, c)
        if not all(abs(x - y) <= z <= x + y and (x + y + z) % 2 == 0 for x, y, z in zip(la, lb, lc)):
            continue
        n += 1
        d = edge.gaunt_definition(6, a, b, c)
        nonzero += abs(d) > 1e-12
        worst = max(worst, abs(edge.gaunt_closed(6, a, b, c) - d))
    assert nonzero > 200 and worst < 1e-13


@pytest.mark.parametrize("N,lmax,parity", [(3, 3, "even"), (4, 2, "all"), (5, 1, "even"), (6, 1, "all")])
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


@pytest.mark.parametrize("N,lmax", [(3, 3), (4, 2), (6, 1)])
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


def _sphere_nodes(deg):
    """Gauss-Legendre in cos(theta) x uniform phi: exact for polynomials of degree
    <= deg on the sphere."""
    x, wx = np.polynomial.legendre.leggauss(deg // 2 + 1)
    nphi = deg + 1
    phi = 2.0 * np.pi * np.arange(nphi) / nphi
    st = np.sqrt(1.0 - x * x)
    v = np.stack([np.outer(st, np.cos(phi)), np.outer(st, np.sin(phi)),
                  np.outer(x, np.ones(nphi))], axis=-1).reshape(-1, 3)
    w = np.outer(wx, np.full(nphi, 2.0 * np.pi / nphi)).reshape(-1)
    return v, w


def _product_projection(N, lmax, z, r):
    """N_L'' / R_0 from the functional identity of eq. edge-correction-tmp,
    [sum_L zeta_L P_L(R^)] [sum_L' f_L' P_L'(R^)] = sum_L'' (N_L'' / R_0) P_L''(R^),
    projected on P_L'' by orthonormality (eq. basis-orthogonality) with a quadrature
    exact for the degree 3 lmax integrands.  P_L from sympy 3j symbols and scipy
    Y_lm (oracle.brute), no Gaunt integral anywhere.  Coefficients are carried as
    real numbers, Re for even and Im for odd multiplets, as the estimator returns
    them; the complex ones are rebuilt here."""
    from itertools import product as iprod
    from oracle import brute
    from oracle.basis import parity_E
    lams = multiplets(N, lmax, "all")
    odd = np.array([parity_E(N, x) < 0 for x in lams])
    v1, w1 = _sphere_nodes(3 * lmax)
    K = N - 1
    idx = np.array(list(iprod(range(len(w1)), repeat=K)))
    vecs = v1[idx]                                   # [P, K, 3]
    wts = np.prod(w1[idx], axis=1)
    P = np.stack([brute.basis_function(N, lam, vecs) for lam in lams])
    assert np.max(np.abs((P * wts) @ P.conj().T - np.eye(len(lams)))) < 1e-12
    cz = np.where(odd, 1j, 1.0) * z
    cf = np.where(odd, 1j, 1.0) * r / r[0]
    F = (cz @ P) * (cf @ P)
    assert np.max(np.abs(F.imag)) < 1e-12 * np.max(np.abs(F))   # a real function
    cN = (P.conj() * wts) @ F
    return np.where(odd, cN.imag, cN.real), odd


@pytest.mark.parametrize("N,lmax", [(3, 2), (4, 1), (4, 2), (5, 1)])
def test_coupling_matrix_matches_product_projection(N, lmax):
    """Pins eq. edge-correction-matrix in mixed parity: sum_L zeta_L M_{L L''} equals
    the projection of the product of the zeta and window functions, for windows
    with odd multiplets.  For the real multiplets (Im of the odd ones) M comes out
    symmetric, so the index order of the solve cannot matter; the i * i sign of
    the odd x odd terms does: the matrix without it misses the projection."""
    from oracle.basis import parity_E
    lams = multiplets(N, lmax, "all")
    n = len(lams)
    G = edge.gaunt_tensor(N, lmax, "all")
    E = np.array([parity_E(N, x) for x in lams], dtype=float)
    rng = np.random.default_rng(11 + N + lmax)
    worst = 0.0
    for trial in range(3):
        z = rng.normal(size=n)
        r = rng.normal(0.0, 0.3, n)
        r[0] = rng.uniform(1.0, 2.0)
        nq, odd = _product_projection(N, lmax, z, r)
        M = edge.coupling_matrix(N, lmax, r[:, None], "all")[0]
        assert np.max(np.abs(M - M.T)) < 1e-15
        worst = max(worst, np.max(np.abs(z @ M - nq)))
        if N >= 4:   # N = 3 has only even multiplets (l1 = l2)
            assert odd.any() and (~odd).any()
            unsigned = np.einsum("p,lpq,q->lq", r / r[0], G, E)
            assert np.max(np.abs(z @ unsigned - nq)) > 1e-3
        # the edge correction recovers zeta from the projected N
        Z = edge.edge_correct(N, lmax, (nq * r[0])[:, None], r[:, None], parity="all")
        assert np.max(np.abs(Z[:, 0] - z)) < 1e-11
    assert worst < 1e-12
