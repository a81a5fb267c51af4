"""Edge correction for the oracle (test infrastructure only).

Follows Section 3.2 (Edge Correction) of the paper:

* generalized Gaunt integral G^{L L' L''} = int dR P_L P_L' P_L''
  (eq. generalized-gaunt-def).  `gaunt_definition` writes the definition out: with
  P_L = sum_M C^L_M prod_i Y_{l_i m_i} (eq. basis-def) the integral factorises over
  the N-1 directions into ordinary Gaunt integrals of three spherical harmonics,
  int Y Y Y = sqrt((2a+1)(2b+1)(2c+1)/(4 pi)) (a b c; 0 0 0)(a b c; m m' m'').
  `gaunt_closed` is the closed form of Appendix A for N = 3, 4, 5 (3j and 9j
  symbols), extended to N = 6 the way the appendix builds the lower orders: one 9j
  symbol per node of the coupling tree (l1 l2 -> l12, l12 l3 -> l123, l123 l4 ->
  l5) and sqrt((2x+1)(2x'+1)(2x''+1)) per intermediate x, over (4 pi)^{5/2}.  The
  two are pinned against each other in tests/test_edge_oracle.py (N = 6 included).
* coupling matrix M_{L L''}(B) = sum_{L'} f_{L'}(B) E(L'') G^{L L' L''} with
  f_{L'} = R_{L'} / R_0 (eq. edge-correction-matrix).  The paper writes it for the
  complex multiplets; odd multiplets are imaginary (Section 3.1) and are carried
  here, as everywhere in this package, by their imaginary parts.  Written for
  those real numbers the sum gains i * i = -1 in every term whose L and L' are
  both odd (G vanishes unless L, L', L'' hold an even number of odd multiplets, so
  no other factor of i is left over);
* the edge-corrected estimator solves N_{L''} / R_0 = sum_L zeta_L M_{L L''} for
  zeta, one linear system per bin tuple B (eq. edge-corrected-NPCF; the system is
  solved as written in eq. edge-correction-matrix, i.e. with M transposed).

Wigner 6j and 9j symbols: Racah's single sum for the 6j symbol (DLMF 34.4.3) and
the 6j-product sum for the 9j symbol (DLMF 34.6.2), in exact rational arithmetic
for the squared 6j values; pinned against sympy.
"""
from fractions import Fraction
from functools import lru_cache
from itertools import product
from math import factorial, pi, sqrt

import numpy as np

from .basis import coupling, multiplets, parity_E, principal
from .wigner3j import wigner3j

__all__ = ["wigner6j", "wigner9j", "gaunt_ylm", "gaunt_definition", "gaunt_closed",
           "gaunt_tensor", "coupling_matrix", "edge_correct"]


def _tri(a, b, c):
    return abs(a - b) <= c <= a + b and (a + b + c) % 1 == 0


def _delta_sq(a, b, c):
    """Triangle coefficient squared: (a+b-c)!(a-b+c)!(-a+b+c)!/(a+b+c+1)!."""
    return Fraction(factorial(a + b - c) * factorial(a - b + c) * factorial(-a + b + c),
                    factorial(a + b + c + 1))


@lru_cache(maxsize=None)
def wigner6j(j1, j2, j3, j4, j5, j6) -> float:
    """{j1 j2 j3; j4 j5 j6} for integer arguments (Racah, DLMF 34.4.3)."""
    if not (_tri(j1, j2, j3) and _tri(j1, j5, j6) and _tri(j4, j2, j6) and _tri(j4, j5, j3)):
        return 0.0
    pre = (_delta_sq(j1, j2, j3) * _delta_sq(j1, j5, j6) * _delta_sq(j4, j2, j6)
           * _delta_sq(j4, j5, j3))
    a = (j1 + j2 + j3, j1 + j5 + j6, j4 + j2 + j6, j4 + j5 + j3)
    b = (j1 + j2 + j4 + j5, j2 + j3 + j5 + j6, j3 + j1 + j6 + j4)
    s = Fraction(0)
    for t in range(max(a), min(b) + 1):
        den = 1
        for x in a:
            den *= factorial(t - x)
        for y in b:
            den *= factorial(y - t)
        s += Fraction((-1) ** t * factorial(t + 1), den)
    return float(s) * sqrt(pre)


@lru_cache(maxsize=None)
def wigner9j(j1, j2, j3, j4, j5, j6, j7, j8, j9) -> float:
    """{j1 j2 j3; j4 j5 j6; j7 j8 j9} = sum_x (-1)^{2x} (2x+1)
    {j1 j4 j7; j8 j9 x} {j2 j5 j8; j4 x j6} {j3 j6 j9; x j1 j2} (DLMF 34.6.2)."""
    lo = max(abs(j1 - j9), abs(j4 - j8), abs(j2 - j6))
    hi = min(j1 + j9, j4 + j8, j2 + j6)
    s = 0.0
    for x in range(lo, hi + 1):
        s += ((2 * x + 1) * wigner6j(j1, j4, j7, j8, j9, x) * wigner6j(j2, j5, j8, j4, x, j6)
              * wigner6j(j3, j6, j9, x, j1, j2))
    return s


def gaunt_ylm(a, b, c, ma, mb, mc) -> float:
    """int dOmega Y_{a ma} Y_{b mb} Y_{c mc} (no conjugation)."""
    if ma + mb + mc != 0:
        return 0.0
    return (sqrt((2 * a + 1) * (2 * b + 1) * (2 * c + 1) / (4 * pi))
            * wigner3j(a, b, c, 0, 0, 0) * wigner3j(a, b, c, ma, mb, mc))


def _ms(ls):
    """All M = (m_1..m_{N-1}) with |m_i| <= l_i and sum m = 0."""
    for M in product(*[range(-l, l + 1) for l in ls]):
        if sum(M) == 0:
            yield M


def gaunt_definition(N, lam, lamp, lampp) -> float:
    """G^{L L' L''} by its definition: sum over M, M' of C C C times the product
    over directions of ordinary Gaunt integrals (M'' fixed by m''_i = -m_i - m'_i)."""
    l, lp, lpp = principal(N, lam), principal(N, lamp), principal(N, lampp)
    s = 0.0
    for M in _ms(l):
        c = coupling(N, lam, M)
        if c == 0.0:
            continue
        for Mp in _ms(lp):
            cp = coupling(N, lamp, Mp)
            if cp == 0.0:
                continue
            Mpp = tuple(-m - mp for m, mp in zip(M, Mp))
            if any(abs(m) > x for m, x in zip(Mpp, lpp)):
                continue
            cpp = coupling(N, lampp, Mpp)
            if cpp == 0.0:
                continue
            g = 1.0
            for i in range(N - 1):
                g *= gaunt_ylm(l[i], lp[i], lpp[i], M[i], Mp[i], Mpp[i])
                if g == 0.0:
                    break
            s += c * cp * cpp * g
    return s


def gaunt_closed(N, lam, lamp, lampp) -> float:
    """Appendix A closed forms for N = 3, 4, 5, and the same construction for N = 6."""
    l, lp, lpp = principal(N, lam), principal(N, lamp), principal(N, lampp)
    prod3 = 1.0
    for i in range(N - 1):
        prod3 *= (sqrt((2 * l[i] + 1) * (2 * lp[i] + 1) * (2 * lpp[i] + 1))
                  * wigner3j(l[i], lp[i], lpp[i], 0, 0, 0))
        if prod3 == 0.0:
            return 0.0
    if N == 3:
        # {l, l}: (1 / 4 pi) sqrt((2l+1)(2l'+1)(2l''+1)) (l l' l''; 0 0 0)^2
        x = wigner3j(l[0], lp[0], lpp[0], 0, 0, 0)
        return sqrt((2 * l[0] + 1) * (2 * lp[0] + 1) * (2 * lpp[0] + 1)) * x * x / (4 * pi)
    if N == 4:
        return prod3 / (4 * pi) ** 1.5 * wigner9j(l[0], lp[0], lpp[0], l[1], lp[1], lpp[1],
                                                  l[2], lp[2], lpp[2])
    if N == 5:
        l12, l12p, l12pp = lam[2], lamp[2], lampp[2]
        return (prod3 / (4 * pi) ** 2 * sqrt((2 * l12 + 1) * (2 * l12p + 1) * (2 * l12pp + 1))
                * wigner9j(l[0], l[1], l12, lp[0], lp[1], l12p, lpp[0], lpp[1], l12pp)
                * wigner9j(l12, l[2], l[3], l12p, lp[2], lp[3], l12pp, lpp[2], lpp[3]))
    if N == 6:
        x12, x12p, x12pp = lam[2], lamp[2], lampp[2]
        x123, x123p, x123pp = lam[4], lamp[4], lampp[4]
        return (prod3 / (4 * pi) ** 2.5
                * sqrt((2 * x12 + 1) * (2 * x12p + 1) * (2 * x12pp + 1))
                * sqrt((2 * x123 + 1) * (2 * x123p + 1) * (2 * x123pp + 1))
                * wigner9j(l[0], l[1], x12, lp[0], lp[1], x12p, lpp[0], lpp[1], x12pp)
                * wigner9j(x12, l[2], x123, x12p, lp[2], x123p, x12pp, lpp[2], x123pp)
                * wigner9j(x123, l[3], l[4], x123p, lp[3], lp[4], x123pp, lpp[3], lpp[4]))
    raise ValueError("closed forms are given for N = 3..6")


@lru_cache(maxsize=None)
def gaunt_tensor(N, lmax, parity="even", method="closed"):
    """G[L, L', L''] over the multiplet list of (N, lmax, parity)."""
    lams = multiplets(N, lmax, parity)
    n = len(lams)
    f = gaunt_closed if method == "closed" else gaunt_definition
    G = np.zeros((n, n, n))
    for a in range(n):
        for b in range(n):
            for c in range(n):
                G[a, b, c] = f(N, lams[a], lams[b], lams[c])
    return G


def coupling_matrix(N, lmax, R, parity="even"):
    """M[B, L, L''] = sum_L' (R[L', B] / R[0, B]) s(L, L') E(L'') G[L, L', L''] for
    multiplets R[L, B] of the randoms (row 0 is L = 0; odd rows are imaginary parts),
    with s(L, L') = -1 when L and L' are both odd (i * i), else +1."""
    lams = multiplets(N, lmax, parity)
    G = gaunt_tensor(N, lmax, parity)
    E = np.array([parity_E(N, x) for x in lams], dtype=float)
    odd = E < 0
    s = np.where(odd[:, None] & odd[None, :], -1.0, 1.0)
    R = np.asarray(R, dtype=float)
    f = R / R[0][None, :]
    return np.einsum("pb,lpq,lp,q->blq", f, G, s, E)


def edge_correct(N, lmax, Nmult, Rmult, parity="even", lmax_out=None):
    """zeta[L, B] solving N[L'', B] / R[0, B] = sum_L zeta[L, B] M[B, L, L''],
    returned for the multiplets with every principal ell <= lmax_out."""
    lams = multiplets(N, lmax, parity)
    M = coupling_matrix(N, lmax, Rmult, parity)
    Nm = np.asarray(Nmult, dtype=float)
    R0 = np.asarray(Rmult, dtype=float)[0]
    nB = Nm.shape[1]
    Z = np.empty_like(Nm)
    for b in range(nB):
        Z[:, b] = np.linalg.solve(M[b].T, Nm[:, b] / R0[b])
    if lmax_out is None:
        return Z
    keep = [i for i, x in enumerate(lams) if max(principal(N, x)) <= lmax_out]
    return Z[keep]
