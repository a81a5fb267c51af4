"""Isotropic-basis tables for the oracle (test infrastructure only).

* Multiplets Lambda (Section 2.1): principal ell_1..ell_{N-1} plus intermediates
  ell_12, ell_123, ... in the order (l1, l2, (l12), l3, (l123), l4, l5), enumerated
  lexicographically with the last entry fastest.  Principal ell_i <= lmax; the
  intermediates are bounded by their triangle conditions only; by default only
  parity-even multiplets (even sum of principal ell) are kept (Section 3.1 and the
  summation section of the implementation).
* Coupling coefficients C^Lambda_M (eq. basis-coupling): E(Lambda) times the
  sqrt(2 l_int + 1) factors times the sum over intermediate m of
  (-1)^kappa times a chain of 3j symbols.  For N = 3 the chain is the single
  symbol (l l 0; m1 m2 0), which reproduces eq. N=3-coeff.
* Radial-bin tuples B: strictly increasing (N-1)-tuples, lexicographic with the
  last index fastest (Section 3.2.1, distinct bins).

Every M with sum m = 0 is listed (the oracle sums the full M sum of eq.
NPCF-mult-discrete-binned-estimator, not the half sum of Appendix B).
"""
from functools import lru_cache
from itertools import combinations, product
from math import sqrt

from .wigner3j import wigner3j

__all__ = ["multiplets", "principal", "parity_E", "coupling", "coupling_terms",
           "bin_tuples"]


def _tri(a, b):
    return range(abs(a - b), a + b + 1)


@lru_cache(maxsize=None)
def multiplets(N: int, lmax: int, parity: str = "even"):
    """Tuple of multiplets; each is a tuple in (l1, l2, (l12), l3, (l123), l4, l5) order."""
    if N not in (3, 4, 5, 6):
        raise ValueError("N must be 3..6")
    L = range(lmax + 1)
    out = []
    if N == 3:
        cand = [(l, l) for l in L]
    elif N == 4:
        cand = [(l1, l2, l3) for l1 in L for l2 in L for l3 in _tri(l1, l2) if l3 <= lmax]
    elif N == 5:
        cand = [(l1, l2, l12, l3, l4)
                for l1 in L for l2 in L for l12 in _tri(l1, l2)
                for l3 in L for l4 in _tri(l12, l3) if l4 <= lmax]
    else:
        cand = [(l1, l2, l12, l3, l123, l4, l5)
                for l1 in L for l2 in L for l12 in _tri(l1, l2)
                for l3 in L for l123 in _tri(l12, l3)
                for l4 in L for l5 in _tri(l123, l4) if l5 <= lmax]
    for lam in cand:
        s = sum(principal(N, lam))
        if parity == "even" and s % 2:
            continue
        if parity == "odd" and not s % 2:
            continue
        out.append(lam)
    return tuple(out)


def principal(N: int, lam):
    """Principal angular momenta (l1..l_{N-1}) of a multiplet."""
    if N <= 4:
        return tuple(lam)
    if N == 5:
        return (lam[0], lam[1], lam[3], lam[4])
    return (lam[0], lam[1], lam[3], lam[5], lam[6])


def intermediates(N: int, lam):
    if N <= 4:
        return ()
    if N == 5:
        return (lam[2],)
    return (lam[2], lam[4])


def parity_E(N: int, lam) -> int:
    """E(Lambda) = (-1)^(sum of principal ell)."""
    return -1 if sum(principal(N, lam)) % 2 else 1


def coupling(N: int, lam, M) -> float:
    """C^Lambda_M of eq. basis-coupling (includes E(Lambda))."""
    ls = principal(N, lam)
    if len(M) != N - 1 or sum(M) != 0:
        return 0.0
    if any(abs(m) > l for m, l in zip(M, ls)):
        return 0.0
    E = parity_E(N, lam)
    if N == 3:
        return E * wigner3j(ls[0], ls[1], 0, M[0], M[1], 0)
    if N == 4:
        return E * wigner3j(ls[0], ls[1], ls[2], M[0], M[1], M[2])
    if N == 5:
        l1, l2, l3, l4 = ls
        l12 = lam[2]
        m1, m2, m3, m4 = M
        m12 = m1 + m2          # fixed by the first 3j symbol
        if abs(m12) > l12:
            return 0.0
        kappa = l12 - m12
        val = ((-1) ** (kappa % 2) * wigner3j(l1, l2, l12, m1, m2, -m12)
               * wigner3j(l12, l3, l4, m12, m3, m4))
        return E * sqrt(2 * l12 + 1) * val
    l1, l2, l3, l4, l5 = ls
    l12, l123 = lam[2], lam[4]
    m1, m2, m3, m4, m5 = M
    m12 = m1 + m2
    m123 = m12 + m3
    if abs(m12) > l12 or abs(m123) > l123:
        return 0.0
    kappa = (l12 - m12) + (l123 - m123)
    val = ((-1) ** (kappa % 2) * wigner3j(l1, l2, l12, m1, m2, -m12)
           * wigner3j(l12, l3, l123, m12, m3, -m123)
           * wigner3j(l123, l4, l5, m123, m4, m5))
    return E * sqrt(2 * l12 + 1) * sqrt(2 * l123 + 1) * val


@lru_cache(maxsize=None)
def coupling_terms(N: int, lmax: int, parity: str = "even"):
    """Full-M-sum term list: list of (lambda_index, (l_1..l_{N-1}), (m_1..m_{N-1}), C).

    Only terms with C != 0 are kept (zero terms contribute nothing).
    """
    terms = []
    for li, lam in enumerate(multiplets(N, lmax, parity)):
        ls = principal(N, lam)
        for M in product(*[range(-l, l + 1) for l in ls[:-1]]):
            mlast = -sum(M)
            if abs(mlast) > ls[-1]:
                continue
            full = tuple(M) + (mlast,)
            c = coupling(N, lam, full)
            if c != 0.0:
                terms.append((li, ls, full, c))
    return tuple(terms)


def bin_tuples(N: int, nbins: int):
    """Strictly increasing (N-1)-tuples of radial bins, last index fastest."""
    return tuple(combinations(range(nbins), N - 1))
