"""Brute-force O(N_g^N) NPCF multiplets (Section 5.2, eq. brute-force-npcf).

TEST INFRASTRUCTURE ONLY.  Used to pin the factorised oracle.

For every primary i and every ordered tuple of secondaries (j_1 .. j_{N-1}) with
j_k in radial bin b_k of i, the tuple contributes

    w_i prod_k w_{j_k} * conj(P_Lambda(d_{i j_1}^, ..., d_{i j_{N-1}}^))

where P_Lambda = sum_M C^Lambda_M prod_k Y_{l_k m_k} (eq. basis-def).  The tuple sum is
carried out explicitly (no factorisation into harmonic coefficients).  The
garbled bin arguments of the printed formula are read as Theta^{b_k}(|r_{j_k} - r_i|)
for k = 1..N-1, with the weights of eq. NPCF-mult-discrete-binned-estimator.

This is independent of the factorised oracle in its building blocks: the 3j
symbols come from sympy.physics.wigner and Y_lm from scipy.special.sph_harm_y;
only the multiplet index set is shared.
"""
from functools import lru_cache
from itertools import product

import numpy as np

from .basis import bin_tuples, intermediates, multiplets, parity_E, principal


@lru_cache(maxsize=None)
def _w3j(j1, j2, j3, m1, m2, m3):
    from sympy.physics.wigner import wigner_3j
    return float(wigner_3j(j1, j2, j3, m1, m2, m3))


def _chain(N, lam, M):
    """Coupling of eq. basis-coupling from sympy 3j symbols (E included)."""
    ls = principal(N, lam)
    ints = intermediates(N, lam)
    E = parity_E(N, lam)
    if N == 3:
        return E * _w3j(ls[0], ls[1], 0, M[0], M[1], 0)
    if N == 4:
        return E * _w3j(ls[0], ls[1], ls[2], M[0], M[1], M[2])
    # general chain: m_{12..k} partial sums; kappa sums (l_int - m_int)
    pref = np.prod([np.sqrt(2 * li + 1) for li in ints])
    msum = M[0] + M[1]
    val = _w3j(ls[0], ls[1], ints[0], M[0], M[1], -msum)
    kappa = ints[0] - msum
    for k in range(1, len(ints)):
        mnext = msum + M[k + 1]
        val *= _w3j(ints[k - 1], ls[k + 1], ints[k], msum, M[k + 1], -mnext)
        kappa += ints[k] - mnext
        msum = mnext
    val *= _w3j(ints[-1], ls[-2], ls[-1], msum, M[-2], M[-1])
    return E * pref * (-1) ** (kappa % 2) * val


@lru_cache(maxsize=None)
def _terms(N, lmax, parity):
    out = []
    for lam in multiplets(N, lmax, parity):
        ls = principal(N, lam)
        tl = []
        for M in product(*[range(-l, l + 1) for l in ls]):
            if sum(M) != 0:
                continue
            c = _chain(N, lam, M)
            if c != 0.0:
                tl.append((M, c))
        out.append((lam, ls, tl))
    return tuple(out)


def _ylm(l, m, v):
    from scipy.special import sph_harm_y
    r = np.linalg.norm(v, axis=-1)
    theta = np.arccos(np.clip(v[..., 2] / r, -1.0, 1.0))
    phi = np.arctan2(v[..., 1], v[..., 0])
    return sph_harm_y(l, m, theta, phi)


def basis_function(N, lam, vecs):
    """P_Lambda(r1^, ..., r_{N-1}^) from eq. basis-def with sympy/scipy building blocks.

    vecs: array [..., N-1, 3].  Returns complex array [...]."""
    vecs = np.asarray(vecs, dtype=np.float64)
    ls = principal(N, lam)
    total = np.zeros(vecs.shape[:-2], dtype=complex)
    for M in product(*[range(-l, l + 1) for l in ls]):
        if sum(M) != 0:
            continue
        c = _chain(N, lam, M)
        if c == 0.0:
            continue
        term = np.full(vecs.shape[:-2], c, dtype=complex)
        for k in range(N - 1):
            term = term * _ylm(ls[k], M[k], vecs[..., k, :])
        total += term
    return total


def brute_zeta(pos, w, N, lmax, edges, box=None, parity="even"):
    """Z^B_Lambda by explicit tuple sums; Re for even, Im for odd multiplets."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    w = np.asarray(w, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.float64)
    nb = len(edges) - 1
    Btab = bin_tuples(N, nb)
    terms = _terms(N, lmax, parity)
    nlam = len(terms)
    Z = np.zeros((nlam, len(Btab)), dtype=complex)
    n = len(w)
    for i in range(n):
        d = pos - pos[i]
        if box is not None:
            L = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
            d = d - L * np.round(d / L)
        r = np.sqrt(np.sum(d * d, axis=1))
        binid = np.full(n, -1)
        for b in range(nb):
            sel = (r >= edges[b]) & (r < edges[b + 1])
            binid[sel] = b
        binid[i] = -1
        members = [np.nonzero(binid == b)[0] for b in range(nb)]
        for bi, B in enumerate(Btab):
            sets = [members[b] for b in B]
            if any(len(s) == 0 for s in sets):
                continue
            grids = np.meshgrid(*sets, indexing="ij")
            idx = [g.reshape(-1) for g in grids]          # tuples of secondaries
            wt = np.ones(len(idx[0]))
            for k in range(N - 1):
                wt = wt * w[idx[k]]
            vecs = [d[idx[k]] for k in range(N - 1)]
            for li, (lam, ls, tl) in enumerate(terms):
                ys = {}
                P = np.zeros(len(wt), dtype=complex)
                for M, c in tl:
                    t = np.full(len(wt), c, dtype=complex)
                    for k in range(N - 1):
                        key = (k, ls[k], M[k])
                        if key not in ys:
                            ys[key] = _ylm(ls[k], M[k], vecs[k])
                        t = t * ys[key]
                    P += t
                Z[li, bi] += w[i] * np.sum(wt * np.conj(P))
    odd = np.array([parity_E(N, lam) < 0 for lam, _, _ in terms], dtype=bool)
    return np.where(odd[:, None], Z.imag, Z.real)
