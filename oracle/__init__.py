"""ORACLE -- plain, slow, FP64 CPU implementation of the discrete isotropic NPCF
estimator of Philcox et al. (2021), written from the paper.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import or run anything in this package.  The
product path (paper_2105_08722_amd) never does, and shares no code with it.

Functions and the passages they follow
--------------------------------------
* multiplets / coupling / coupling_terms / bin_tuples (oracle.basis):
  Section 2.1 eq. basis-def and eq. basis-coupling; distinct bins of Section 3.2.1.
* wigner3j (oracle.wigner3j): Racah formula, DLMF 34.2.4, exact rationals.
* ylm: orthonormal Y_lm with Condon-Shortley phase (Section 2.1), by the
  normalised Legendre recurrence (C, oracle/npcf_oracle.c).
* alm: raw harmonic coefficients of eq. binned-discrete-alm (no 1/v_b).
* zeta: Z^B_L = sum_i w_i sum_M E(L) C^L_M prod_k a~ of eq.
  NPCF-mult-discrete-binned-estimator (no 1/V), full M sum.
* dmr_weights: randoms weighted negatively so the total weight is zero
  (Section 4.2, reconstruction of the geometry-corrected NPCF).
* split_zeta: random-split co-adding (Section 4.2): the randoms are cut into
  consecutive disjoint parts, each part k gives the D-R catalog data + part k
  (weights by dmr_weights within the part) and its Z^(k) by `zeta`; the result is
  the mean over the parts.
* brute_zeta (oracle.brute): O(N_g^N) tuple sum of P*_Lambda, eq.
  brute-force-npcf, with sympy 3j symbols and scipy Y_lm.
* mesh_alm / mesh_zeta / zeta_from_alm (oracle.mesh): the gridded-data estimator
  of Section 3.2 (Gridded Data) by its definition -- eq. alm-binned-def as a direct
  correlation over periodic mesh offsets, cells as primaries weighted by delta, the
  full M sum -- pinned against the discrete oracle on catalogs moved to their cell
  centres (tests/test_mesh_oracle.py).

Pins (tests/test_oracle_pins.py): 3j vs sympy; Y_lm vs scipy; the printed
P_110 value of Section 5.2; the N=3 Legendre closed form (eq. N=3-basis); the
4PCF Legendre limits; P_0 = (4 pi)^{-(N-1)/2} (eq. basis-zero-ell) through the
pair-count closed form of Z_0; sum_M C^2 = 1 and quadrature orthonormality
(eq. basis-orthogonality); C_{-M} = E C_M (eq. basis-coupling-M-inversion);
rotation invariance; reflection Z -> E Z (eq. basis-parity-relation); the
brute-force tuple sum for N = 3..6; homogeneity in the weights; the multiplet
and task counts printed in Section 5.1/5.3.  No function is parity unpinned.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

from .basis import (bin_tuples, coupling, coupling_terms, multiplets, parity_E,
                    principal)
from .wigner3j import wigner3j

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "npcf_oracle.c")
_LIB = os.path.join(_HERE, "_npcf_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (IEEE FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", _LIB, "-lm"]
        subprocess.check_call(cmd)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_ylm.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, P]
        lib.oracle_ylm.restype = ctypes.c_int
        lib.oracle_alm.argtypes = [P, P, ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_int,
                                   P, ctypes.c_int64, P, ctypes.c_int]
        lib.oracle_alm.restype = ctypes.c_int
        lib.oracle_zeta.argtypes = ([P, P, ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P,
                                     ctypes.c_int, P, P, ctypes.c_int64, P, P, P, P,
                                     ctypes.c_int])
        lib.oracle_zeta.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def nlm(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def ylm(lmax: int, d) -> np.ndarray:
    """Y_lm(d^) for 0 <= m <= l <= lmax as complex array indexed l(l+1)/2 + m."""
    out = np.zeros(2 * nlm(lmax))
    rc = _load().oracle_ylm(int(lmax), float(d[0]), float(d[1]), float(d[2]), _ptr(out))
    if rc != 0:
        raise ValueError("zero separation has no direction")
    return out[0::2] + 1j * out[1::2]


def _prep(pos, w, box, edges):
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
    edges = np.ascontiguousarray(edges, dtype=np.float64).reshape(-1)
    if box is not None:
        box = np.ascontiguousarray(np.broadcast_to(np.asarray(box, dtype=np.float64), (3,)))
    if len(w) != len(pos):
        raise ValueError("pos and w lengths differ")
    if not np.all(np.diff(edges) > 0) or edges[0] <= 0:
        raise ValueError("edges must be strictly increasing and positive")
    return pos, w, box, edges


def _prims(n, primaries):
    if primaries is None:
        return np.arange(n, dtype=np.int64)
    return np.ascontiguousarray(primaries, dtype=np.int64)


def alm(pos, w, lmax, edges, box=None, primaries=None, nthreads=0) -> np.ndarray:
    """Raw a~^b_lm (no 1/v_b) for the primaries: complex [nprim, nbins, nlm(lmax)]."""
    pos, w, box, edges = _prep(pos, w, box, edges)
    prim = _prims(len(w), primaries)
    nb = len(edges) - 1
    out = np.zeros((len(prim), nb, nlm(lmax), 2))
    _load().oracle_alm(_ptr(pos), _ptr(w), len(w), _ptr(box), _ptr(edges), nb, int(lmax),
                       _ptr(prim), len(prim), _ptr(out), int(nthreads))
    return out[..., 0] + 1j * out[..., 1]


def term_arrays(N, lmax, parity="even"):
    """Full-M-sum term list as arrays (lam, l, m, E*C) for the C loops."""
    terms = coupling_terms(N, lmax, parity)
    lams = multiplets(N, lmax, parity)
    t_lam = np.array([t[0] for t in terms], dtype=np.int32)
    t_l = np.array([t[1] for t in terms], dtype=np.int32).reshape(-1, N - 1)
    t_m = np.array([t[2] for t in terms], dtype=np.int32).reshape(-1, N - 1)
    t_c = np.array([parity_E(N, lams[t[0]]) * t[3] for t in terms], dtype=np.float64)
    return t_lam, t_l, t_m, t_c


def zeta(pos, w, N, lmax, edges, box=None, parity="even", primaries=None,
         nthreads=0, return_abs=False, complex_out=False):
    """Raw Z^B_Lambda, FP64, shape [n_multiplets, n_bin_tuples].

    Real part for parity-even multiplets, imaginary part for parity-odd ones
    (Section 3.1: odd multiplets are purely imaginary).  With return_abs, also
    sum_i |w_i H_i| of the same component (the conditioning numerator).
    """
    pos, w, box, edges = _prep(pos, w, box, edges)
    prim = _prims(len(w), primaries)
    nb = len(edges) - 1
    lams = multiplets(N, lmax, parity)
    btab = np.ascontiguousarray(np.array(bin_tuples(N, nb), dtype=np.int32).reshape(-1, N - 1))
    nB = btab.shape[0]
    nlam = len(lams)
    zr = np.zeros(nlam * nB); zi = np.zeros(nlam * nB)
    ar = np.zeros(nlam * nB); ai = np.zeros(nlam * nB)
    if nB > 0 and nlam > 0:
        t_lam, t_l, t_m, t_c = term_arrays(N, lmax, parity)
        t_l = np.ascontiguousarray(t_l); t_m = np.ascontiguousarray(t_m)
        _load().oracle_zeta(_ptr(pos), _ptr(w), len(w), _ptr(box), _ptr(edges), nb, int(lmax),
                            N - 1, nlam, len(t_lam), _ptr(t_lam), _ptr(t_l), _ptr(t_m),
                            _ptr(t_c), nB, _ptr(btab), _ptr(prim), len(prim),
                            _ptr(zr), _ptr(zi), _ptr(ar), _ptr(ai), int(nthreads))
    zr = zr.reshape(nlam, nB); zi = zi.reshape(nlam, nB)
    ar = ar.reshape(nlam, nB); ai = ai.reshape(nlam, nB)
    if complex_out:
        return zr + 1j * zi
    odd = np.array([parity_E(N, l) < 0 for l in lams], dtype=bool)
    z = np.where(odd[:, None], zi, zr)
    if return_abs:
        return z, np.where(odd[:, None], ai, ar)
    return z


def dmr_weights(w_data, w_rand):
    """Data-minus-randoms weights: w_R <- -w_R * sum(w_D)/sum(w_R) (FP64, exact sums)."""
    w_data = np.asarray(w_data, dtype=np.float64)
    w_rand = np.asarray(w_rand, dtype=np.float64)
    sd = math.fsum(w_data.tolist())
    sr = math.fsum(w_rand.tolist())
    return np.concatenate([w_data, -w_rand * (sd / sr)])


def split_zeta(data_pos, data_w, rand_pos, rand_w, split_sizes, N, lmax, edges, box=None,
               parity="even", nthreads=0):
    """Mean over the random parts of the D-R multiplets, and the per-part values
    [n_parts, n_multiplets, n_bin_tuples] (Section 4.2, random splits co-added)."""
    data_pos = np.asarray(data_pos, dtype=np.float64)
    rand_pos = np.asarray(rand_pos, dtype=np.float64)
    per = []
    o = 0
    for n in split_sizes:
        pos = np.concatenate([data_pos, rand_pos[o:o + n]])
        w = dmr_weights(data_w, rand_w[o:o + n])
        per.append(zeta(pos, w, N, lmax, edges, box=box, parity=parity, nthreads=nthreads))
        o += n
    per = np.array(per)
    return per.mean(axis=0), per


def normalise(Z, N, edges, volume):
    """zeta = Z / (V prod_k v_{b_k}), v_b = 4 pi/3 (r_{b+1}^3 - r_b^3) the bin volume of
    eq. alm-binned-def, 1/V of eq. NPCF-mult-discrete-binned-estimator."""
    edges = np.asarray(edges, dtype=np.float64)
    vb = 4.0 * math.pi / 3.0 * (edges[1:] ** 3 - edges[:-1] ** 3)
    btab = bin_tuples(N, len(edges) - 1)
    scale = np.array([1.0 / (volume * np.prod([vb[b] for b in B])) for B in btab])
    return Z * scale[None, :]


__all__ = ["build", "ylm", "alm", "zeta", "dmr_weights", "normalise", "multiplets",
           "coupling", "coupling_terms", "bin_tuples", "parity_E", "principal",
           "wigner3j", "term_arrays", "nlm", "basis_value"]


def basis_value(N, lam, vecs):
    """P_Lambda(r1^, ..., r_{N-1}^) = sum_M C^Lambda_M prod_k Y_{l_k m_k}(r_k^) (eq. basis-def),
    from the oracle's own C table and Y_lm.  vecs: [N-1, 3]."""
    ls = principal(N, lam)
    lmax = max(ls)
    ys = [ylm(lmax, v) for v in vecs]

    def y(k, l, m):
        v = ys[k][l * (l + 1) // 2 + abs(m)]
        return v if m >= 0 else (-1) ** (m % 2) * np.conj(v)

    from itertools import product as _product
    total = 0.0 + 0.0j
    for M in _product(*[range(-l, l + 1) for l in ls]):
        if sum(M) != 0:
            continue
        c = coupling(N, lam, M)
        if c == 0.0:
            continue
        t = c
        for k in range(N - 1):
            t = t * y(k, ls[k], M[k])
        total += t
    return total
