"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each uses a closed form, a
printed value, an independent library routine, an identity of the basis, or an
explicit tuple sum.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import basis
from oracle.brute import brute_zeta

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


def _small_catalog(n, seed, L=10.0):
    rng = _rng(seed)
    return rng.uniform(0.0, L, (n, 3)), rng.uniform(0.5, 1.5, n)


# ---------------------------------------------------------------- building blocks

def test_wigner3j_matches_sympy():
    from sympy.physics.wigner import wigner_3j
    rng = _rng(7)
    checked = 0
    while checked < 300:
        j1, j2 = rng.integers(0, 9, 2)
        j3 = rng.integers(abs(j1 - j2), j1 + j2 + 1)
        m1 = rng.integers(-j1, j1 + 1)
        m2 = rng.integers(-j2, j2 + 1)
        m3 = -m1 - m2
        if abs(m3) > j3:
            continue
        ref = float(wigner_3j(int(j1), int(j2), int(j3), int(m1), int(m2), int(m3)))
        got = oracle.wigner3j(int(j1), int(j2), int(j3), int(m1), int(m2), int(m3))
        assert got == pytest.approx(ref, abs=1e-15, rel=1e-14)
        checked += 1
    # selection rules
    assert oracle.wigner3j(1, 1, 3, 0, 0, 0) == 0.0
    assert oracle.wigner3j(1, 1, 1, 0, 0, 0) == 0.0      # odd sum with all m = 0
    assert oracle.wigner3j(2, 2, 2, 1, 1, -1) == 0.0     # sum m != 0


def test_ylm_matches_scipy_condon_shortley():
    from scipy.special import sph_harm_y
    rng = _rng(11)
    for _ in range(50):
        d = rng.normal(size=3) * rng.uniform(0.1, 100)
        y = oracle.ylm(10, d)
        r = np.linalg.norm(d)
        th = math.acos(d[2] / r)
        ph = math.atan2(d[1], d[0])
        for l in range(11):
            for m in range(l + 1):
                ref = sph_harm_y(l, m, th, ph)
                assert abs(y[l * (l + 1) // 2 + m] - ref) < 1e-13
    # poles: only m = 0 survives
    y = oracle.ylm(6, [0.0, 0.0, -3.0])
    for l in range(7):
        assert abs(y[l * (l + 1) // 2] - (-1) ** l * math.sqrt((2 * l + 1) / (4 * math.pi))) < 1e-14
        for m in range(1, l + 1):
            assert abs(y[l * (l + 1) // 2 + m]) < 1e-15


def test_p110_printed_cartesian_form():
    g = json.load(open(os.path.join(GOLDEN, "p110.json")))
    rng = _rng(3)
    for _ in range(20):
        v = rng.normal(size=(3, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        got = oracle.basis_value(g["N"], tuple(g["multiplet"]), v)
        want = g["coefficient_of_dot_r1_r2"] * float(v[0] @ v[1])
        assert abs(got.imag) < 1e-15
        assert got.real == pytest.approx(want, abs=1e-15)


def test_p0_constant_all_N():
    rng = _rng(5)
    for N in (3, 4, 5, 6):
        v = rng.normal(size=(N - 1, 3))
        lam = basis.multiplets(N, 0)[0]
        assert all(l == 0 for l in lam)
        got = oracle.basis_value(N, lam, v)
        assert got.real == pytest.approx((4 * math.pi) ** (-(N - 1) / 2), rel=1e-14)


def test_coupling_orthonormal_and_conjugation():
    """sum_M C^L_M C^L'_M = delta (orthonormality of the basis, since the Y_lm are
    orthonormal) and C_{-M} = E C_M."""
    for N, lmax in ((3, 6), (4, 4), (5, 3), (6, 2)):
        lams = basis.multiplets(N, lmax, "all")
        tabs = {}
        for lam in lams:
            ls = basis.principal(N, lam)
            tab = {}
            for M in itertools.product(*[range(-l, l + 1) for l in ls]):
                if sum(M) == 0:
                    c = basis.coupling(N, lam, M)
                    if c != 0.0:
                        tab[M] = c
            tabs[lam] = tab
            E = basis.parity_E(N, lam)
            for M, c in tab.items():
                neg = tuple(-m for m in M)
                assert tab.get(neg, 0.0) == pytest.approx(E * c, abs=1e-15)
        by_principal = {}
        for lam in lams:
            by_principal.setdefault(basis.principal(N, lam), []).append(lam)
        for group in by_principal.values():
            for a in group:
                for b in group:
                    s = sum(c * tabs[b].get(M, 0.0) for M, c in tabs[a].items())
                    assert s == pytest.approx(1.0 if a == b else 0.0, abs=1e-13)


def test_paper_task_counts():
    g = json.load(open(os.path.join(GOLDEN, "paper_counts.json")))
    nb = g["nbins"]
    for row in g["gpu_a"]:
        nlam = len(oracle.multiplets(row["N"], row["lmax"], "even"))
        nB = len(oracle.bin_tuples(row["N"], nb))
        assert nlam * nB == row["tasks"]
    for row in g["gpu_b"]:
        if row["N"] == 5:
            continue  # covered (slow) below
        terms = oracle.coupling_terms(row["N"], row["lmax"], "even")
        half = sum(1 for t in terms if t[2][-1] >= 0)
        assert half * len(oracle.bin_tuples(row["N"], nb)) == row["tasks"]


@pytest.mark.slow
def test_paper_task_counts_5pcf():
    g = json.load(open(os.path.join(GOLDEN, "paper_counts.json")))
    for row in g["gpu_b"]:
        if row["N"] != 5:
            continue
        terms = oracle.coupling_terms(row["N"], row["lmax"], "even")
        half = sum(1 for t in terms if t[2][-1] >= 0)
        assert half * len(oracle.bin_tuples(row["N"], g["nbins"])) == row["tasks"]


# ---------------------------------------------------------------- the estimator

@pytest.mark.parametrize("N,lmax,nbins,npts", [(3, 4, 4, 16), (4, 3, 4, 16), (5, 2, 5, 14),
                                               (6, 1, 6, 13)])
def test_factorised_equals_brute_force(N, lmax, nbins, npts):
    pos, w = _small_catalog(npts, 100 + N)
    edges = np.linspace(0.8, 9.0, nbins + 1)
    for parity in ("even", "all"):
        if N == 3 and parity == "all":
            continue
        z = oracle.zeta(pos, w, N, lmax, edges, parity=parity)
        zb = brute_zeta(pos, w, N, lmax, edges, parity=parity)
        scale = np.max(np.abs(zb))
        assert scale > 0
        assert np.max(np.abs(z - zb)) <= 1e-12 * scale


def test_brute_force_periodic():
    pos, w = _small_catalog(16, 9, L=8.0)
    edges = np.linspace(0.5, 4.0, 5)
    z = oracle.zeta(pos, w, 4, 2, edges, box=8.0)
    zb = brute_zeta(pos, w, 4, 2, edges, box=8.0)
    assert np.max(np.abs(z - zb)) <= 1e-12 * np.max(np.abs(zb))


def _dirs(pos, i, box):
    d = pos - pos[i]
    if box is not None:
        d = d - box * np.round(d / box)
    r = np.sqrt(np.sum(d * d, axis=1))
    return d, r


def test_3pcf_legendre_closed_form():
    """Z^{b1 b2}_l = (-1)^l sqrt(2l+1)/(4 pi) sum_i w_i sum_{j in b1, k in b2} w_j w_k
    L_l(d_ij^ . d_ik^), from eq. N=3-basis inserted in the discrete estimator."""
    from scipy.special import eval_legendre
    rng = _rng(21)
    n, L = 120, 100.0
    pos = rng.uniform(0, L, (n, 3)); w = rng.uniform(-1, 1.5, n)
    edges = np.linspace(5.0, 40.0, 6)
    lmax = 6
    z = oracle.zeta(pos, w, 3, lmax, edges, box=L)
    Btab = oracle.bin_tuples(3, 5)
    ref = np.zeros_like(z)
    for i in range(n):
        d, r = _dirs(pos, i, L)
        u = d / np.where(r > 0, r, 1)[:, None]
        b = np.searchsorted(edges, r, side="right") - 1
        b[(r < edges[0]) | (r >= edges[-1])] = -1
        b[i] = -1
        for bi, (b1, b2) in enumerate(Btab):
            s1 = np.nonzero(b == b1)[0]; s2 = np.nonzero(b == b2)[0]
            if len(s1) == 0 or len(s2) == 0:
                continue
            mu = u[s1] @ u[s2].T
            ww = np.outer(w[s1], w[s2])
            for l in range(lmax + 1):
                ref[l, bi] += w[i] * (-1) ** l * math.sqrt(2 * l + 1) / (4 * math.pi) * np.sum(
                    ww * eval_legendre(l, mu))
    assert np.max(np.abs(z - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_4pcf_legendre_limits():
    """Lambda = (0,l,l), (l,0,l), (l,l,0) reduce to Y_00 times the N=3 Legendre form."""
    from scipy.special import eval_legendre
    rng = _rng(22)
    n, L = 60, 60.0
    pos = rng.uniform(0, L, (n, 3)); w = rng.uniform(0.2, 1.2, n)
    edges = np.linspace(4.0, 28.0, 5)
    lmax = 3
    lams = oracle.multiplets(4, lmax)
    z = oracle.zeta(pos, w, 4, lmax, edges, box=L)
    Btab = oracle.bin_tuples(4, 4)
    for i_lam, lam in enumerate(lams):
        if 0 not in lam:
            continue
        zero = lam.index(0)
        l = max(lam)
        ref = np.zeros(len(Btab))
        for i in range(n):
            d, r = _dirs(pos, i, L)
            u = d / np.where(r > 0, r, 1)[:, None]
            b = np.searchsorted(edges, r, side="right") - 1
            b[(r < edges[0]) | (r >= edges[-1])] = -1
            b[i] = -1
            for bi, B in enumerate(Btab):
                others = [B[k] for k in range(3) if k != zero]
                s0 = np.nonzero(b == B[zero])[0]
                s1 = np.nonzero(b == others[0])[0]
                s2 = np.nonzero(b == others[1])[0]
                if min(len(s0), len(s1), len(s2)) == 0:
                    continue
                mu = u[s1] @ u[s2].T
                ref[bi] += (w[i] * np.sum(w[s0]) * (-1) ** l * math.sqrt(2 * l + 1)
                            / (4 * math.pi) ** 1.5 * np.sum(np.outer(w[s1], w[s2]) * eval_legendre(l, mu)))
        scale = max(np.max(np.abs(ref)), 1e-300)
        assert np.max(np.abs(z[i_lam] - ref)) <= 1e-12 * scale, lam


@pytest.mark.parametrize("N", [3, 4, 5, 6])
def test_monopole_pair_count_closed_form(N):
    """Z_0^B = (4 pi)^{-(N-1)/2} sum_i w_i prod_k (sum_{j in b_k} w_j)  (P_0 constant)."""
    rng = _rng(30 + N)
    n, L = 80, 50.0
    pos = rng.uniform(0, L, (n, 3)); w = rng.uniform(-1.0, 1.0, n)
    nb = N + 1
    edges = np.linspace(3.0, 24.0, nb + 1)
    z = oracle.zeta(pos, w, N, 1, edges, box=L)
    lam0 = oracle.multiplets(N, 1).index(tuple([0] * len(oracle.multiplets(N, 1)[0])))
    ref = np.zeros(z.shape[1])
    for i in range(n):
        d, r = _dirs(pos, i, L)
        S = np.zeros(nb)
        for b in range(nb):
            sel = (r >= edges[b]) & (r < edges[b + 1])
            sel[i] = False
            S[b] = np.sum(w[sel])
        for bi, B in enumerate(oracle.bin_tuples(N, nb)):
            ref[bi] += w[i] * np.prod(S[list(B)])
    ref *= (4 * math.pi) ** (-(N - 1) / 2)
    assert np.max(np.abs(z[lam0] - ref)) <= 1e-12 * np.max(np.abs(ref))


def _rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a*a+b*b-c*c-d*d, 2*(b*c-a*d), 2*(b*d+a*c)],
                     [2*(b*c+a*d), a*a-b*b+c*c-d*d, 2*(c*d-a*b)],
                     [2*(b*d-a*c), 2*(c*d+a*b), a*a-b*b-c*c+d*d]])


@pytest.mark.parametrize("N,lmax", [(4, 3), (5, 2), (6, 1)])
def test_rotation_invariance(N, lmax):
    rng = _rng(40 + N)
    pos = rng.normal(0, 8.0, (70, 3)); w = rng.uniform(-1, 1, 70)
    edges = np.linspace(2.0, 14.0, N + 1)
    z = oracle.zeta(pos, w, N, lmax, edges, parity="all")
    R = _rotation(rng)
    zr = oracle.zeta(pos @ R.T, w, N, lmax, edges, parity="all")
    assert np.max(np.abs(z - zr)) <= 1e-11 * np.max(np.abs(z))


@pytest.mark.parametrize("N,lmax", [(4, 3), (5, 2)])
def test_reflection_multiplies_by_E(N, lmax):
    rng = _rng(50 + N)
    pos = rng.normal(0, 8.0, (60, 3)); w = rng.uniform(-1, 1, 60)
    edges = np.linspace(2.0, 14.0, N + 1)
    lams = oracle.multiplets(N, lmax, "all")
    E = np.array([oracle.parity_E(N, l) for l in lams], dtype=float)
    z = oracle.zeta(pos, w, N, lmax, edges, parity="all")
    zr = oracle.zeta(-pos, w, N, lmax, edges, parity="all")
    assert np.max(np.abs(zr - E[:, None] * z)) <= 1e-11 * np.max(np.abs(z))
    assert np.max(np.abs(z[E < 0])) > 1e-6 * np.max(np.abs(z))   # odd part is non-trivial


def test_even_multiplets_are_real_odd_imaginary():
    pos, w = _small_catalog(40, 60, L=20.0)
    edges = np.linspace(1.0, 10.0, 5)
    zc = oracle.zeta(pos, w, 4, 3, edges, parity="all", complex_out=True)
    lams = oracle.multiplets(4, 3, "all")
    scale = np.max(np.abs(zc))
    for li, lam in enumerate(lams):
        if oracle.parity_E(4, lam) > 0:
            assert np.max(np.abs(zc[li].imag)) <= 1e-13 * scale
        else:
            assert np.max(np.abs(zc[li].real)) <= 1e-13 * scale


def test_weight_homogeneity_and_order_invariance():
    pos, w = _small_catalog(50, 70, L=20.0)
    edges = np.linspace(1.0, 10.0, 5)
    z = oracle.zeta(pos, w, 4, 2, edges)
    z2 = oracle.zeta(pos, 2.5 * w, 4, 2, edges)
    assert np.max(np.abs(z2 - 2.5 ** 4 * z)) <= 1e-12 * np.max(np.abs(z2))
    perm = _rng(71).permutation(len(w))
    zp = oracle.zeta(pos[perm], w[perm], 4, 2, edges)
    assert np.max(np.abs(zp - z)) <= 1e-12 * np.max(np.abs(z))


def test_periodic_translation_invariance():
    rng = _rng(80)
    L = 30.0
    pos = rng.uniform(0, L, (60, 3)); w = rng.uniform(-1, 1, 60)
    edges = np.linspace(2.0, 14.0, 5)
    z = oracle.zeta(pos, w, 4, 2, edges, box=L)
    shifted = np.mod(pos + np.array([11.3, -4.2, 25.9]), L)
    zs = oracle.zeta(shifted, w, 4, 2, edges, box=L)
    assert np.max(np.abs(zs - z)) <= 1e-10 * np.max(np.abs(z))


def test_dmr_weights_sum_to_zero():
    rng = _rng(90)
    wd = rng.uniform(0.5, 1.5, 1000); wr = rng.uniform(0.5, 1.5, 3000)
    w = oracle.dmr_weights(wd, wr)
    assert abs(math.fsum(w.tolist())) < 1e-10
    assert np.all(w[1000:] < 0)


def test_alm_definition_single_pair():
    """One secondary: a~^b_lm = w_j Y_lm of the separation (secondary minus primary)."""
    pos = np.array([[1.0, 2.0, 3.0], [4.0, -1.0, 7.0]])
    w = np.array([0.7, -1.3])
    edges = np.array([1.0, 5.0, 9.0])
    a = oracle.alm(pos, w, 4, edges, primaries=[0])
    d = pos[1] - pos[0]
    b = 1 if np.linalg.norm(d) >= 5.0 else 0
    assert np.allclose(a[0, b], -1.3 * oracle.ylm(4, d), atol=1e-15)
    assert np.all(a[0, 1 - b] == 0)
