"""CPU checks of the C ABI: the library loads, exports every declared symbol, and
its host-side tables agree with the oracle and with independent references.
No device compute is called here."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2105_08722_amd import encore

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "encore.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(encore_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = encore.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(encore.SIGNATURES)


def test_version_string():
    assert "gfx950" in encore.version()


@pytest.mark.parametrize("N,lmax", [(3, 10), (4, 5), (4, 10), (5, 3), (5, 4), (6, 3)])
def test_multiplet_table_matches_oracle(N, lmax):
    for allp in (False, True):
        tab = encore.multiplet_table(N, lmax, allp)
        ref = np.array(oracle.multiplets(N, lmax, "all" if allp else "even"))
        assert tab.shape == ref.shape
        assert np.array_equal(tab, ref)
        assert encore.num_multiplets(N, lmax, allp) == len(ref)


def test_bin_tuple_counts():
    for N in range(3, 7):
        for nb in (0, 1, N - 2, N - 1, 10, 16):
            assert encore.num_bin_tuples(N, nb) == len(oracle.bin_tuples(N, nb))


def test_wigner3j_matches_sympy():
    from sympy.physics.wigner import wigner_3j
    rng = np.random.default_rng(3)
    n = 0
    while n < 300:
        j1, j2 = rng.integers(0, 12, 2)
        j3 = int(rng.integers(abs(j1 - j2), j1 + j2 + 1))
        m1 = int(rng.integers(-j1, j1 + 1)); m2 = int(rng.integers(-j2, j2 + 1)); m3 = -m1 - m2
        if abs(m3) > j3:
            continue
        ref = float(wigner_3j(int(j1), int(j2), j3, m1, m2, m3))
        assert encore.wigner3j(int(j1), int(j2), j3, m1, m2, m3) == pytest.approx(ref, abs=1e-14)
        n += 1


def _random_alm(nbins, lmax, rng):
    """a~ with m >= 0 (complex; m = 0 real, as for any real field)."""
    a = rng.normal(size=(nbins, (lmax + 1) * (lmax + 2) // 2)) + 1j * rng.normal(
        size=(nbins, (lmax + 1) * (lmax + 2) // 2))
    for l in range(lmax + 1):
        a[:, l * (l + 1) // 2] = a[:, l * (l + 1) // 2].real
    return a


def _get(a, b, l, m):
    v = a[b, l * (l + 1) // 2 + abs(m)]
    return v if m >= 0 else (-1) ** (m % 2) * np.conj(v)


@pytest.mark.parametrize("N,lmax", [(3, 6), (4, 4), (5, 3), (6, 2)])
def test_half_sum_terms_equal_full_sum(N, lmax):
    """Appendix B: the library's half-sum terms (m_{N-1} >= 0, weight 2 S E C, Re/Im)
    reproduce the oracle's full M sum on coefficients with the conjugation symmetry."""
    rng = np.random.default_rng(10 + N)
    nbins = N
    a = _random_alm(nbins, lmax, rng)
    lam, l, m, coef = encore.coupling_terms(N, lmax, allparity=True)
    lams = oracle.multiplets(N, lmax, "all")
    Btab = oracle.bin_tuples(N, nbins)
    full = np.zeros((len(lams), len(Btab)), dtype=complex)
    t_lam, t_l, t_m, t_c = oracle.term_arrays(N, lmax, "all")
    for t in range(len(t_lam)):
        for bi, B in enumerate(Btab):
            p = t_c[t]
            for k in range(N - 1):
                p = p * _get(a, B[k], t_l[t, k], t_m[t, k])
            full[t_lam[t], bi] += p
    half = np.zeros((len(lams), len(Btab)))
    odd = np.array([oracle.parity_E(N, x) < 0 for x in lams])
    for t in range(len(lam)):
        for bi, B in enumerate(Btab):
            p = 1.0 + 0j
            for k in range(N - 1):
                p = p * _get(a, B[k], l[t, k], m[t, k])
            half[lam[t], bi] += coef[t] * (p.imag if odd[lam[t]] else p.real)
    ref = np.where(odd[:, None], full.imag, full.real)
    assert np.max(np.abs(half - ref)) <= 1e-12 * np.max(np.abs(ref))
    # the other component of the full sum vanishes
    other = np.where(odd[:, None], full.real, full.imag)
    assert np.max(np.abs(other)) <= 1e-12 * np.max(np.abs(ref))


def test_paper_gpu_b_task_count_from_library_terms():
    """135,120 GPU-b tasks for the 4PCF at lmax = 5 (Section 5.3): nonzero half-sum
    terms times 120 bin triples."""
    lam, l, m, coef = encore.coupling_terms(4, 5)
    assert len(coef) * encore.num_bin_tuples(4, 10) == 135120
    assert np.all(m[:, -1] >= 0)


def test_host_argument_errors():
    with pytest.raises(encore.EncoreError) as e:
        encore.num_multiplets(7, 2)
    assert e.value.code == encore.EINVAL
    with pytest.raises(encore.EncoreError):
        encore.num_multiplets(5, 6)
    with pytest.raises(encore.EncoreError) as e:
        encore.lib().encore_multiplet_table(4, 5, 0, None, 0) and encore._check(
            encore.lib().encore_multiplet_table(4, 5, 0, None, 0))
    assert e.value.code == encore.ESIZE
    assert "needs" in str(e.value)


def test_split_grids_refuse_bad_sizes():
    """build_split_grids checks the part sizes before touching the device."""
    rng = np.random.default_rng(0)
    d, r = rng.uniform(0, 10, (5, 3)), rng.uniform(0, 10, (9, 3))
    for sizes in ([4, 4], [9, 0], [10], [-1, 10]):
        with pytest.raises(ValueError):
            encore.build_split_grids(None, d, np.ones(5), r, np.ones(9), sizes, 2.0)
