"""Edge correction on the device (through the C ABI) against the FP64 oracle.

Tolerance: the device builds the coupling matrix from the same generalized Gaunt
integrals (closed forms of Appendix A, evaluated independently in long double on
the host) and solves the per-B systems in FP64 by Gaussian elimination with
partial pivoting and back substitution; the oracle uses numpy's LU solve.  The matrices are close to
(4 pi)^{-(N-1)/2} times the identity (condition numbers of order one), so both
results agree to rounding: bound 1e-11 relative to max|zeta| and 1e-12 relative to
max|M| for the matrices.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import edge as oedge
from paper_2105_08722_amd import encore, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-edge] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = encore.Context(0)
    yield c
    c.close()


def _window_multiplets(N, lmax, nB, parity, seed):
    """Synthetic multiplets: R_0 dominant with few-per-cent higher multiplets."""
    rng = np.random.default_rng(seed)
    n = len(oracle.multiplets(N, lmax, parity))
    R = rng.normal(0.0, 0.03, (n, nB)) * rng.uniform(0.5, 2.0, nB)[None, :]
    R[0] = rng.uniform(1.0, 3.0, nB)
    Nm = rng.normal(0.0, 1.0, (n, nB))
    return Nm, R


@pytest.mark.parametrize("N,lmax,nbins,allp", [(3, 4, 4, False), (3, 3, 4, True), (4, 3, 5, False),
                                               (4, 2, 4, True), (5, 2, 5, False), (5, 1, 5, True),
                                               (6, 1, 6, False), (6, 1, 6, True)])
def test_edge_matches_oracle(ctx, N, lmax, nbins, allp):
    _say("edge correction N=%d lmax=%d nbins=%d allparity=%s" % (N, lmax, nbins, allp))
    parity = "all" if allp else "even"
    nB = encore.num_bin_tuples(N, nbins)
    Nm, R = _window_multiplets(N, lmax, nB, parity, 10 * N + lmax)
    z, M, bad = encore.edge_correct(ctx, N, lmax, nbins, Nm, R, allparity=allp, return_coupling=True)
    Mo = oedge.coupling_matrix(N, lmax, R, parity)
    zo = oedge.edge_correct(N, lmax, Nm, R, parity)
    assert bad == 0
    assert np.max(np.abs(M - Mo)) <= 1e-12 * np.max(np.abs(Mo))
    assert np.max(np.abs(z - zo)) <= 1e-11 * np.max(np.abs(zo))
    # lmax_out: the lower multiplets of the same solution
    if lmax > 0:
        z1 = encore.edge_correct(ctx, N, lmax, nbins, Nm, R, allparity=allp, lmax_out=lmax - 1)
        zo1 = oedge.edge_correct(N, lmax, Nm, R, parity, lmax_out=lmax - 1)
        assert z1.shape == zo1.shape
        assert np.max(np.abs(z1 - zo1)) <= 1e-11 * np.max(np.abs(zo1))


def test_edge_periodic_window_is_scaled_identity(ctx):
    """R with only R_0 (uniform periodic geometry, eq. R-periodic-form): M is
    (4 pi)^{-(N-1)/2} times the identity and zeta = (4 pi)^{(N-1)/2} N / R_0."""
    _say("edge correction, periodic window")
    N, lmax, nbins = 4, 3, 5
    nB = encore.num_bin_tuples(N, nbins)
    n = encore.num_multiplets(N, lmax)
    rng = np.random.default_rng(2)
    R = np.zeros((n, nB))
    R[0] = rng.uniform(1.0, 2.0, nB)
    Nm = rng.normal(size=(n, nB))
    z, M, bad = encore.edge_correct(ctx, N, lmax, nbins, Nm, R, return_coupling=True)
    c = (4 * np.pi) ** (-(N - 1) / 2)
    assert bad == 0
    assert np.max(np.abs(M - c * np.eye(n)[None])) <= 1e-15
    assert np.max(np.abs(z - Nm / R[0][None, :] / c)) <= 1e-12 * np.max(np.abs(z))


def test_edge_singular_bins_and_errors(ctx):
    """B with R_0 = 0 get NaN and are counted; the others are solved; systems of
    more than 4096 multiplets and short buffers are refused."""
    _say("edge correction, singular bins and errors")
    N, lmax, nbins = 3, 3, 4
    nB = encore.num_bin_tuples(N, nbins)
    Nm, R = _window_multiplets(N, lmax, nB, "even", 7)
    R[0, 2] = 0.0
    z, _, bad = encore.edge_correct(ctx, N, lmax, nbins, Nm, R, return_coupling=True)
    assert bad == 1
    assert np.all(np.isnan(z[:, 2]))
    ok = [b for b in range(nB) if b != 2]
    zo = oedge.edge_correct(N, lmax, Nm[:, ok], R[:, ok])
    assert np.max(np.abs(z[:, ok] - zo)) <= 1e-11 * np.max(np.abs(zo))
    with pytest.raises(encore.EncoreError) as e:
        n6 = encore.num_multiplets(6, 4)          # 10113 multiplets
        nB6 = encore.num_bin_tuples(6, 6)
        encore.edge_correct(ctx, 6, 4, 6, np.ones((n6, nB6)), np.ones((n6, nB6)))
    assert e.value.code == encore.EUNSUPPORTED


def test_edge_end_to_end_survey_window(ctx):
    """Multiplets measured by the library on a non-periodic window (randoms in a
    cube, a clustered catalog minus randoms), then edge-corrected on the device and
    by the oracle from the same multiplets."""
    _say("edge correction end to end (cube window)")
    N, lmax, nbins = 4, 3, 4
    L = 120.0
    rng = np.random.default_rng(11)
    dpos, _ = synth.neyman_scott(900, L, 12, nbar_parent=5e-5, sigma=3.0)
    rpos = rng.uniform(0.0, L, (2700, 3))
    edges = np.linspace(8.0, 40.0, nbins + 1)
    pos = np.concatenate([dpos, rpos])
    w = np.ones(len(pos))
    with encore.build_grid(ctx, rpos, np.ones(len(rpos)), r_max=edges[-1]) as g:
        R = encore.npcf(ctx, g, N, lmax, edges, precision="fp64")
    with encore.build_grid(ctx, pos, w, r_max=edges[-1], n_data=len(dpos)) as g:
        Nm = encore.npcf(ctx, g, N, lmax, edges, precision="fp64")
    z, M, bad = encore.edge_correct(ctx, N, lmax, nbins, Nm, R, lmax_out=lmax - 1, return_coupling=True)
    zo = oedge.edge_correct(N, lmax, Nm, R, lmax_out=lmax - 1)
    Mo = oedge.coupling_matrix(N, lmax, R)
    assert bad == 0
    assert np.max(np.abs(M - Mo)) <= 1e-12 * np.max(np.abs(Mo))
    assert np.max(np.abs(z - zo)) <= 1e-11 * np.max(np.abs(zo))
    # the window couples multiplets: M is not the periodic scaled identity
    n = M.shape[1]
    assert np.max(np.abs(M - (4 * np.pi) ** -1.5 * np.eye(n)[None])) > 1e-4


def test_edge_timings(ctx):
    """After an edge correction the timing slots hold its device time alone."""
    _say("edge correction timings")
    N, lmax, nbins = 4, 2, 4
    nB = encore.num_bin_tuples(N, nbins)
    Nm, R = _window_multiplets(N, lmax, nB, "even", 3)
    encore.edge_correct(ctx, N, lmax, nbins, Nm, R)
    t = ctx.last_timings()
    assert t["total_ms"] > 0.0
    assert t["gather_ms"] == 0.0 and t["couple_ms"] == 0.0 and t["contract_ms"] == 0.0
    assert t["batches"] == 0 and t["pairs"] == 0


@pytest.mark.parametrize("strong", [False, True])
def test_edge_blocked_solve_many_panels(ctx, strong):
    """The blocked LU on systems of 585 multiplets (5PCF, lmax 4: 19 panels of 32
    columns, trailing updates over several 128 x 128 tiles), against numpy's LU solve
    of the device's own coupling matrices (the Gaunt terms are pinned separately
    against the oracle).  A mild window (R_0 dominant) and a strong one (every R_L of
    order R_0, so that the matrices are far from diagonal and the pivoting exchanges
    rows)."""
    N, lmax, nbins = 5, 4, 6
    _say("edge blocked solve N=%d lmax=%d strong=%s" % (N, lmax, strong))
    nB = encore.num_bin_tuples(N, nbins)
    n = encore.num_multiplets(N, lmax)
    rng = np.random.default_rng(11 + strong)
    R = rng.normal(0.0, 1.0 if strong else 0.03, (n, nB))
    R[0] = rng.uniform(1.0, 3.0, nB)
    Nm = rng.normal(0.0, 1.0, (n, nB))
    z, M, bad = encore.edge_correct(ctx, N, lmax, nbins, Nm, R, return_coupling=True)
    assert bad == 0
    for b in range(nB):
        A = M[b].T                                   # eq. edge-correction-matrix: sum_L zeta_L M[L][L'']
        zr = np.linalg.solve(A, Nm[:, b] / R[0, b])
        # two backward-stable solvers agree to ~cond(A) * eps
        cond = np.linalg.cond(A)
        if strong and b == 0:
            _say("  cond of the first matrix: %.1e" % cond)
        assert np.max(np.abs(z[:, b] - zr)) <= 1e-13 * cond * np.max(np.abs(zr))
