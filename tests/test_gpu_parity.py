"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (tests/parity_bars.py)
  * FP64 path: the device uses the same FP64 bin decisions as the oracle and FP64
    arithmetic throughout; differences are rounding-order only: 1e-10 of max|Z|.
  * FP32 path: FP32 unit vectors and Y_lm from FP64 separations, each FP32 term
    added into FP64 per-lane accumulators reduced across lanes in FP64, FP32
    coupling products, FP64 sums over primaries.  Split-BF16 path: the FP32 gather
    with FP32 sums, then
    coupling products on the matrix cores with both operands split into bf16
    hi + lo and hi*hi + hi*lo + lo*hi summed in FP32 (flushed into FP64 every 256
    primaries); each product carries at most 3 * 2^-18 = 1.1e-5 of its magnitude.
    For both, every multiplet meets e_L <= u max(kappa_L, 1) + u with u = 1e-6
    (FP32) and 1e-5 (split-BF16), kappa_L the conditioning of the sum over primaries.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
import parity_bars as bars
from paper_2105_08722_amd import encore, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-parity] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = encore.Context(0)
    yield c
    c.close()


def _normwise(zg, zo):
    """Per-multiplet ||zg - zo|| / ||zo|| (multiplets with ||zo|| below 1e-9 max are skipped)."""
    num = np.linalg.norm(zg - zo, axis=1)
    den = np.linalg.norm(zo, axis=1)
    keep = den > 1e-9 * max(den.max(), 1e-300)
    return np.where(keep, num / np.where(keep, den, 1.0), 0.0)


def _uniform(n, L, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, L, (n, 3)), rng.uniform(0.5, 1.5, n)


# ------------------------------------------------------------------ harmonic coefficients

@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("lmax", [0, 3, 5, 10])
def test_alm_fp64_matches_oracle(ctx, periodic, lmax):
    _say("alm fp64 periodic=%s lmax=%d" % (periodic, lmax))
    pos, w = _uniform(3000, 100.0, 7 + lmax)
    edges = np.linspace(4.0, 30.0, 9)
    box = 100.0 if periodic else None
    prim = np.random.default_rng(1).choice(len(w), 40, replace=False)
    with encore.build_grid(ctx, pos, w, r_max=edges[-1], box=box) as g:
        ag = encore.debug_alm(ctx, g, lmax, edges, prim, "fp64")
    ao = oracle.alm(pos, w, lmax, edges, box=box, primaries=prim)
    scale = np.max(np.abs(ao))
    assert np.max(np.abs(ag - ao)) <= 1e-12 * scale


@pytest.mark.parametrize("lmax", [2, 5, 8])
def test_alm_fp32_matches_oracle(ctx, lmax):
    _say("alm fp32 lmax=%d" % lmax)
    pos, w = _uniform(3000, 100.0, 17)
    edges = np.linspace(4.0, 30.0, 11)
    prim = np.arange(0, 3000, 97)
    with encore.build_grid(ctx, pos, w, r_max=edges[-1], box=100.0) as g:
        ag = encore.debug_alm(ctx, g, lmax, edges, prim, "fp32")
    ao = oracle.alm(pos, w, lmax, edges, box=100.0, primaries=prim)
    for i in range(len(prim)):
        assert np.max(np.abs(ag[i] - ao[i])) <= 1e-6 * np.max(np.abs(ao[i]))


def test_alm_clustered_nonperiodic_offset_box(ctx):
    """Clustered points, non-periodic, far from the origin; one edge set reaching
    beyond the catalog (empty bins) and primaries at the corners."""
    _say("alm clustered non-periodic")
    pos, w = synth.neyman_scott(4000, 200.0, 5, nbar_parent=5e-5, sigma=3.0)
    pos = pos + np.array([1000.0, -5000.0, 250.0])
    w = w * np.random.default_rng(2).uniform(-1, 1, len(w))
    edges = np.array([1.0, 3.0, 7.0, 15.0, 40.0, 90.0])
    corner = [int(np.argmin(pos.sum(1))), int(np.argmax(pos.sum(1)))]
    prim = np.array(corner + list(range(0, 4000, 211)))
    with encore.build_grid(ctx, pos, w, r_max=edges[-1]) as g:
        ag = encore.debug_alm(ctx, g, 4, edges, prim, "fp64")
    ao = oracle.alm(pos, w, 4, edges, primaries=prim)
    assert np.max(np.abs(ag - ao)) <= 1e-12 * np.max(np.abs(ao))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_alm_chunk_boundaries(ctx, precision):
    """Catalogs on one cell row, every point within r_max of every other: each
    primary's candidates are exactly the n points, so n = 63, 64, 65, 127, 128, 129
    and 192 put the end of the candidate walk one short of, on, and one past a
    64-candidate chunk (and the prefetched chunk past the end)."""
    _say("alm chunk boundaries %s" % precision)
    rng = np.random.default_rng(11)
    edges = np.array([0.1, 35.0, 70.0])
    for n in [1, 2, 63, 64, 65, 127, 128, 129, 192]:
        pos = np.zeros((n, 3))
        pos[:, 0] = 0.5 + 0.3 * np.arange(n)
        pos[:, 1:] = 0.3 + rng.uniform(-0.2, 0.2, (n, 2))
        w = rng.uniform(0.5, 1.5, n)
        prim = np.arange(n)
        with encore.build_grid(ctx, pos, w, r_max=edges[-1]) as g:
            ag = encore.debug_alm(ctx, g, 3, edges, prim, precision)
        ao = oracle.alm(pos, w, 3, edges, primaries=prim)
        if n == 1:
            assert np.all(ag == 0) and np.all(ao == 0)
            continue
        bar = 1e-12 if precision == "fp64" else 1e-6
        for i in range(n):
            assert np.max(np.abs(ag[i] - ao[i])) <= bar * np.max(np.abs(ao[i])), (n, i)


# ------------------------------------------------------------------ multiplets

CASES = [
    # N, lmax, npts, nbins, periodic, allparity
    (3, 6, 1500, 7, True, False),
    (4, 3, 1200, 6, True, False),
    (4, 3, 900, 5, False, True),
    (5, 2, 800, 5, True, False),
    (5, 2, 500, 5, False, True),
    (6, 1, 500, 6, True, False),
    (6, 2, 400, 5, False, False),
]


@pytest.mark.parametrize("N,lmax,npts,nbins,periodic,allp", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32", "splitbf16"])
def test_zeta_matches_oracle(ctx, N, lmax, npts, nbins, periodic, allp, precision):
    _say("zeta N=%d lmax=%d n=%d nb=%d periodic=%s allparity=%s %s"
         % (N, lmax, npts, nbins, periodic, allp, precision))
    L = 60.0
    pos, w = _uniform(npts, L, 100 * N + lmax)
    edges = np.linspace(3.0, 25.0, nbins + 1)
    box = L if periodic else None
    with encore.build_grid(ctx, pos, w, r_max=edges[-1], box=box) as g:
        zg = encore.npcf(ctx, g, N, lmax, edges, precision=precision, allparity=allp)
    zo, za = oracle.zeta(pos, w, N, lmax, edges, box=box, parity="all" if allp else "even",
                         return_abs=True)
    assert zg.shape == zo.shape
    e, r = bars.check(zg, zo, za, precision, "zeta")
    _say("  max e_L = %.2e, max e_L/(kappa+1) = %.2e" % (e, r))
    if precision == "fp64":
        assert np.max(_normwise(zg, zo)) <= 1e-9


@pytest.mark.parametrize("N,lmax,nbins,npts", [(3, 0, 1, 37), (3, 1, 2, 300), (4, 0, 3, 1), (4, 1, 3, 17)])
def test_splitbf16_smallest_blocks(ctx, N, lmax, nbins, npts):
    """Split-bf16 with the fewest coefficients per primary (one 16-row block holds
    fewer entries than its weight slots) and row counts that leave a partial last
    block: equal to the oracle to the split-bf16 bar."""
    _say("split-bf16 small blocks N=%d lmax=%d nbins=%d n=%d" % (N, lmax, nbins, npts))
    L = 40.0
    pos, w = _uniform(npts, L, 7 * N + lmax + nbins)
    edges = np.linspace(4.0, 19.0, nbins + 1)
    with encore.build_grid(ctx, pos, w, r_max=edges[-1], box=L) as g:
        zg = encore.npcf(ctx, g, N, lmax, edges, precision="splitbf16")
    zo, za = oracle.zeta(pos, w, N, lmax, edges, box=L, return_abs=True)
    assert zg.shape == zo.shape
    bars.check(zg, zo, za, "splitbf16", "small blocks")


def test_dmr_weights_and_subset(ctx):
    _say("D-R weighting + primary subset")
    rng = np.random.default_rng(44)
    L = 80.0
    dpos, _ = synth.neyman_scott(700, L, 9, nbar_parent=2e-4, sigma=2.0)
    rpos = rng.uniform(0, L, (1400, 3))
    pos = np.concatenate([dpos, rpos])
    w_in = np.concatenate([np.ones(700), rng.uniform(0.8, 1.2, 1400)])
    w = oracle.dmr_weights(w_in[:700], w_in[700:])
    edges = np.linspace(4.0, 30.0, 7)
    subset = rng.choice(len(w), 300, replace=False)
    with encore.build_grid(ctx, pos, w_in, r_max=edges[-1], box=L, n_data=700) as g:
        zg = encore.npcf(ctx, g, 4, 3, edges, precision="fp64", primaries=subset)
        zg_all = encore.npcf(ctx, g, 4, 3, edges, precision="fp64")
        rest = np.setdiff1d(np.arange(len(w)), subset)
        zg_rest = encore.npcf(ctx, g, 4, 3, edges, precision="fp64", primaries=rest)
    zo = oracle.zeta(pos, w, 4, 3, edges, box=L, primaries=subset)
    assert np.max(np.abs(zg - zo)) <= 1e-10 * np.max(np.abs(zo))
    # linearity in the primaries: Z(all) = Z(S) + Z(complement)
    assert np.max(np.abs(zg_all - zg - zg_rest)) <= 1e-10 * np.max(np.abs(zg_all))


def test_normalize_flag(ctx):
    _say("normalize")
    pos, w = _uniform(600, 50.0, 5)
    edges = np.linspace(3.0, 20.0, 5)
    with encore.build_grid(ctx, pos, w, r_max=edges[-1], box=50.0) as g:
        zn = encore.npcf(ctx, g, 4, 2, edges, precision="fp64", normalize=True)
        zr = encore.npcf(ctx, g, 4, 2, edges, precision="fp64")
    ref = oracle.normalise(zr, 4, edges, 50.0 ** 3)
    assert np.max(np.abs(zn - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_degenerate_inputs(ctx):
    _say("degenerate inputs")
    pos, w = _uniform(200, 30.0, 3)
    edges = np.linspace(2.0, 10.0, 3)          # 2 bins
    with encore.build_grid(ctx, pos, w, r_max=10.0, box=30.0) as g:
        z = encore.npcf(ctx, g, 5, 2, edges)      # needs 4 bins: no bin tuples
        assert z.shape[1] == 0
        z0 = encore.npcf(ctx, g, 3, 2, edges, primaries=np.array([], dtype=np.int64))
        assert z0.shape == (3, 1) and np.all(z0 == 0)
        with pytest.raises(encore.EncoreError):
            encore.npcf(ctx, g, 3, 2, np.array([2.0, 20.0]))     # beyond r_max
        with pytest.raises(encore.EncoreError):
            encore.npcf(ctx, g, 3, 2, edges, primaries=np.array([5, 200]))  # index out of range
        # the split-bf16 6PCF at lmax 4 with 16 bins has more output tiles than its
        # 32-bit dense index can address
        with pytest.raises(encore.EncoreError) as e:
            encore.npcf(ctx, g, 6, 4, np.linspace(1.0, 10.0, 17), precision="splitbf16")
        assert e.value.code == encore.EUNSUPPORTED
    # one point: no pairs at all
    with encore.build_grid(ctx, np.array([[1.0, 2.0, 3.0]]), np.array([2.0]), r_max=10.0) as g:
        z = encore.npcf(ctx, g, 3, 3, edges, precision="fp64")
        assert np.all(z == 0)
    # a point outside the periodic box is rejected
    bad = pos.copy(); bad[7, 1] = 30.0
    with pytest.raises(encore.EncoreError) as e:
        encore.build_grid(ctx, bad, w, r_max=10.0, box=30.0)
    assert e.value.code == encore.EINVAL
    nan = pos.copy(); nan[3, 0] = np.nan
    with pytest.raises(encore.EncoreError):
        encore.build_grid(ctx, nan, w, r_max=10.0)


def test_device_pointer_grid_matches_host(ctx):
    import torch
    _say("device-pointer grid")
    pos, w = _uniform(900, 40.0, 12)
    edges = np.linspace(2.0, 15.0, 5)
    tp = torch.from_numpy(pos).cuda()
    tw = torch.from_numpy(w).cuda()
    g1 = encore.build_grid_device(ctx, tp, tw, r_max=15.0, box=40.0)
    torch.cuda.synchronize()
    with encore.build_grid(ctx, pos, w, r_max=15.0, box=40.0) as g2:
        z1 = encore.npcf(ctx, g1, 4, 3, edges, precision="fp64")
        z2 = encore.npcf(ctx, g2, 4, 3, edges, precision="fp64")
    g1.free()
    assert np.max(np.abs(z1 - z2)) <= 1e-12 * np.max(np.abs(z2))


@pytest.mark.parametrize("precision", ["fp64", "fp32", "splitbf16"])
def test_graph_plan_replays_match_eager(ctx, precision):
    """encore_plan: the captured graph replayed three times, with eager library
    work and synchronisation between the replays; every replay equals the eager
    encore_npcf result bit for bit (same kernels, same order) and the oracle."""
    _say("graph plan %s" % precision)
    pos, w = _uniform(1500, 60.0, 321)
    edges = np.linspace(3.0, 25.0, 7)
    with encore.build_grid(ctx, pos, w, r_max=edges[-1], box=60.0) as g:
        eager = encore.npcf(ctx, g, 4, 3, edges, precision=precision)
        with encore.Plan(ctx, g, 4, 3, edges, precision=precision) as plan:
            with pytest.raises(encore.EncoreError):
                g.free()                       # the plan holds the grid
            for rep in range(3):
                z = plan.execute()
                assert np.array_equal(z, eager), rep
                other = encore.npcf(ctx, g, 3, 4, edges, precision="fp64")   # eager work between
                assert np.all(np.isfinite(other))
        zn = encore.npcf(ctx, g, 4, 3, edges, precision=precision, normalize=True)
        with encore.Plan(ctx, g, 4, 3, edges, precision=precision, normalize=True) as plan:
            assert np.array_equal(plan.execute(), zn)
            assert np.array_equal(plan.execute(), zn)
    zo, za = oracle.zeta(pos, w, 4, 3, edges, box=60.0, return_abs=True)
    bars.check(eager, zo, za, precision, "graph plan")


def test_autotune_then_parity():
    """encore_autotune on a D-R catalog picks a cell shape and a gather
    bins-per-item value among the compiled ones; grids built and calls made
    afterwards on that context (which use them) still match the oracle."""
    _say("autotune")
    rng = np.random.default_rng(5)
    L = 90.0
    dpos, _ = synth.neyman_scott(2500, L, 19, nbar_parent=2e-4, sigma=2.0)
    rpos = rng.uniform(0, L, (5000, 3))
    pos = np.concatenate([dpos, rpos])
    w_in = np.ones(len(pos))
    w = oracle.dmr_weights(w_in[:2500], w_in[2500:])
    edges = np.linspace(4.0, 30.0, 11)
    with encore.Context(0) as c:
        for prec in ["fp32", "splitbf16"]:
            rep = encore.autotune(c, pos, w_in, 4, 5, edges, box=L, n_data=2500, precision=prec,
                                  n_sample=1000)
            _say("  %s: %s" % (prec, rep))
            assert (rep["cell_divisor"], rep["x_subdivision"]) in [(5, 16), (5, 8), (6, 16), (6, 8), (8, 8), (8, 4), (5, 24), (4, 16)]
            # compiled bins-per-item values at lmax 5: FP32 path (FP64 sums) {2, 1}, split-bf16 {2, 3}
            assert rep["bins_per_item"] in ((2, 1) if prec == "fp32" else (2, 3))
            assert 0 < rep["best_ms"] <= rep["default_ms"]
            prim = rng.choice(len(pos), 200, replace=False)
            with encore.build_grid(c, pos, w_in, r_max=edges[-1], box=L, n_data=2500) as g:
                zg = encore.npcf(c, g, 4, 5, edges, precision=prec, primaries=prim)
            zo, za = oracle.zeta(pos, w, 4, 5, edges, box=L, primaries=prim, return_abs=True)
            bars.check(zg, zo, za, prec, "autotuned")


# ------------------------------------------------------------------ benchmark workloads

def test_config1_3pcf_full(ctx):
    """The 3PCF workload in full: 2000 uniform points, periodic 500 Mpc/h, lmax = 10,
    10 bins over [20, 160], FP64."""
    cfg = synth.config(1)
    _say(cfg["name"])
    with encore.build_grid(ctx, cfg["pos"], cfg["w"], r_max=160.0, box=cfg["box"]) as g:
        zg = encore.npcf(ctx, g, 3, 10, cfg["edges"], precision="fp64")
        zf = encore.npcf(ctx, g, 3, 10, cfg["edges"], precision="fp32")
    zo, za = oracle.zeta(cfg["pos"], cfg["w"], 3, 10, cfg["edges"], box=cfg["box"], return_abs=True)
    bars.check(zg, zo, za, "fp64", "config 1")
    e, r = bars.check(zf, zo, za, "fp32", "config 1")
    _say("  fp32: max e_L = %.2e, max e_L/(kappa+1) = %.2e" % (e, r))


@pytest.fixture(scope="module")
def cfg2():
    return synth.config(2)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config2_alm_full_launch_sampled(ctx, cfg2, precision):
    """Full-size 4PCF workload (200k clustered data + 600k randoms, D-R weights):
    gather over all 800k primaries in one launch, sampled rows vs the oracle."""
    _say("config2 full-launch alm " + precision)
    n = len(cfg2["w"])
    w = oracle.dmr_weights(cfg2["w"][:cfg2["n_data"]], cfg2["w"][cfg2["n_data"]:])
    rng = np.random.default_rng(2024)
    prim = np.concatenate([rng.choice(cfg2["n_data"], 12, replace=False),
                           cfg2["n_data"] + rng.choice(n - cfg2["n_data"], 12, replace=False)])
    with encore.build_grid(ctx, cfg2["pos"], cfg2["w"], r_max=160.0, box=cfg2["box"],
                           n_data=cfg2["n_data"]) as g:
        ag = encore.debug_alm(ctx, g, 5, cfg2["edges"], prim, precision, full_launch=True)
    ao = oracle.alm(cfg2["pos"], w, 5, cfg2["edges"], box=cfg2["box"], primaries=prim)
    worst = 0.0
    for i in range(len(prim)):
        err = np.max(np.abs(ag[i] - ao[i])) / np.max(np.abs(ao[i]))
        worst = max(worst, err)
        assert err <= (1e-12 if precision == "fp64" else 1e-6), (i, err)
    _say("  max |da|/max|a| per row = %.2e" % worst)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "splitbf16"])
def test_config2_zeta_sampled_primaries(ctx, cfg2, precision):
    """4PCF lmax = 5 on the full 800k-point D-R catalog, summed over 48 sampled
    primaries (all 800k are secondaries), vs the oracle on the same primaries."""
    _say("config2 zeta sampled " + precision)
    n = len(cfg2["w"])
    w = oracle.dmr_weights(cfg2["w"][:cfg2["n_data"]], cfg2["w"][cfg2["n_data"]:])
    prim = np.random.default_rng(7).choice(n, 48, replace=False)
    with encore.build_grid(ctx, cfg2["pos"], cfg2["w"], r_max=160.0, box=cfg2["box"],
                           n_data=cfg2["n_data"]) as g:
        zg = encore.npcf(ctx, g, 4, 5, cfg2["edges"], precision=precision, primaries=prim)
    zo, za = oracle.zeta(cfg2["pos"], w, 4, 5, cfg2["edges"], box=cfg2["box"], primaries=prim,
                         return_abs=True)
    e, r = bars.check(zg, zo, za, precision, "config 2")
    _say("  max e_L = %.3e, max e_L/(kappa+1) = %.3e, median kappa = %.1f"
         % (e, r, np.median(bars.kappa(zo, za))))


@pytest.mark.parametrize("N,lmax,nbins,nprim", [(3, 10, 10, None), (4, 6, 12, None), (4, 10, 8, 40),
                                                (5, 5, 13, 4)])
def test_splitbf16_unstaged_blocks(ctx, N, lmax, nbins, nprim):
    """More than 256 coefficients per primary (the paper's lmax = 10 4PCF, the 3PCF at
    lmax = 10, the 5PCF at lmax = 5 with 13 bins): the split-bf16 coupling reads its
    K blocks in global memory instead of staging them in LDS; vs the oracle."""
    nent = nbins * (lmax + 1) * (lmax + 2) // 2
    assert nent > 256
    _say("unstaged split-bf16 N=%d lmax=%d nbins=%d (%d coefficients per primary)" % (N, lmax, nbins, nent))
    pos, w = _uniform(700, 60.0, 40 + N)
    edges = np.linspace(3.0, 26.0, nbins + 1)
    prim = None if nprim is None else np.random.default_rng(N).choice(len(w), nprim, replace=False)
    with encore.build_grid(ctx, pos, w, r_max=edges[-1], box=60.0) as g:
        zg = encore.npcf(ctx, g, N, lmax, edges, precision="splitbf16", primaries=prim)
    zo, za = oracle.zeta(pos, w, N, lmax, edges, box=60.0, primaries=prim, return_abs=True)
    e, r = bars.check(zg, zo, za, "splitbf16", "unstaged")
    _say("  max e_L = %.2e, max e_L/(kappa+1) = %.2e" % (e, r))


@pytest.fixture(scope="module")
def cfg3():
    return synth.config(3)


@pytest.mark.parametrize("N,lmax,nprim", [(5, 4, 12), (6, 3, 6)])
@pytest.mark.parametrize("precision", ["fp32", "splitbf16"])
def test_config3_wedge_sampled_primaries(ctx, cfg3, N, lmax, nprim, precision):
    """Survey-wedge workload in full (500k clustered data + 1.5M randoms in a
    non-periodic 600-1200 Mpc/h shell wedge with holes, FKP weights, D-R): 5PCF at
    lmax = 4 and 6PCF at lmax = 3 summed over seeded primaries, all 2M points as
    secondaries, vs the oracle."""
    _say("config3 wedge N=%d lmax=%d %s" % (N, lmax, precision))
    n = len(cfg3["w"])
    w = oracle.dmr_weights(cfg3["w"][:cfg3["n_data"]], cfg3["w"][cfg3["n_data"]:])
    prim = np.random.default_rng(30 + N).choice(n, nprim, replace=False)
    with encore.build_grid(ctx, cfg3["pos"], cfg3["w"], r_max=160.0, n_data=cfg3["n_data"]) as g:
        zg = encore.npcf(ctx, g, N, lmax, cfg3["edges"], precision=precision, primaries=prim)
    zo, za = oracle.zeta(cfg3["pos"], w, N, lmax, cfg3["edges"], primaries=prim, return_abs=True)
    e = _normwise(zg, zo)
    kappa = bars.kappa(zo, za)
    _say("  max e_L = %.3e, median e_L = %.3e, median kappa = %.1f, max e_L/(kappa+1) = %.2e"
         % (e.max(), np.median(e), np.median(kappa), np.max(e / (np.maximum(kappa, 1.0) + 1.0))))
    # The D-R field cancels inside each harmonic coefficient (sum_j |w_j Y_lm| /
    # |a~_lm| has median ~24 and reaches 1e3..1e5 on this geometry): the FP32
    # gather's FP64 accumulators keep that from reaching Z.
    bars.check(zg, zo, za, precision, "wedge")


# ------------------------------------------------------------------ batched jobs

@pytest.mark.parametrize("precision", ["fp64", "fp32", "splitbf16"])
def test_batch_each_job_matches_alone_and_oracle(ctx, precision):
    """Uneven catalogs (periodic and not, one point, one repeated) in one batched
    call: each job's zeta equals its single-job result and the oracle."""
    _say("batched jobs %s" % precision)
    N, lmax = 4, 3
    edges = np.linspace(3.0, 25.0, 6)
    specs = [(900, 60.0, True), (250, 60.0, False), (1, 60.0, True), (1400, 70.0, True),
             (600, 50.0, False)]
    cats, grids = [], []
    for k, (n, L, per) in enumerate(specs):
        pos, w = _uniform(n, L, 500 + k)
        box = L if per else None
        cats.append((pos, w, box))
        grids.append(encore.build_grid(ctx, pos, w, r_max=edges[-1], box=box))
    grids.append(grids[0])
    cats.append(cats[0])
    try:
        zb = encore.npcf_batch(ctx, grids, N, lmax, edges, precision=precision)
        alone = [encore.npcf(ctx, g, N, lmax, edges, precision=precision) for g in grids]
    finally:
        for g in grids[:-1]:
            g.free()
    assert zb.shape[0] == len(grids)
    for j, (pos, w, box) in enumerate(cats):
        zal = alone[j]
        zo, zabs = oracle.zeta(pos, w, N, lmax, edges, box=box, return_abs=True)
        # Per-job coupling splits and an in-order reduction: bit-identical to alone.
        assert np.array_equal(zb[j], zal), j
        bars.check(zb[j], zo, zabs, precision, "batched job %d" % j)
    assert np.array_equal(zb[0], zb[-1])


@pytest.mark.parametrize("precision", ["fp32", "splitbf16"])
def test_batch_matches_alone_many_slices(ctx, precision):
    """Twelve uneven catalogs with the benchmark kernels (lmax=5, two bin groups
    per work item): bit-identical to alone, also when the rows are cut into many
    slices that jobs straddle."""
    _say("batched jobs lmax=5 %s, 12 catalogs" % precision)
    N, lmax = 4, 5
    edges = np.linspace(4.0, 30.0, 11)
    rng = np.random.default_rng(77)
    grids, ns = [], []
    for k in range(12):
        n = int(rng.integers(200, 4000))
        pos, w = _uniform(n, 100.0, 900 + k)
        grids.append(encore.build_grid(ctx, pos, w, r_max=edges[-1], box=100.0))
        ns.append(n)
    try:
        zb = encore.npcf_batch(ctx, grids, N, lmax, edges, precision=precision)
        for j, g in enumerate(grids):
            za = encore.npcf(ctx, g, N, lmax, edges, precision=precision)
            assert np.array_equal(zb[j], za), (j, ns[j])
        # slices of at most 2500 rows: jobs straddle slice boundaries
        os.environ["ENCORE_MAX_SLICE_ROWS"] = "2500"
        try:
            zs = encore.npcf_batch(ctx, grids, N, lmax, edges, precision=precision)
            assert ctx.last_timings()["batches"] > 5
            for j, g in enumerate(grids):
                za = encore.npcf(ctx, g, N, lmax, edges, precision=precision)
                assert np.array_equal(zs[j], za), (j, ns[j])
                assert np.max(np.abs(zs[j] - zb[j])) <= 1e-5 * np.max(np.abs(zb[j])), (j, ns[j])
        finally:
            del os.environ["ENCORE_MAX_SLICE_ROWS"]
    finally:
        for g in grids:
            g.free()
