"""Gridded-data estimator (encore_npcf_mesh, Section 3.2 Gridded Data) against the
oracle's direct correlation over mesh offsets, through the C ABI; and against the
discrete path on the catalog moved to its cell centres."""
import sys

import numpy as np
import pytest

import oracle
import parity_bars as bars
from oracle import mesh as omesh
from paper_2105_08722_amd import encore, synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-mesh] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = encore.Context(0)
    yield c
    c.close()


def _catalog(npts, n, L, seed):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, L, (npts, 3))
    w = rng.uniform(-1.0, 1.5, npts)
    return pos, w


CASES = [  # N, lmax, n, allparity
    (3, 4, 16, False),
    (4, 3, 16, False),
    (4, 2, 12, True),
    (5, 1, 16, False),
    (6, 1, 12, False),
    (6, 1, 12, True),
]


@pytest.mark.parametrize("N,lmax,n,allp", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32", "splitbf16"])
def test_mesh_matches_oracle(ctx, N, lmax, n, allp, precision):
    """A sparse mesh (a catalog counted per cell, mixed-sign weights; several
    points share cells): Z against the oracle's direct correlation."""
    import torch
    _say("mesh N=%d lmax=%d n=%d allparity=%s %s" % (N, lmax, n, allp, precision))
    L = float(n)                                   # cell side 1
    # no mesh distance falls on an edge (squared edges are not integers); the 6PCF
    # needs five bins for a bin tuple
    edges = np.array([1.5, 2.3, 3.1, 3.9, 4.7, 5.5]) if N == 6 else np.array([1.5, 2.7, 4.1, 5.3, 5.9])
    assert encore.num_bin_tuples(N, len(edges) - 1) > 0
    pos, w = _catalog(600, n, L, 7 * N + lmax)
    delta = synth.mesh_counts(pos, w, n, L)
    zg = encore.npcf_mesh(ctx, torch.from_numpy(delta).cuda(), L, N, lmax, edges, precision=precision,
                          allparity=allp)
    zo, za = omesh.mesh_zeta(delta, L, N, lmax, edges, parity="all" if allp else "even", return_abs=True)
    e, r = bars.check(zg, zo, za, precision, "mesh")
    _say("  max e_L = %.2e, max e_L/(kappa+1) = %.2e, timings %s" % (e, r, ctx.last_timings()))


def test_mesh_equals_discrete_path_on_cell_centres(ctx):
    """The same catalog through the discrete path, every point moved to its cell
    centre: the two device paths agree to FP64 rounding."""
    import torch
    n, L = 16, 16.0
    edges = np.array([1.5, 2.7, 4.1, 5.3, 6.6])
    pos, w = _catalog(900, n, L, 3)
    cells = np.floor(pos / (L / n)).astype(np.int64) % n
    delta = synth.mesh_counts(pos, w, n, L)
    zm = encore.npcf_mesh(ctx, torch.from_numpy(delta).cuda(), L, 4, 3, edges, precision="fp64")
    with encore.build_grid(ctx, (cells + 0.5) * (L / n), w, r_max=edges[-1], box=L) as g:
        zd = encore.npcf(ctx, g, 4, 3, edges, precision="fp64")
    assert np.max(np.abs(zm - zd)) <= 1e-10 * np.max(np.abs(zd))


def test_mesh_dense_overdensity_field(ctx):
    """A dense field (every cell a primary): a clustered overdensity on 20^3 cells,
    FP64 and split-bf16, against the oracle."""
    import torch
    n, L = 20, 200.0                               # cell side 10
    edges = np.array([12.0, 27.0, 41.0, 58.0, 79.0, 95.0])
    delta = synth.mesh_overdensity(n, L, 20000, 12)
    t = torch.from_numpy(delta).cuda()
    zo, za = omesh.mesh_zeta(delta, L, 4, 2, edges, return_abs=True)
    for prec in ["fp64", "splitbf16"]:
        zg = encore.npcf_mesh(ctx, t, L, 4, 2, edges, precision=prec)
        e, r = bars.check(zg, zo, za, prec, "dense mesh")
        _say("  dense %s: max e_L = %.2e" % (prec, e))


def test_mesh_kernel_transforms_reused(ctx):
    """A call with the previous call's shape reuses the transformed kernel fields:
    the same field gives the same Z bit for bit, another field on that shape still
    matches the oracle, and a change of edges rebuilds the transforms."""
    import torch
    n, L = 16, 16.0
    edges = np.array([1.5, 2.6, 3.7, 5.1])
    edges2 = np.array([1.5, 2.9, 4.3, 5.6])
    d1 = synth.mesh_counts(*_catalog(700, n, L, 21), n, L)
    d2 = synth.mesh_counts(*_catalog(500, n, L, 22), n, L)
    t1, t2 = torch.from_numpy(d1).cuda(), torch.from_numpy(d2).cuda()
    za = encore.npcf_mesh(ctx, t1, L, 4, 2, edges, precision="fp64")
    assert ctx.last_timings()["pairs"] == 0        # first call of this shape
    zb = encore.npcf_mesh(ctx, t1, L, 4, 2, edges, precision="fp64")
    assert ctx.last_timings()["pairs"] == 1        # transforms reused
    assert np.array_equal(za, zb)
    zc = encore.npcf_mesh(ctx, t2, L, 4, 2, edges, precision="splitbf16")
    assert ctx.last_timings()["pairs"] == 1        # the precision is not part of the shape
    zo, zabs = omesh.mesh_zeta(d2, L, 4, 2, edges, return_abs=True)
    bars.check(zc, zo, zabs, "splitbf16", "mesh, reused transforms")
    zd = encore.npcf_mesh(ctx, t2, L, 4, 2, edges2, precision="fp64")
    assert ctx.last_timings()["pairs"] == 0
    zo, zabs = omesh.mesh_zeta(d2, L, 4, 2, edges2, return_abs=True)
    bars.check(zd, zo, zabs, "fp64", "mesh, rebuilt transforms")
    ze = encore.npcf_mesh(ctx, t1, L, 4, 2, edges, precision="fp64")
    assert ctx.last_timings()["pairs"] == 0
    assert np.array_equal(ze, za)


def test_mesh_rejects_bad_arguments(ctx):
    import torch
    delta = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(encore.EncoreError) as e:
        encore.npcf_mesh(ctx, delta, 8.0, 3, 2, np.array([1.0, 2.0, 4.5]))     # beyond box/2
    assert e.value.code == encore.EINVAL
    with pytest.raises(TypeError):
        encore.npcf_mesh(ctx, delta.float(), 8.0, 3, 2, np.array([1.0, 2.0, 3.0]))
    z = encore.npcf_mesh(ctx, delta, 8.0, 3, 2, np.array([1.0, 2.0, 3.0]))       # empty field
    assert np.all(z == 0.0)
