"""Pins of the gridded-data oracle (Section 3.2, Gridded Data), CPU only.

A catalog assigned to a periodic mesh cell by cell gives, through the mesh
estimator (direct correlation over mesh offsets, cells as primaries weighted by
their summed weight), exactly the discrete estimator's Z of the catalog with every
point moved to its cell centre: pairs within one cell are at zero separation
(below edges[0]) in both, and every point of a cell sees the same coefficients.
"""
import numpy as np
import pytest

import oracle
from oracle import mesh


def _snapped(n_pts, n, L, seed, clustered=False):
    rng = np.random.default_rng(seed)
    if clustered:   # several points per cell
        centres = rng.uniform(0, L, (n_pts // 6, 3))
        pos = (centres[rng.integers(0, len(centres), n_pts)] + rng.normal(0, 0.6 * L / n, (n_pts, 3))) % L
    else:
        pos = rng.uniform(0, L, (n_pts, 3))
    w = rng.uniform(-1.0, 1.5, n_pts)
    cells = np.floor(pos / (L / n)).astype(np.int64) % n
    return pos, w, cells


@pytest.mark.parametrize("N,lmax,parity", [(3, 4, "even"), (4, 2, "all"), (5, 1, "even")])
def test_zeta_from_alm_matches_discrete_oracle(N, lmax, parity):
    """The full-M sum over given coefficients equals the C oracle's Z (which forms
    its own coefficients) on the same catalog."""
    rng = np.random.default_rng(3 + N)
    pos = rng.uniform(0, 30.0, (220, 3))
    w = rng.uniform(0.5, 1.5, 220)
    edges = np.linspace(2.0, 12.0, 6)
    a = oracle.alm(pos, w, lmax, edges, box=30.0)
    z = mesh.zeta_from_alm(a, w, N, lmax, parity)
    zo = oracle.zeta(pos, w, N, lmax, edges, box=30.0, parity=parity)
    assert np.max(np.abs(z - zo)) <= 1e-12 * np.max(np.abs(zo))


@pytest.mark.parametrize("N,lmax,parity,clustered", [(3, 4, "even", False), (4, 2, "all", True),
                                                      (5, 1, "even", True)])
def test_mesh_equals_discrete_on_cell_centres(N, lmax, parity, clustered):
    n, L = 16, 16.0                       # cell side 1; no mesh distance falls on an edge
    edges = np.array([1.5, 2.7, 4.1, 5.3, 6.6])
    pos, w, cells = _snapped(400, n, L, 10 + N, clustered)
    delta = mesh.ngp_assign(pos, w, n, L)
    assert np.isclose(delta.sum(), w.sum())
    if clustered:
        assert len(np.unique(cells, axis=0)) < len(cells)      # shared cells exercised
    zm = mesh.mesh_zeta(delta, L, N, lmax, edges, parity)
    zo = oracle.zeta(mesh.cell_centres(cells, n, L), w, N, lmax, edges, box=L, parity=parity)
    assert np.max(np.abs(zm - zo)) <= 1e-11 * np.max(np.abs(zo))


def test_mesh_alm_matches_discrete_alm_on_cell_centres():
    n, L = 12, 24.0                       # cell side 2
    edges = np.array([2.5, 4.3, 7.9, 11.1])
    pos, w, cells = _snapped(150, n, L, 5)
    delta = mesh.ngp_assign(pos, w, n, L)
    pick = np.arange(0, 150, 7)
    am = mesh.mesh_alm(delta, L, 5, edges, cells[pick])
    ao = oracle.alm(mesh.cell_centres(cells, n, L), w, 5, edges, box=L, primaries=pick)
    assert np.max(np.abs(am - ao)) <= 1e-12 * np.max(np.abs(ao))


def test_mesh_offsets_bins_are_exact():
    """Offsets exactly on a squared edge go to the upper bin; offsets at or beyond
    the last edge, and the zero offset, are outside every bin."""
    u, b = mesh.mesh_offsets(10, 10.0, np.array([1.0, 2.0, 3.0]))
    r2 = (u * u).sum(1)
    assert np.all(r2 >= 1) and np.all(r2 < 9)
    assert np.all(b[r2 == 4] == 1) and np.all(b[r2 == 1] == 0)
    assert len(u) == np.sum([(i * i + j * j + k * k >= 1) and (i * i + j * j + k * k < 9)
                             for i in range(-3, 4) for j in range(-3, 4) for k in range(-3, 4)])
