"""Seeded synthetic catalogs (inputs only: no estimator arithmetic lives here).

Every generator is deterministic in its seed (numpy PCG64 via default_rng) and
returns FP64 positions [n, 3] plus positive FP64 weights [n].  Data and randoms
are returned separately; forming the data-minus-randoms weights is part of the
estimator and is done by the library (and, independently, by the oracle).

Workloads (stand-ins for the mock galaxy catalogs of the paper, which are not
available):

* uniform_box            uniform points in a periodic cube
* neyman_scott           clustered points: Poisson parents, Poisson(mean_children)
                         children with isotropic Gaussian offsets, wrapped into the
                         periodic cube, then thinned uniformly to exactly n points
* survey_wedge           a non-periodic spherical-shell wedge with circular holes
                         (data clustered as above, randoms uniform in the volume)
* fkp_weights            w = 1 / (1 + nbar * P0)
"""
import math

import numpy as np

__all__ = ["uniform_box", "neyman_scott", "survey_wedge", "fkp_weights",
           "linear_edges", "mock_dmr_catalog", "batch_sizes", "mesh_counts", "mesh_overdensity",
           "config"]


def linear_edges(rmin: float, rmax: float, nbins: int) -> np.ndarray:
    return np.linspace(rmin, rmax, nbins + 1)


def uniform_box(n: int, box: float, seed: int):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box, size=(n, 3))
    pos = np.where(pos >= box, 0.0, pos)
    return pos, np.ones(n)


def neyman_scott(n: int, box: float, seed: int, nbar_parent: float = 3e-5,
                 mean_children: float = 10.0, sigma: float = 5.0):
    """Neyman-Scott clustered catalog thinned to exactly n points (periodic cube).

    If the parent density is too low to reach n points it is raised
    (parents ~ Poisson(1.1 n / mean_children)) before thinning."""
    rng = np.random.default_rng(seed)
    vol = box ** 3
    lam_p = max(nbar_parent * vol, 1.1 * n / mean_children)
    while True:
        npar = rng.poisson(lam_p)
        parents = rng.uniform(0.0, box, size=(npar, 3))
        nchild = rng.poisson(mean_children, size=npar)
        total = int(nchild.sum())
        if total >= n:
            break
        lam_p *= 1.2
    owner = np.repeat(np.arange(npar), nchild)
    pos = parents[owner] + rng.normal(0.0, sigma, size=(total, 3))
    pos = np.mod(pos, box)
    pos = np.where(pos >= box, 0.0, pos)
    keep = rng.choice(total, size=n, replace=False)
    keep.sort()
    return np.ascontiguousarray(pos[keep]), np.ones(n)


def _in_wedge(pos, rmin, rmax, ra_max_deg, dec_half_deg, holes):
    x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
    r = np.sqrt(x * x + y * y + z * z)
    ra = np.degrees(np.arctan2(y, x)) % 360.0
    dec = np.degrees(np.arcsin(np.clip(z / np.maximum(r, 1e-300), -1, 1)))
    ok = (r >= rmin) & (r < rmax) & (ra < ra_max_deg) & (np.abs(dec) <= dec_half_deg)
    for (hra, hdec, hrad) in holes:
        # angular distance to the hole centre
        c = (np.sin(np.radians(dec)) * np.sin(np.radians(hdec)) +
             np.cos(np.radians(dec)) * np.cos(np.radians(hdec)) *
             np.cos(np.radians(ra - hra)))
        ok &= np.degrees(np.arccos(np.clip(c, -1, 1))) > hrad
    return ok


def _uniform_wedge(n, rng, rmin, rmax, ra_max, dec_half, holes):
    out = []
    got = 0
    while got < n:
        m = int((n - got) * 1.3) + 1000
        r = np.cbrt(rng.uniform(rmin ** 3, rmax ** 3, m))
        ra = np.radians(rng.uniform(0.0, ra_max, m))
        sdec = rng.uniform(-math.sin(math.radians(dec_half)), math.sin(math.radians(dec_half)), m)
        cdec = np.sqrt(1.0 - sdec * sdec)
        p = np.stack([r * cdec * np.cos(ra), r * cdec * np.sin(ra), r * sdec], axis=1)
        p = p[_in_wedge(p, rmin, rmax, ra_max, dec_half, holes)]
        out.append(p)
        got += len(p)
    return np.concatenate(out)[:n]


def survey_wedge(n_data: int, n_rand: int, seed: int, rmin: float = 600.0,
                 rmax: float = 1200.0, ra_max: float = 90.0, dec_half: float = 30.0,
                 n_holes: int = 5, hole_deg: float = 2.0, sigma: float = 5.0,
                 mean_children: float = 10.0):
    """Non-periodic wedge RA in [0, ra_max), |Dec| <= dec_half, r in [rmin, rmax) with
    n_holes circular holes.  Returns (data_pos, rand_pos, holes)."""
    rng = np.random.default_rng(seed)
    holes = [(rng.uniform(0, ra_max), rng.uniform(-dec_half, dec_half), hole_deg)
             for _ in range(n_holes)]
    data = []
    got = 0
    while got < n_data:
        npar = int(1.3 * (n_data - got) / mean_children) + 100
        parents = _uniform_wedge(npar, rng, rmin, rmax, ra_max, dec_half, holes)
        nchild = rng.poisson(mean_children, size=npar)
        owner = np.repeat(np.arange(npar), nchild)
        p = parents[owner] + rng.normal(0.0, sigma, size=(len(owner), 3))
        p = p[_in_wedge(p, rmin, rmax, ra_max, dec_half, holes)]
        data.append(p)
        got += len(p)
    data = np.concatenate(data)
    keep = np.sort(rng.choice(len(data), size=n_data, replace=False))
    data = np.ascontiguousarray(data[keep])
    rand = np.ascontiguousarray(_uniform_wedge(n_rand, rng, rmin, rmax, ra_max, dec_half, holes))
    return data, rand, holes


def fkp_weights(n: int, nbar: float, p0: float = 1e4) -> np.ndarray:
    return np.full(n, 1.0 / (1.0 + nbar * p0))


def mock_dmr_catalog(nd: int, box: float, seed: int):
    """One mock of the batched and served workloads: Neyman-Scott data thinned to
    nd points plus 3 nd uniform randoms in a periodic cube (input weights 1; the
    data-minus-randoms weights are formed by the estimator).  Returns (pos, w)."""
    dpos, dw = neyman_scott(nd, box, seed)
    rpos, rw = uniform_box(3 * nd, box, seed + 7919)
    return np.concatenate([dpos, rpos]), np.concatenate([dw, rw])


def mesh_counts(pos, w, n: int, box: float):
    """Weights of a catalog summed per cell of a periodic n^3 mesh (cell index
    floor(x n / box) per axis), C order [ix, iy, iz]: the input field of the gridded
    workload."""
    idx = np.floor(np.asarray(pos) / (box / n)).astype(np.int64) % n
    flat = (idx[:, 0] * n + idx[:, 1]) * n + idx[:, 2]
    return np.bincount(flat, weights=np.asarray(w, dtype=np.float64), minlength=n ** 3).reshape(n, n, n)


def mesh_overdensity(n: int, box: float, npts: int, seed: int):
    """A clustered overdensity field delta = rho / mean(rho) - 1 on a periodic n^3
    mesh: a Neyman-Scott catalog of npts points counted per cell."""
    pos, w = neyman_scott(npts, box, seed)
    rho = mesh_counts(pos, w, n, box)
    return rho / rho.mean() - 1.0


def batch_sizes(njobs: int = 64, seed: int = 4000):
    """Data counts of the batched workload's mocks, N_D ~ U{50k..400k}; mock k is
    mock_dmr_catalog(sizes[k], 1000, seed + k)."""
    return np.random.default_rng(seed).integers(50_000, 400_001, size=njobs)


def config(k: int, scale: float = 1.0):
    """The five benchmark workloads as plain dicts of inputs.

    scale < 1 shrinks the point counts (same density profile is NOT kept; use only
    for quick tests)."""
    edges = linear_edges(20.0, 160.0, 10)
    if k == 1:
        n = int(2000 * scale)
        pos, w = uniform_box(n, 500.0, 1001)
        return dict(name="3PCF uniform periodic 500 Mpc/h, 2000 points, lmax=10",
                    pos=pos, w=w, n_data=n, N=3, lmax=10, edges=edges, box=500.0)
    if k == 2:
        nd = int(200_000 * scale)
        nr = 3 * nd
        dpos, dw = neyman_scott(nd, 1000.0, 1002)
        rpos, rw = uniform_box(nr, 1000.0, 2002)
        return dict(name="4PCF Neyman-Scott D-R periodic 1000 Mpc/h, %d data + %d randoms, lmax=5"
                    % (nd, nr),
                    pos=np.concatenate([dpos, rpos]), w=np.concatenate([dw, rw]),
                    n_data=nd, N=4, lmax=5, edges=edges, box=1000.0)
    if k == 3:
        nd = int(500_000 * scale)
        nr = 3 * nd
        dpos, rpos, holes = survey_wedge(nd, nr, 1003)
        vol = (math.radians(90.0) * 2 * math.sin(math.radians(30.0)) *
               (1200.0 ** 3 - 600.0 ** 3) / 3.0)
        nbar = nd / vol
        wd = fkp_weights(nd, nbar)
        wr = fkp_weights(nr, nbar)
        return dict(name="5PCF/6PCF survey wedge, %d data + %d randoms" % (nd, nr),
                    pos=np.concatenate([dpos, rpos]), w=np.concatenate([wd, wr]),
                    n_data=nd, N=5, lmax=4, edges=edges, box=None, holes=holes)
    raise ValueError("config %d is built by the batch / serving drivers" % k)
