"""Pins of the oracle's random-split co-adding (Section 4.2), CPU only.

The per-part estimator is the pinned `zeta`; what is pinned here is the split
structure: the parts are consecutive and disjoint, each part is weighted as its
own data-minus-randoms catalog (total weight zero within the part), and the parts
are averaged, not summed.
"""
import numpy as np

import oracle
from oracle.brute import brute_zeta


def _catalogs(nd, nr, L, seed):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0, L, (nd, 3)), rng.uniform(0.5, 1.5, nd),
            rng.uniform(0, L, (nr, 3)), rng.uniform(0.5, 1.5, nr))


def test_split_mean_equals_brute_force_per_part():
    """Tiny catalogs: the mean over three unequal parts of the O(N_g^N) tuple sums,
    each part weighted so that its randoms carry minus the data's total weight."""
    L = 8.0
    dpos, dw, rpos, rw = _catalogs(6, 12, L, 21)
    sizes = [3, 4, 5]
    edges = np.linspace(0.6, 4.0, 4)
    mean, per = oracle.split_zeta(dpos, dw, rpos, rw, sizes, 4, 2, edges, box=L)
    ref = []
    o = 0
    for n in sizes:
        wr = rw[o:o + n]
        w = np.concatenate([dw, -wr * (dw.sum() / wr.sum())])
        assert abs(w.sum()) < 1e-12
        ref.append(brute_zeta(np.concatenate([dpos, rpos[o:o + n]]), w, 4, 2, edges, box=L))
        o += n
    ref = np.array(ref)
    scale = np.max(np.abs(ref))
    assert scale > 0
    assert np.max(np.abs(per - ref)) <= 1e-12 * scale
    assert np.max(np.abs(mean - ref.mean(axis=0))) <= 1e-12 * scale


def test_identical_parts_average_to_one_part():
    """K copies of one random part: every part gives the same Z, and the co-added
    result is that Z (a mean, not K times it)."""
    L = 20.0
    dpos, dw, rpos, rw = _catalogs(40, 60, L, 5)
    edges = np.linspace(1.0, 8.0, 5)
    K = 3
    mean, per = oracle.split_zeta(dpos, dw, np.tile(rpos, (K, 1)), np.tile(rw, K), [60] * K, 3, 3, edges,
                                  box=L)
    one = oracle.zeta(np.concatenate([dpos, rpos]), oracle.dmr_weights(dw, rw), 3, 3, edges, box=L)
    for k in range(K):
        assert np.array_equal(per[k], per[0])
    assert np.max(np.abs(mean - one)) <= 1e-13 * np.max(np.abs(one))


def test_part_weights_follow_their_own_randoms():
    """Parts of different total random weight get different random weights: the
    result differs from weighting all randoms together (the per-part rule is what
    the estimator needs, since each part must have total weight zero)."""
    L = 20.0
    dpos, dw, rpos, rw = _catalogs(40, 90, L, 8)
    rw[:30] *= 3.0
    edges = np.linspace(1.0, 8.0, 4)
    _, per = oracle.split_zeta(dpos, dw, rpos, rw, [30, 60], 3, 2, edges, box=L)
    wall = oracle.dmr_weights(dw, rw)
    pos0 = np.concatenate([dpos, rpos[:30]])
    w_global = np.concatenate([dw, wall[40:70]])
    z_global = oracle.zeta(pos0, w_global, 3, 2, edges, box=L)
    assert np.max(np.abs(per[0] - z_global)) > 1e-3 * np.max(np.abs(per[0]))
