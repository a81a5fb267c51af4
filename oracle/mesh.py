"""Gridded-data estimator for the oracle (test infrastructure only).

Follows Section 3.2 (Gridded Data): for a density field delta on a periodic mesh
of n^3 cells of side h = L / n, the harmonic coefficients of every cell are the
binned correlation of eq. alm-binned-def,

    a~^b_lm(s) = sum_u delta(s + u) Y_lm(u^) Theta^b(|u|)        (no 1/v_b, raw),

u running over the mesh offsets in the minimum image (|u| < edges[-1] <= L/2), the
offset pointing from the primary cell s to the secondary cell s + u as in the
discrete estimator; the multiplets are then

    Z^B_L = sum_s delta(s) sum_M E(L) C^L_M prod_k a~^{b_k}_{l_k m_k}(s)

(eq. NPCF-mult-binned-estimator with the integral over s a sum over cells, no 1/V),
the three steps of the gridded procedure in the paper's order: the a~ fields,
the product of N - 1 of them weighted by delta and summed over cells, the sum over M
with the coupling weights.

This is the definition written out: a direct sum over offsets for every cell that
holds weight (no Fourier transform).  A catalog assigned to the mesh by cell
(nearest grid point) gives the same Z as the discrete estimator on the catalog
with every point moved to its cell's centre; tests/test_mesh_oracle.py pins both
functions that way, and zeta_from_alm also against the discrete oracle's own a~.

Bins are decided as everywhere in this package: edges[b]^2 <= r^2 < edges[b+1]^2
with r^2 = (ux*ux + uy*uy) + uz*uz in FP64.
"""
import numpy as np

from . import ylm, nlm, term_arrays
from .basis import bin_tuples, multiplets, parity_E

__all__ = ["ngp_assign", "cell_centres", "mesh_offsets", "mesh_alm", "zeta_from_alm", "mesh_zeta"]


def ngp_assign(pos, w, n, box):
    """Weights summed into the cell holding each point (periodic mesh n^3, cell side
    box / n, index floor(x / h) per axis): delta[ix, iy, iz]."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    idx = np.floor(pos / (box / n)).astype(np.int64) % n
    delta = np.zeros((n, n, n))
    np.add.at(delta, (idx[:, 0], idx[:, 1], idx[:, 2]), w)
    return delta


def cell_centres(cells, n, box):
    """Positions (i + 1/2) h of the cells [k, 3]."""
    return (np.asarray(cells, dtype=np.float64) + 0.5) * (box / n)


def mesh_offsets(n, box, edges):
    """Mesh offsets u (in cells) with edges[0] <= |u| h < edges[-1]: integer offsets
    [k, 3], their radial bins [k] and Y_lm(u^) is left to the caller."""
    h = box / n
    edges = np.asarray(edges, dtype=np.float64)
    if edges[-1] > box / 2:
        raise ValueError("edges[-1] must not exceed half the box")
    R = int(np.ceil(edges[-1] / h))   # offsets of +-n/2 cells lie at >= L/2: outside every bin
    rng = np.arange(-R, R + 1)
    u = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), axis=-1).reshape(-1, 3)
    d = u * h
    r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    e2 = edges * edges
    b = np.searchsorted(e2, r2, side="right") - 1        # e2[b] <= r2 < e2[b+1]
    keep = (b >= 0) & (b < len(edges) - 1)
    return u[keep], b[keep]


def mesh_alm(delta, box, lmax, edges, cells):
    """a~^b_lm at the given cells [k, 3] of the periodic mesh delta [n, n, n]:
    complex [k, nbins, nlm(lmax)], m >= 0, index l(l+1)/2 + m."""
    delta = np.asarray(delta, dtype=np.float64)
    n = delta.shape[0]
    h = box / n
    edges = np.asarray(edges, dtype=np.float64)
    nb = len(edges) - 1
    u, b = mesh_offsets(n, box, edges)
    Y = np.array([ylm(lmax, ui * h) for ui in u])       # [noff, nlm]
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
    out = np.zeros((len(cells), nb, nlm(lmax)), dtype=complex)
    for c, s in enumerate(cells):
        t = (s[None, :] + u) % n
        vals = delta[t[:, 0], t[:, 1], t[:, 2]]          # delta(s + u)
        for bb in range(nb):
            sel = b == bb
            out[c, bb] = vals[sel] @ Y[sel]
    return out


def zeta_from_alm(a, w, N, lmax, parity="even", return_abs=False):
    """Z^B_L = sum_i w_i sum_M E(L) C^L_M prod_k a~^{b_k}_{l_k m_k}(i) over every M (full
    sum; a~ of negative m from a~_{l,-m} = (-1)^m conj(a~_{lm}), the weights being
    real).  a: complex [nprim, nbins, nlm(lmax)].  Re for even, Im for odd multiplets;
    with return_abs also sum_i |w_i H_i| of the same component (H_i the sum over M
    of primary i)."""
    a = np.asarray(a)
    w = np.asarray(w, dtype=np.float64)
    nb = a.shape[1]
    lams = multiplets(N, lmax, parity)
    btab = np.array(bin_tuples(N, nb), dtype=np.int64).reshape(-1, N - 1)
    odd = np.array([parity_E(N, lam) < 0 for lam in lams], dtype=bool)
    H = np.zeros((len(lams), a.shape[0], len(btab)), dtype=complex)
    if len(btab) > 0:
        t_lam, t_l, t_m, t_c = term_arrays(N, lmax, parity)

        def coef(l, m):                                  # [nprim, nbins]
            v = a[:, :, l * (l + 1) // 2 + abs(m)]
            return v if m >= 0 else (-1) ** (abs(m) % 2) * np.conj(v)

        for t in range(len(t_lam)):
            prod = np.full((a.shape[0], len(btab)), t_c[t], dtype=complex)
            for k in range(N - 1):
                prod = prod * coef(int(t_l[t, k]), int(t_m[t, k]))[:, btab[:, k]]
            H[t_lam[t]] += prod
    wH = H * w[None, :, None]
    Z = wH.sum(axis=1)
    z = np.where(odd[:, None], Z.imag, Z.real)
    if not return_abs:
        return z
    comp = np.where(odd[:, None, None], wH.imag, wH.real)
    return z, np.abs(comp).sum(axis=1)


def mesh_zeta(delta, box, N, lmax, edges, parity="even", return_abs=False):
    """Z of the gridded estimator: every cell with nonzero delta is a primary of
    weight delta(s)."""
    delta = np.asarray(delta, dtype=np.float64)
    cells = np.argwhere(delta != 0.0)
    a = mesh_alm(delta, box, lmax, edges, cells)
    return zeta_from_alm(a, delta[cells[:, 0], cells[:, 1], cells[:, 2]], N, lmax, parity, return_abs)
