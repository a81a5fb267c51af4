"""Parity bars of the reduced-precision paths against the FP64 oracle.

Per multiplet, normwise over bin tuples, e_L = ||Z_gpu - Z_orc|| / ||Z_orc||, with
the conditioning kappa_L = ||sum_i |w_i H_i|| / ||Z_orc|| of the sum over primaries
(the oracle returns sum_i |w_i H_i|).  The bar is

    e_L <= u * max(kappa_L, 1) + u,   u = 1e-6 (FP32 path), 1e-5 (split-bf16 path),

for every multiplet; FP64 is held to 1e-10 of max|Z| (rounding order only).
"""
import numpy as np

UNIT = {"fp32": 1e-6, "splitbf16": 1e-5}


def normwise(zg, zo):
    """Per-multiplet ||zg - zo|| / ||zo|| (multiplets with ||zo|| below 1e-9 of the
    largest are skipped: their bins hold no pairs)."""
    num = np.linalg.norm(zg - zo, axis=1)
    den = np.linalg.norm(zo, axis=1)
    keep = den > 1e-9 * max(den.max(), 1e-300)
    return np.where(keep, num / np.where(keep, den, 1.0), 0.0)


def kappa(zo, za):
    return np.linalg.norm(za, axis=1) / np.maximum(np.linalg.norm(zo, axis=1), 1e-300)


def check(zg, zo, za, precision, what=""):
    """Assert the bar of `precision` ('fp64', 'fp32', 'splitbf16'); returns
    (max e_L, max e_L / (max(kappa_L, 1) + 1)) for the log."""
    zg = np.asarray(zg).reshape(zo.shape)
    if zo.size == 0:
        return 0.0, 0.0
    if precision == "fp64":
        scale = max(np.max(np.abs(zo)), 1e-300)
        err = np.max(np.abs(zg - zo)) / scale
        assert err <= 1e-10, (what, err)
        return err, err
    u = UNIT[precision]
    e = normwise(zg, zo)
    k = np.maximum(kappa(zo, za), 1.0)
    ratio = e / (k + 1.0)
    worst = int(np.argmax(ratio))
    assert np.all(e <= u * k + u), (what, precision, "multiplet %d: e=%.3e kappa=%.3g bar=%.3e"
                                    % (worst, e[worst], k[worst], u * k[worst] + u))
    return float(e.max()), float(ratio.max())
