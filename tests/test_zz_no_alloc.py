"""encore_npcf_noalloc (no device allocation in the call) against encore_npcf,
through the C ABI: two calls in a row, the second on a smaller input, in each
precision; a job cut into several slices of the scratch buffer; and a job whose
sums cannot fit the scratch buffer."""
import sys

import numpy as np
import pytest

import oracle
import parity_bars as bars
from paper_2105_08722_amd import encore

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-noalloc] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = encore.Context(0)
    yield c
    c.close()


def _cat(n, L, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, L, (n, 3)), rng.uniform(0.5, 1.5, n)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "splitbf16"])
def test_noalloc_equals_npcf_two_calls(ctx, precision):
    """One slice each: the allocation-free call equals encore_npcf bit for bit
    (same kernels, same split of the primaries) and meets the oracle bar; the
    second call runs a smaller catalog and a primary subset over the scratch the
    first one left behind."""
    L = 60.0
    edges = np.linspace(3.0, 25.0, 7)
    for k, (n, periodic, sub) in enumerate([(1500, True, None), (400, False, 97)]):
        _say("%s call %d: %d points periodic=%s subset=%s" % (precision, k + 1, n, periodic, sub))
        pos, w = _cat(n, L, 40 + k)
        box = L if periodic else None
        prim = np.random.default_rng(k).choice(n, sub, replace=False) if sub else None
        with encore.build_grid(ctx, pos, w, r_max=edges[-1], box=box) as g:
            ref = encore.npcf(ctx, g, 4, 3, edges, precision=precision, primaries=prim)
            got = encore.npcf(ctx, g, 4, 3, edges, precision=precision, primaries=prim, noalloc=True)
            assert ctx.last_timings()["batches"] == 1
        assert np.array_equal(got, ref), k
        zo, za = oracle.zeta(pos, w, 4, 3, edges, box=box, primaries=prim, return_abs=True)
        bars.check(got, zo, za, precision, "noalloc call %d" % (k + 1))


def test_noalloc_several_slices_fp64(ctx):
    """A job larger than one slice of the scratch buffer (lmax 5, 10 bins, FP64:
    3.4 kB of coefficients per primary, 200k primaries): the allocation-free call
    runs it in several slices and equals encore_npcf to FP64 rounding; a smaller
    job follows on the same scratch."""
    edges = np.linspace(4.0, 40.0, 11)
    for k, n in enumerate([200_000, 30_000]):
        _say("fp64 several slices, call %d: %d points" % (k + 1, n))
        pos, w = _cat(n, 400.0, 70 + k)
        with encore.build_grid(ctx, pos, w, r_max=edges[-1], box=400.0) as g:
            ref = encore.npcf(ctx, g, 4, 5, edges, precision="fp64")
            got = encore.npcf(ctx, g, 4, 5, edges, precision="fp64", noalloc=True)
            nslice = ctx.last_timings()["batches"]
        _say("  %d slices" % nslice)
        if k == 0:
            assert nslice > 1
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_noalloc_refuses_what_does_not_fit(ctx):
    """5PCF at lmax 5 over 16 bins holds 553 MB of per-job sums: more than the
    scratch buffer, refused with ESIZE; the next call still works."""
    pos, w = _cat(300, 40.0, 9)
    edges = np.linspace(2.0, 18.0, 17)
    with encore.build_grid(ctx, pos, w, r_max=edges[-1], box=40.0) as g:
        with pytest.raises(encore.EncoreError) as e:
            encore.npcf(ctx, g, 5, 5, edges, precision="fp64", noalloc=True)
        assert e.value.code == encore.ESIZE
        assert "scratch" in str(e.value)
        small = np.linspace(2.0, 18.0, 5)
        ref = encore.npcf(ctx, g, 4, 2, small, precision="fp32")
        got = encore.npcf(ctx, g, 4, 2, small, precision="fp32", noalloc=True)
        assert np.array_equal(got, ref)
