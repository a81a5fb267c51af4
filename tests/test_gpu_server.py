"""Serving loop on the GPU: jobs of mixed N, lmax, sizes and precisions submitted
while others run; each result must be bit-identical to the same catalog run
alone through encore_npcf (and match the oracle), a failing job fails alone, and
admission keeps the held device memory within the budget."""
import threading
import time

import numpy as np
import pytest

import oracle
import parity_bars as bars
from paper_2105_08722_amd import encore

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-server] " + msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = encore.Context(0)
    yield c
    c.close()


def _jobs(seed):
    rng = np.random.default_rng(seed)
    specs = []
    kinds = [(3, 6, "fp64"), (4, 3, "fp32"), (5, 2, "fp32"), (4, 3, "fp64"), (3, 6, "fp32"),
             (4, 3, "splitbf16")]
    for k in range(10):
        N, lmax, prec = kinds[k % len(kinds)]
        n = int(rng.integers(150, 1500))
        L = float(rng.uniform(45.0, 70.0))
        pos = rng.uniform(0, L, (n, 3))
        w = rng.uniform(0.5, 1.5, n)
        periodic = bool(k % 3 != 1)
        specs.append(dict(pos=pos, w=w, N=N, lmax=lmax, precision=prec, box=L if periodic else None,
                          edges=np.linspace(3.0, 20.0, 6)))
    return specs


def _alone(ctx, sp):
    with encore.build_grid(ctx, sp["pos"], sp["w"], r_max=sp["edges"][-1], box=sp["box"]) as g:
        return encore.npcf(ctx, g, sp["N"], sp["lmax"], sp["edges"], precision=sp["precision"])


@pytest.mark.parametrize("n_lanes", [1, 3])
def test_server_mix_equals_alone(ctx, n_lanes):
    _say("mixed stream, %d lanes" % n_lanes)
    specs = _jobs(11 + n_lanes)
    bad = dict(specs[4])
    bad["pos"] = bad["pos"].copy()
    bad["pos"][7, 1] = np.nan                      # fails at grid build, alone
    with encore.Server(ctx, hbm_budget=1 << 30, n_lanes=n_lanes, max_active=4, slice_rows=700) as srv:
        ids = []

        def feed():
            rng = np.random.default_rng(3)
            for k, sp in enumerate(specs):
                ids.append(srv.submit(sp["pos"], sp["w"], sp["N"], sp["lmax"], sp["edges"], box=sp["box"],
                                      precision=sp["precision"]))
                if k == 4:
                    ids.append(srv.submit(bad["pos"], bad["w"], bad["N"], bad["lmax"], bad["edges"],
                                          box=bad["box"], precision=bad["precision"]))
                time.sleep(float(rng.uniform(0, 0.01)))

        th = threading.Thread(target=feed)
        th.start()
        th.join()
        results = {}
        for jid in ids:
            try:
                results[jid] = srv.wait(jid, timeout=120)
            except encore.EncoreError as e:
                results[jid] = e
        st = srv.stats()
    order = specs[:5] + [bad] + specs[5:]
    for jid, sp in zip(ids, order):
        r = results[jid]
        if sp is bad:
            assert isinstance(r, encore.EncoreError) and r.code == encore.EINVAL
            continue
        assert not isinstance(r, Exception), r
        z, t = r
        assert t["submit"] <= t["admit"] <= t["start"] <= t["done"]
        za = _alone(ctx, sp)
        assert np.array_equal(z, za), (jid, sp["N"], sp["lmax"], sp["precision"])
    assert st["done"] == len(specs) and st["failed"] == 1
    assert st["peak_bytes_held"] <= 1 << 30
    # one result of each kind against the oracle
    for sp, jid in list(zip(order, ids))[:3]:
        zo, zabs = oracle.zeta(sp["pos"], sp["w"], sp["N"], sp["lmax"], sp["edges"], box=sp["box"],
                               return_abs=True)
        bars.check(results[jid][0], zo, zabs, sp["precision"], "served job")


def test_server_admission_budget(ctx):
    """A budget that holds about one job: jobs run one after another, held memory
    never exceeds it, results unchanged."""
    _say("admission under a small budget")
    specs = _jobs(5)[:5]
    with encore.Server(ctx, hbm_budget=800_000, n_lanes=2, max_active=8, slice_rows=100_000) as srv:
        ids = [srv.submit(sp["pos"], sp["w"], sp["N"], sp["lmax"], sp["edges"], box=sp["box"],
                          precision=sp["precision"]) for sp in specs]
        res = [srv.wait(j, timeout=120) for j in ids]
        st = srv.stats()
        with pytest.raises(encore.EncoreError) as ei:
            big = np.random.default_rng(0).uniform(0, 50, (20000, 3))
            srv.submit(big, np.ones(20000), 4, 3, specs[0]["edges"], box=50.0)
        assert ei.value.code == encore.ESIZE
    assert st["peak_bytes_held"] <= 800_000
    for (z, t), sp in zip(res, specs):
        assert np.array_equal(z, _alone(ctx, sp))
    # arrival order is kept: admissions are non-decreasing in submit order
    adm = [t["admit"] for _, t in res]
    assert adm == sorted(adm)
