"""The C oracle (oracle/npcf_oracle.c) built with AddressSanitizer +
UndefinedBehaviorSanitizer around a small driver, run on small catalogs (open and
periodic, N = 3..5, a primary subset), with the same results as the ordinary
build on the same thread count."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle.basis import bin_tuples, multiplets

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("oracle_asan") / "oracle_driver")
    subprocess.run(["gcc", "-std=gnu99", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(HERE, "cpp", "oracle_driver.c"), os.path.join(ROOT, "oracle", "npcf_oracle.c"),
                    "-o", exe, "-lm"], check=True)
    return exe


@pytest.mark.parametrize("N,lmax,periodic,subset", [(3, 4, True, False), (4, 2, False, True), (5, 1, True, True)])
def test_oracle_under_sanitizers(tmp_path, driver, N, lmax, periodic, subset):
    rng = np.random.default_rng(N)
    n, L = 300, 40.0
    pos = rng.uniform(0, L, (n, 3))
    w = rng.uniform(-1.0, 1.5, n)
    edges = np.linspace(2.0, 15.0, 5)
    nb = len(edges) - 1
    box = np.full(3, L)
    prim = np.sort(rng.choice(n, 37, replace=False)).astype(np.int64) if subset else np.arange(n, dtype=np.int64)
    t_lam, t_l, t_m, t_c = oracle.term_arrays(N, lmax)
    btab = np.array(bin_tuples(N, nb), dtype=np.int32).reshape(-1, N - 1)
    nlam, nB = len(multiplets(N, lmax)), btab.shape[0]
    nthreads = 2
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(inp, "wb") as f:
        np.array([n, nb, lmax, N - 1, nlam, len(t_lam), nB, len(prim), int(periodic), nthreads],
                 dtype=np.int64).tofile(f)
        for a, dt in [(pos, np.float64), (w, np.float64), (box, np.float64), (edges, np.float64),
                      (t_lam, np.int32), (t_l, np.int32), (t_m, np.int32), (t_c, np.float64), (btab, np.int32),
                      (prim, np.int64)]:
            np.ascontiguousarray(a, dtype=dt).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, inp, out], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    got = np.fromfile(out, dtype=np.float64)
    nout = nlam * nB
    z = got[:4 * nout].reshape(4, nlam, nB)
    alm = got[4 * nout:].reshape(len(prim), nb, oracle.nlm(lmax), 2)
    bx = L if periodic else None
    zc = oracle.zeta(pos, w, N, lmax, edges, box=bx, primaries=prim, nthreads=nthreads, complex_out=True)
    assert np.array_equal(z[0], zc.real) and np.array_equal(z[1], zc.imag)
    ac = oracle.alm(pos, w, lmax, edges, box=bx, primaries=prim, nthreads=nthreads)
    assert np.array_equal(alm[..., 0], ac.real) and np.array_equal(alm[..., 1], ac.imag)
