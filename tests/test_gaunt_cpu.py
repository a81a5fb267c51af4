"""The library's Gaunt-table builder (gaunt.cpp, host code of the edge correction)
against the oracle's closed forms, built with g++ under AddressSanitizer +
UndefinedBehaviorSanitizer and again under ThreadSanitizer (the table is built on
several threads)."""
import os
import subprocess

import numpy as np
import pytest

from oracle import edge
from oracle.basis import multiplets, parity_E

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2105_08722_amd", "csrc")
CASES = [(3, 4, "all"), (4, 2, "all"), (5, 1, "all"), (5, 2, "even"), (6, 1, "all")]


def _write_oracle(path):
    with open(path, "w") as f:
        for N, lmax, parity in CASES:
            lams = multiplets(N, lmax, parity)
            G = edge.gaunt_tensor(N, lmax, parity)
            E = np.array([parity_E(N, x) for x in lams], dtype=float)
            odd = E < 0
            s = np.where(odd[:, None] & odd[None, :], -1.0, 1.0)
            V = G * s[:, :, None] * E[None, None, :]        # [a, b, c] as a table term holds it
            # exact zeros may come out of the 9j sums as ~1e-18 on either side
            nz = np.argwhere(np.abs(V) > 1e-14 * np.max(np.abs(V)))
            f.write("%d %d %d %d %d\n" % (N, lmax, parity == "all", len(lams), len(nz)))
            for a, b, c in nz:
                f.write("%d %d %d %.17g\n" % (a, b, c, V[a, b, c]))


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_gaunt_table_matches_oracle(tmp_path, san):
    data = str(tmp_path / "gaunt.txt")
    _write_oracle(data)
    exe = str(tmp_path / "test_gaunt")
    srcs = [os.path.join(HERE, "cpp", "test_gaunt.cpp"), os.path.join(CSRC, "gaunt.cpp"),
            os.path.join(CSRC, "tables.cpp")]
    subprocess.run(["g++", "-std=c++20", "-O1", "-g", "-Wall", "-Werror", "-pthread", "-fsanitize=" + san] + srcs +
                   ["-o", exe], check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe, data], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all passed" in r.stdout
