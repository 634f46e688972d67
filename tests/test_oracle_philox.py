"""Pin the oracle's Philox4x32-10 against rocRAND, an independent implementation.

rocRAND's philox4x32_10 state maps (seed, subsequence, offset) to
key = (seed lo, seed hi) and counter = (offset/4 lo, offset/4 hi,
subsequence lo, subsequence hi); the probe is compiled for the host only.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import philox4x32_10

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND probe")
    exe = str(tmp_path_factory.mktemp("rr") / "probe")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_probe.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return exe


def test_philox_matches_rocrand(probe):
    rng = np.random.default_rng(7)
    cases = []
    for _ in range(300):
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        c = [int(x) for x in rng.integers(0, 2**32, 4, dtype=np.uint64)]
        c[1] &= (1 << 29) - 1  # offset = 4 * (c0 + c1 * 2^32) must fit in 64 bits
        cases.append((seed, c))
    cases += [(0, [0, 0, 0, 0]), (1, [5, 0, 17, (3 << 24) | 2]), (2**64 - 1, [2**32 - 1, 0, 2**32 - 1, 2**32 - 1])]
    inp = "".join("%d %d %d\n" % (s, c[2] + (c[3] << 32), 4 * (c[0] + (c[1] << 32))) for s, c in cases)
    out = subprocess.run([probe], input=inp.encode(), stdout=subprocess.PIPE, check=True).stdout.decode()
    rows = [list(map(int, ln.split())) for ln in out.strip().splitlines()]
    assert len(rows) == len(cases)
    for (seed, c), ref in zip(cases, rows):
        got = philox4x32_10(c, [seed & 0xFFFFFFFF, seed >> 32])
        assert list(map(int, got)) == ref, (seed, c)
