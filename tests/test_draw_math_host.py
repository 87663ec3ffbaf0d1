"""The seeding's logarithm, sine and cosine of a draw (csrc/tpmc_math.hpp),
built for the host and compared with 40-digit values over the range of k
(both ends, powers of two, the sqrt(2) fold, random k): ln u for
u = (k + 1/2) 2^-32 within 1.5 ulp (the largest errors, ~1.4 ulp, sit near
u = 0.7, where -ln 2 and ln m partly cancel), sin and cos of 2 pi u within
2 x 2^-53 absolute.  No GPU is needed."""
import math
import os
import random
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1312_3691_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("draw_math") / "harness")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-I", CSRC,
                    os.path.join(ROOT, "tests", "draw_math_harness.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_draw_math_against_40_digits(harness):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    rng = random.Random(7)
    ks = [0, 1, 2, 3, (1 << 31) - 1, 1 << 31, (1 << 32) - 2, (1 << 32) - 1]
    ks += [(1 << j) + d for j in range(32) for d in (-1, 0, 1) if 0 <= (1 << j) + d < (1 << 32)]
    # around the sqrt(2) fold of the mantissa of n = 2k + 1
    ks += [int(math.sqrt(2) * (1 << j)) // 2 + d for j in range(4, 33) for d in (-1, 0, 1)]
    ks += [rng.getrandbits(32) for _ in range(4000)]
    ks = sorted({k for k in ks if 0 <= k < (1 << 32)})
    out = subprocess.run([harness], input="\n".join(map(str, ks)), capture_output=True, text=True, check=True).stdout
    rows = [[float.fromhex(v) for v in line.split()] for line in out.strip().split("\n")]
    assert len(rows) == len(ks)
    worst = worst_sc = 0.0
    for k, (lg, s, c) in zip(ks, rows):
        u = (mp.mpf(k) + mp.mpf(0.5)) * mp.mpf(2) ** -32
        exact = mp.log(u)
        worst = max(worst, float(abs(mp.mpf(lg) - exact) / math.ulp(abs(float(exact)))))
        # sin and cos multiply unit vectors: absolute error in units of 2^-53
        for v, t in ((s, mp.sin(2 * mp.pi * u)), (c, mp.cos(2 * mp.pi * u))):
            worst_sc = max(worst_sc, float(abs(mp.mpf(v) - t)) / 2.0 ** -53)
    assert worst <= 1.5, worst
    assert worst_sc <= 2.0, worst_sc
