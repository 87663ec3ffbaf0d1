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


@pytest.fixture(scope="module")
def ee_harness(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("exp_erfc") / "harness")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-I", CSRC,
                    os.path.join(ROOT, "tests", "exp_erfc_harness.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def test_exp_erfc_grid_against_40_digits(ee_harness):
    """exp(-y^2) and erfc(y) from the table at y_j = j/256 shifted by the Hermite
    series: within 2 ulp of 40-digit values wherever they are normal doubles
    (the grid points, both ends of every shift, the table's end, random y),
    within one subnormal unit below that, zero above the table; and with too
    few terms the error must show (so the check can fail).  Also the FP32
    erfcx32 of the seeding's approach stage, within 3e-7 relative."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    rng = random.Random(3)
    ys = [0.0, 1e-300, 1e-10, 0.5 / 256, 1 / 256, 27.49, 27.5, 27.6, 30.0, 100.0]
    ys += [j / 256 + d for j in range(0, 7041, 37) for d in (-1 / 512, -1e-9, 0.0, 1e-9, 1 / 512 - 1e-12)]
    ys += [rng.uniform(0, 27.5) for _ in range(3000)] + [rng.uniform(0, 10) for _ in range(3000)]
    ys = [y for y in ys if y >= 0]
    out = subprocess.run([ee_harness], input="\n".join(float(y).hex() for y in ys), capture_output=True, text=True,
                         check=True).stdout
    rows = [[float.fromhex(v) for v in line.split()] for line in out.strip().split("\n")]
    assert len(rows) == len(ys)
    worst = {}
    for y, r in zip(ys, rows):
        ym = mp.mpf(y)
        for k, nterms in enumerate((8, 9, 10, 11)):
            for name, v, exact in (("e", r[2 * k], mp.exp(-ym * ym)), ("erfc", r[2 * k + 1], mp.erfc(ym))):
                if y >= 27.5:
                    err = 0.0 if v == 0.0 else math.inf
                elif float(exact) < 2.2250738585072014e-308:  # subnormal: absolute, in units of 2^-1074
                    err = abs(v - float(exact)) / 5e-324
                else:
                    err = float(abs(mp.mpf(v) - exact) / exact) / 2.0 ** -53
                worst[(nterms, name)] = max(worst.get((nterms, name), 0.0), err)
    for nterms in (10, 11):  # the library uses 10
        assert worst[(nterms, "e")] <= 2.0, worst
        assert worst[(nterms, "erfc")] <= 2.0, worst
    assert worst[(8, "e")] > 100.0, worst  # truncation visible with too few terms
    # erfcx32 (FP32, the seeding's approach stage): within 3e-7 relative of exp(y^2) erfc(y) at the FP32 y
    wx = 0.0
    for r in rows:
        if 0.0 <= r[8] <= 30.0:
            yf = mp.mpf(r[8])
            exact = mp.exp(yf * yf) * mp.erfc(yf)
            wx = max(wx, float(abs(mp.mpf(r[9]) - exact) / exact))
    assert wx <= 3e-7, wx
