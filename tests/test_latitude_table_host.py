"""Host check of the fine latitude table's design (no GPU).

The seed latitude mu = sin(phi) has density proportional to chi(S mu) on
[-1, 1], chi(s) = exp(-s^2) + sqrt(pi) s (1 + erf s) (the inward flux of the
drifting Maxwellian through a surface element whose normal makes latitude phi
with the stream, Sec. III.A.1).  The library tabulates the root mu(S, u) of
its CDF once per device (rows in ln S, columns in the logit of u) and reads it
through a four-point Lagrange cubic in ln S and linear interpolation in the
logit; the seeding estimate takes that value as it is, and the exact FP64
solve starts from it so that one Halley step ends the solve.  Both rest on
the interpolation being within 1e-5 of the root over the table's S range.

This test takes the layout constants from the library's header, builds the
table entries it needs from roots of the CDF written here in closed form
(integral of chi(S m) dm, derived by parts and checked against quadrature),
and measures the interpolation error at random S and draws.
"""
import math
import os
import re

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import brentq
from scipy.special import erf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1312_3691_amd", "csrc", "tpmc_internal.h")


def _constants():
    text = open(HEADER).read()
    out = {}
    for name in ("kLatFNS", "kLatFNT", "kLatFL0", "kLatFDL", "kLatFT0", "kLatFDT", "kLatFSmin", "kLatFSmax"):
        m = re.search(r"\b%s\s*=\s*([-0-9.eE/ f]+?)[,;]" % name, text)
        assert m, name
        out[name] = float(eval(m.group(1).replace("f", "")))  # e.g. "1.0f / 64.0f"
    return out


def _chi(s):
    return math.exp(-s * s) + math.sqrt(math.pi) * s * (1.0 + math.erf(s))


def _F(m, S):
    """An antiderivative of chi(S m) in m."""
    e = math.exp(-(S * m) ** 2)
    return (math.sqrt(math.pi) / (2.0 * S) * erf(S * m)
            + math.sqrt(math.pi) * S * (0.5 * m * m + (0.5 * m * m - 0.25 / (S * S)) * erf(S * m)) + 0.5 * m * e)


def _root(S, u):
    lo = _F(-1.0, S)
    Z = _F(1.0, S) - lo
    return brentq(lambda m: (_F(m, S) - lo) - u * Z, -1.0, 1.0, xtol=1e-15, rtol=1e-15)


def test_antiderivative_matches_quadrature():
    for S in (0.3, 1.0, 4.0, 9.5):
        for a, b in ((-1.0, -0.2), (-0.5, 0.7), (0.1, 1.0)):
            q, _ = quad(lambda m: _chi(S * m), a, b, epsabs=1e-13, epsrel=1e-13)
            assert _F(b, S) - _F(a, S) == pytest.approx(q, rel=1e-11, abs=1e-13)


def test_fine_table_interpolation_error_below_1e5():
    c = _constants()
    ns, nt = int(c["kLatFNS"]), int(c["kLatFNT"])
    L0, DL, T0, DT = c["kLatFL0"], c["kLatFDL"], c["kLatFT0"], c["kLatFDT"]
    # the S range it serves has all four rows inside the table
    for S in (c["kLatFSmin"], c["kLatFSmax"]):
        i = math.floor((math.log(S) - L0) / DL)
        assert i - 1 >= 0 and i + 2 <= ns - 1, S
    rng = np.random.default_rng(20131216)
    cache = {}

    def entry(i, j):  # table entries are stored in FP32
        if (i, j) not in cache:
            S = math.exp(L0 + i * DL)
            t = T0 + j * DT
            cache[(i, j)] = float(np.float32(_root(S, 1.0 / (1.0 + math.exp(-t)))))
        return cache[(i, j)]

    worst = 0.0
    for n in range(240):
        S = math.exp(math.log(c["kLatFSmin"]) + rng.random() * math.log(c["kLatFSmax"] / c["kLatFSmin"]))
        if n % 4 == 0:  # draws towards the ends (the far tails, u < 1e-6, are left out: there the
            u = 10.0 ** rng.uniform(-6.0, -2.0)  # CDF's cancellation in FP64 exceeds the bar)
            u = 1.0 - u if rng.random() < 0.5 else u
        else:
            u = rng.random()
        pos = (math.log(S) - L0) / DL
        i = math.floor(pos)
        f = pos - i
        w = (-f * (f - 1) * (f - 2) / 6, (f + 1) * (f - 1) * (f - 2) / 2, -(f + 1) * f * (f - 2) / 2,
             (f + 1) * f * (f - 1) / 6)
        t = math.log(u) - math.log1p(-u)
        ft = min(max((t - T0) / DT, 0.0), nt - 1.0)
        j = min(int(ft), nt - 2)
        b = ft - j
        est = sum(w[k] * ((1 - b) * entry(i - 1 + k, j) + b * entry(i - 1 + k, j + 1)) for k in range(4))
        worst = max(worst, abs(est - _root(S, u)))
    assert worst < 1e-5, worst
