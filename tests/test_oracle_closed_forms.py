"""Pins of the oracle's closed-form pieces (CPU only).

Each test checks an oracle function against something other than itself: the
paper's printed formulas integrated numerically, textbook kinetic-theory
results, analytic limits, or published known-answer vectors.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import closed_forms as CF

GOLD = os.path.join(os.path.dirname(__file__), "golden")
TAU = math.sqrt(0.3)


def test_philox_known_answers(orc):
    """Philox4x32-10 against the published Random123 known-answer vectors."""
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        assert orc.philox(v[0:4], v[4:6]) == v[6:10]


@pytest.mark.parametrize("S", [0.3, 1.0, 2.0, 5.0, 10.0])
def test_gamma_hat_is_the_flux_integral(orc, S):
    """Gamma/(n c_mp) (Sec. III.A.1 final form) against the paper's own
    intermediate integral (eq. integration, velocity part done) over latitude,
    and against pi r^2 <|w|> of a drifting Maxwellian (textbook mean speed,
    integrated here over speed)."""
    r = 1.3
    lib = orc.lib()

    def integrand(phi):
        u = S * math.sin(phi)
        return 0.5 * math.pi * (math.exp(-u * u) + math.sqrt(math.pi) * u * (1 + math.erf(u))) * r * r * math.cos(phi)

    val, _ = integrate.quad(integrand, -math.pi / 2, math.pi / 2, epsabs=1e-13, epsrel=1e-13)
    flux = val * 2 * math.pi / math.pi ** 1.5
    assert lib.orc_gamma_hat(S, r) == pytest.approx(flux, rel=1e-11)

    def speed(v):  # |w| weighted by the drifting Maxwellian, angle integrated analytically
        return 2 / math.sqrt(math.pi) * v ** 2 * math.exp(-(v - S) ** 2) * (1 - math.exp(-4 * S * v)) / (2 * S)

    mean_speed, _ = integrate.quad(speed, 0, S + 40, epsabs=1e-14, epsrel=1e-13, limit=200)
    assert lib.orc_gamma_hat(S, r) == pytest.approx(math.pi * r * r * mean_speed, rel=1e-10)
    assert lib.orc_Z(S) == pytest.approx(lib.orc_gamma_hat(S, r) / (math.sqrt(math.pi) * r * r), rel=1e-14)


def test_gamma_hat_rest_gas(orc):
    """S -> 0: a gas at rest, flux into a sphere = 4 pi r^2 * n c_mp / (2 sqrt(pi))."""
    lib = orc.lib()
    assert lib.orc_gamma_hat(0.0, 2.0) == pytest.approx(4 * math.pi * 4.0 / (2 * math.sqrt(math.pi)), rel=1e-15)
    assert lib.orc_gamma_hat(1e-5, 2.0) == pytest.approx(lib.orc_gamma_hat(0.0, 2.0), rel=1e-9)


@pytest.mark.parametrize("S", [0.05, 0.5, 2.0, 5.0, 10.0])
def test_F_mu_is_the_integral_of_g(orc, S):
    """The oracle's CDF of mu = sin(phi) against quadrature of g(phi|S) as
    printed (Sec. III.A.1), and its inverse."""
    lib = orc.lib()
    tot, _ = integrate.quad(lambda p: CF.g_phi(p, S), -math.pi / 2, math.pi / 2, epsabs=1e-13)
    assert tot == pytest.approx(1.0, abs=1e-10)
    for t in (-0.9, -0.5, -0.1, 0.0, 0.3, 0.7, 0.95):
        ref, _ = integrate.quad(lambda p: CF.g_phi(p, S), -math.pi / 2, math.asin(t), epsabs=1e-14, epsrel=1e-12)
        assert lib.orc_F_mu(t, S) == pytest.approx(ref, abs=1e-11, rel=1e-9)
        u = lib.orc_F_mu(t, S)
        if 1e-9 < u < 1 - 1e-9:
            assert lib.orc_inv_F_mu(u, S) == pytest.approx(t, abs=1e-11)


def test_g_limits():
    """Limits printed in Sec. III.A.1: S -> 0 gives cos(phi)/2; S -> inf gives
    sin(2 phi) for phi >= 0 and 0 below."""
    phi = np.linspace(-1.5, 1.5, 31)
    assert np.allclose(CF.g_phi(phi, 1e-6), 0.5 * np.cos(phi), atol=1e-6)
    big = CF.g_phi(phi, 200.0)
    ref = np.where(phi >= 0, np.sin(2 * phi), 0.0)
    assert np.allclose(big, ref, atol=2e-2)


@pytest.mark.parametrize("s", [-3.0, -1.0, 0.0, 0.7, 4.0, 9.0])
def test_F_n_is_the_integral_of_vel_dist1(orc, s):
    """CDF of the inward normal speed against quadrature of eq. vel_dist1, its
    normalisation and mean, and the inverse."""
    lib = orc.lib()
    tot, _ = integrate.quad(lambda x: float(CF.p_vn(x, s)), 0, max(s, 0) + 12, epsabs=1e-14, limit=200)
    assert tot == pytest.approx(1.0, abs=1e-10)
    mean, _ = integrate.quad(lambda x: x * float(CF.p_vn(x, s)), 0, max(s, 0) + 12, epsabs=1e-14, limit=200)
    assert CF.mean_vn(s) == pytest.approx(mean, rel=1e-9)
    for x in (0.05, 0.4, 1.0, max(s, 0) + 0.3, max(s, 0) + 1.5):
        ref, _ = integrate.quad(lambda y: float(CF.p_vn(y, s)), 0, x, epsabs=1e-15, epsrel=1e-12, limit=200)
        assert lib.orc_F_n(x, s) == pytest.approx(ref, abs=1e-12, rel=1e-9)
        u = lib.orc_F_n(x, s)
        if 1e-9 < u < 1 - 1e-9:
            assert lib.orc_inv_F_n(u, s) == pytest.approx(x, rel=1e-10)


@pytest.mark.parametrize("S", [2.0, 5.0, 10.0])
def test_element_model_integrates_to_eq_sphere(S):
    """The per-element flux model integrated over a sphere (d area = 2 pi r^2
    d gamma) reproduces eq. sphere exactly, and its specular form reproduces
    eq. sphere without the re-emission term."""
    def drag(gamma, acc):
        n = np.array([[-gamma, math.sqrt(max(0.0, 1 - gamma * gamma)), 0.0]])
        return float(CF.element_force(n, np.array([1.0, 0, 0]), S, TAU, acc)[0, 0])

    for acc, ref in ((1.0, CF.sphere_cd(S, TAU)), (0.0, CF.sphere_cd_specular(S))):
        val, _ = integrate.quad(lambda g: drag(g, acc), -1, 1, epsabs=1e-13, epsrel=1e-12)
        assert 4.0 / (S * S) * val == pytest.approx(ref, rel=1e-10)


def test_plate_formula_and_its_printed_form():
    """The double-sided per-element sum equals eq. plate with the re-emission
    term halved; the printed form differs from it by exactly that term; the
    hyperthermal normal-incidence limit is 2 + sqrt(pi)/S_W."""
    import paper_1312_3691_amd.inputs as I
    V, T = I.plate()
    for S in (0.5, 1.0, 3.0, 8.0):
        for a in (0, 20, 45, 70, 90):
            r = math.radians(a)
            U = np.array([math.sin(r), 0, -math.cos(r)])
            F, _, _ = CF.mesh_force(V, T, U, S, TAU, 1.0, two_sided=True)
            assert F @ U == pytest.approx(CF.plate_cd(S, a, TAU), rel=1e-12, abs=1e-14)
            diff = CF.plate_cd_printed(S, a, TAU) - CF.plate_cd(S, a, TAU)
            assert diff == pytest.approx(2 / (math.sqrt(math.pi) * S) * 0.5 * math.pi * TAU * math.cos(r) ** 2, abs=1e-12)
    for S in (1e3, 1e4):  # the next term of the expansion is 1/S^2
        assert abs(CF.plate_cd(S, 0, TAU) - (2 + math.sqrt(math.pi) * TAU / S)) < 1.01 / S ** 2


def test_golden_closed_form_tables_regenerate():
    """closed_forms.json (written by tests/golden/make_golden.py) still matches
    the closed forms, and the icosphere per-facet value sits below eq. sphere
    by the faceting bias."""
    d = json.load(open(os.path.join(GOLD, "closed_forms.json")))
    for row in d["plate"]:
        assert CF.plate_cd(row["S"], row["alpha"], TAU) == pytest.approx(row["cd_diffuse"], rel=1e-12)
        assert CF.plate_cd_specular(row["S"], row["alpha"]) == pytest.approx(row["cd_specular"], rel=1e-12, abs=1e-15)
    for row in d["sphere"]:
        assert CF.sphere_cd(row["S"], TAU) == pytest.approx(row["cd"], rel=1e-12)
    ico = d["icosphere3_S5"]
    assert ico["cd_facet"] == pytest.approx(2.1981704, abs=2e-7)
    assert ico["cd_smooth"] == pytest.approx(2.2086417, abs=2e-7)


def test_fine_icosphere_approaches_eq_sphere():
    import paper_1312_3691_amd.inputs as I
    V, T = I.icosphere(5)
    F, M, _ = CF.mesh_force(V.astype(np.float64), T, (1.0, 0, 0), 5.0, TAU, 1.0)
    assert F[0] / math.pi == pytest.approx(CF.sphere_cd(5.0, TAU), rel=5e-4)
    assert np.allclose(M, 0, atol=1e-9)


def test_golden_bench_cases_regenerate():
    """bench_cases_exact.json (written by tests/golden/make_bench_exact.py, read
    by the benchmark's accuracy report) holds the per-facet closed forms of all
    120 cases: the plate rows equal the corrected eq. plate values (diffuse) and
    the specular plate form, and the cylinder rows match a four-digit table of
    the capped cylinder's per-facet C_D at 0/30/60/90 degrees computed
    independently of the oracle."""
    d = json.load(open(os.path.join(GOLD, "bench_cases_exact.json")))["cases"]
    assert len(d) == 120
    for row in d:
        if row["kind"] == "plate":
            ref = (CF.plate_cd(row["S"], row["angle"], TAU) if row["alpha"] == 1.0
                   else CF.plate_cd_specular(row["S"], row["angle"]))
            assert row["CD"] == pytest.approx(ref, rel=1e-9, abs=1e-12)
    cyl = {(r["S"], r["angle"], r["alpha"]): r["CD"] for r in d if r["kind"] == "cylinder"}
    table = {1.0: ((4.8409, 4.6158), (4.9621, 4.2132), (5.0040, 4.0842), (4.9198, 4.3637)),
             3.0: ((2.4997, 3.3108), (2.8549, 2.6252), (2.9739, 2.3985), (2.7124, 2.8845)),
             8.0: ((1.8972, 3.1611), (2.4870, 2.4072), (2.6394, 2.1627), (2.2285, 2.6968))}
    for S, row in table.items():
        for a, (diffuse, specular) in zip((0.0, 30.0, 60.0, 90.0), row):
            assert cyl[(S, a, 1.0)] == pytest.approx(diffuse, abs=6e-5)
            assert cyl[(S, a, 0.0)] == pytest.approx(specular, abs=6e-5)
