"""Free-molecular closed forms used to pin the oracle (test infrastructure).

Everything is dimensionless: velocities in units of c_mp, forces in units of
the dynamic pressure q = rho U^2 / 2 (so a "force" here is a drag area, m^2),
tau = sqrt(T_w / T_inf) = S / S_W.

Per-element model (Sec. II.B: the influx of momentum integrated over the
free-stream distribution plus the outflux of the re-emission distribution).
For a surface element with outward normal n, free-stream direction U and
gamma = -U.n, s = S gamma, the incident fluxes per unit area are
    number      N_i = chi(s) / (2 sqrt(pi)),   chi(s) = e^{-s^2} + sqrt(pi) s (1 + erf s)
    normal mom. P_i = s e^{-s^2} / (2 sqrt(pi)) + (s^2 + 1/2)(1 + erf s) / 2
    tangential  N_i S (U + gamma n)
(in units of n c_mp and rho c_mp^2).  Diffuse re-emission at T_w returns the
N_i particles with mean normal speed sqrt(pi) tau / 2; specular re-emission
returns P_i and the tangential momentum.  The force per unit area is then
    diffuse   f = -(P_i + N_i sqrt(pi) tau / 2) n + N_i S (U + gamma n)
    specular  f = -2 P_i n
and F / q = (2 / S^2) sum_k A_k f_k.  For a convex body (no shadowing, no
re-hits) this per-facet sum is the exact expectation of the TPMC estimator.

Summed over both faces of a flat plate it gives eq. plate with its last term
halved, sqrt(pi) tau cos^2(alpha) / (... ) -- see ``plate_cd``; integrated over
a sphere it gives eq. sphere exactly.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc

SQRTPI = math.sqrt(math.pi)


def chi(s):
    s = np.asarray(s, dtype=np.float64)
    return np.exp(-s * s) + SQRTPI * s * erfc(-s)


def Z(S: float) -> float:
    """Denominator of g(phi|S) (Sec. III.A.1)."""
    if S < 1e-8:
        return 2.0
    return math.exp(-S * S) + SQRTPI * (S + 0.5 / S) * math.erf(S)


def gamma_hat(S: float, r: float) -> float:
    """Gamma / (n c_mp): number flux into a sphere of radius r (Sec. III.A.1)."""
    if S < 1e-8:
        return 2.0 * SQRTPI * r * r
    return (SQRTPI * math.exp(-S * S) + (math.pi / (2 * S) + math.pi * S) * math.erf(S)) * r * r


def g_phi(phi, S):
    """Incidence-latitude likelihood g(phi|S), transcribed from Sec. III.A.1."""
    phi = np.asarray(phi, dtype=np.float64)
    sp = np.sin(phi)
    num = np.cos(phi) * (np.exp(-S * S * sp * sp) + S * SQRTPI * sp * (1 + erf(S * sp)))
    den = math.exp(-S * S) + SQRTPI * (1 + 2 * S * S) * math.erf(S) / (2 * S)
    return num / den


def p_vn(x, s):
    """eq. vel_dist1 read as p(x|s) = 2 x e^{-(x-s)^2} / chi(s), x = v_n / c_mp >= 0."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(x >= 0, 2 * x * np.exp(-(x - s) ** 2) / chi(s), 0.0)


def mean_vn(s: float) -> float:
    """Mean of p(x|s): [s e^{-s^2} + sqrt(pi)(1/2 + s^2)(1 + erf s)] / chi(s)."""
    return (s * math.exp(-s * s) + SQRTPI * (0.5 + s * s) * math.erfc(-s)) / float(chi(s))


# ---------------------------------------------------------------------------
# per-element force
# ---------------------------------------------------------------------------


def element_force(n_out, U, S, tau, acc):
    """Force per unit area (units rho c_mp^2) on elements with outward normals
    ``n_out`` [k, 3]; ``acc`` = probability of diffuse re-emission."""
    n = np.atleast_2d(np.asarray(n_out, dtype=np.float64))
    U = np.asarray(U, dtype=np.float64)
    g = -(n @ U)
    s = S * g
    Ni = chi(s) / (2 * SQRTPI)
    Pi = s * np.exp(-s * s) / (2 * SQRTPI) + (s * s + 0.5) * erfc(-s) / 2
    Ut = U[None, :] + g[:, None] * n
    f_diff = -(Pi + Ni * SQRTPI * tau / 2)[:, None] * n + (Ni * S)[:, None] * Ut
    f_spec = -(2 * Pi)[:, None] * n
    return acc * f_diff + (1 - acc) * f_spec


def facet_geometry(V, T):
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    v0, v1, v2 = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    cr = np.cross(v1 - v0, v2 - v0)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    n = cr / np.maximum(2 * area, 1e-300)[:, None]
    cen = (v0 + v1 + v2) / 3.0
    return n, area, cen


def mesh_force(V, T, U, S, tau, acc, x_ref=(0.0, 0.0, 0.0), two_sided=False):
    """Per-facet exact F/q and M/q of a body with no shadowing and no re-hits
    (convex closed meshes; both faces of a flat plate with ``two_sided``).
    Returns (F_over_q [3], M_over_q [3], per-facet F_over_q [nt, 3])."""
    n, area, cen = facet_geometry(V, T)
    f = element_force(n, U, S, tau, acc)
    if two_sided:
        f = f + element_force(-n, U, S, tau, acc)
    Fk = (2.0 / (S * S)) * area[:, None] * f
    F = Fk.sum(axis=0)
    M = np.cross(cen - np.asarray(x_ref, dtype=np.float64), Fk).sum(axis=0)
    return F, M, Fk


# ---------------------------------------------------------------------------
# flat plate, sphere, concave hemisphere (Sec. II.B)
# ---------------------------------------------------------------------------


def plate_cd(S, alpha_deg, tau):
    """Double-sided plate, diffuse, A_ref = one-side area, alpha from the normal.
    eq. plate with the re-emission term (pi tau / 2) cos^2(alpha): the printed
    term (pi S / S_W) cos^2(alpha) is twice what the momentum-flux model gives
    (its hyperthermal limit must be 2 + sqrt(pi)/S_W, and only the halved term
    integrates over a sphere to eq. sphere)."""
    a = math.radians(alpha_deg)
    s = S * math.cos(a)
    return 2 / (SQRTPI * S) * (math.exp(-s * s) + SQRTPI * math.cos(a) * (S + 1 / (2 * S)) * math.erf(s)
                               + 0.5 * math.pi * tau * math.cos(a) ** 2)


def plate_cd_printed(S, alpha_deg, tau):
    """eq. plate exactly as printed (kept to document the factor of two)."""
    a = math.radians(alpha_deg)
    s = S * math.cos(a)
    SW = S / tau
    return 2 / (SQRTPI * S) * (math.exp(-s * s) + SQRTPI * S * math.cos(a) * (1 + 1 / (2 * S * S)) * math.erf(s)
                               + math.pi * S / SW * math.cos(a) ** 2)


def plate_cd_specular(S, alpha_deg):
    a = math.radians(alpha_deg)
    s = S * math.cos(a)
    return 4 * math.cos(a) / (S * S) * (s / SQRTPI * math.exp(-s * s) + (0.5 + s * s) * math.erf(s))


def sphere_cd(S, tau):
    """eq. sphere (Bird), A_ref = pi r^2, diffuse; 1/S_W = tau / S."""
    return (math.exp(-S * S) / (SQRTPI * S ** 3) * (1 + 2 * S * S)
            + (4 * S ** 4 + 4 * S * S - 1) / (2 * S ** 4) * math.erf(S)
            + 2 * SQRTPI * tau / (3 * S))


def sphere_cd_specular(S):
    """Specular sphere: eq. sphere without its re-emission term (equal to the
    momentum flux into an absorbing sphere)."""
    return (math.exp(-S * S) / (SQRTPI * S ** 3) * (1 + 2 * S * S)
            + (4 * S ** 4 + 4 * S * S - 1) / (2 * S ** 4) * math.erf(S))


def pratt_cd(S, tau, eps_D=1.05349):
    """eq. hypersphere: concave hemisphere, hyperthermal, full accommodation."""
    return 2.0 + eps_D * SQRTPI * tau / S


def cd_sigma_rule(sigma_rel_sqrtN: float, n: int) -> float:
    return sigma_rel_sqrtN / math.sqrt(n)
