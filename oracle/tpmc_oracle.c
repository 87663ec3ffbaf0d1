/*
 * tpmc_oracle.c -- FP64 CPU oracle of the TPMC drag hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see tpmc_oracle.h).  Plain, slow and written for a
 * reader checking it against the paper: every inverse CDF is solved by pure
 * bisection, every ray is tested against every triangle (or, for large meshes,
 * against the triangles of every box of a plain median-split hierarchy that it
 * enters; same closest hit), every sum is a Neumaier-compensated FP64 sum.  Nothing here is shared with the GPU path.
 *
 * Paper: J. B. Parham and L. A. Barba, "Finding the Force -- Consistent
 * Particle Seeding for Satellite Aerodynamics", AIAA.
 */
#include "tpmc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_SQRTPI 1.77245385090551602730

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, from its published definition (Salmon et al., SC'11):       */
/* ten rounds of two 32x32->64 multiplies, the key bumped by the Weyl         */
/* constants between rounds.                                                  */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Four words of the stream of particle pid at step `step`.
 * Counter = (pid lo, pid hi, step, 0), key = (seed lo, seed hi). */
static void orc_stream(uint64_t seed, uint64_t pid, uint32_t step, uint32_t out[4]) {
  uint32_t ctr[4] = {(uint32_t)pid, (uint32_t)(pid >> 32), step, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

/* Uniform variates in (0, 1), exact in their type.
 * Seeding (FP64 path): u = (k + 1/2) 2^-32.  Reflection (FP32 path):
 * u = (floor(k / 2^9) + 1/2) 2^-23. */
static double u64_of(uint32_t k) { return ((double)k + 0.5) * 0x1p-32; }
static double u32_of(uint32_t k) { return ((double)(k >> 9) + 0.5) * 0x1p-23; }

/* ------------------------------------------------------------------------- */
/* Compensated summation (Neumaier's improvement of Kahan summation).         */
/* ------------------------------------------------------------------------- */
static void nsum(double* s, double* c, double x) {
  double t = *s + x;
  if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
  else *c += (x - t) + *s;
  *s = t;
}

/* ------------------------------------------------------------------------- */
/* Seeding model, Sec. III.A.1-2.                                              */
/* ------------------------------------------------------------------------- */

/* chi(s) = e^{-s^2} + sqrt(pi) s (1 + erf s): the bracket of the per-area
 * inward number flux (eq. integration) and the normaliser of eq. vel_dist1.
 * 1 + erf s is written erfc(-s) so that it stays accurate for s < 0. */
double orc_chi(double s) { return exp(-s * s) + ORC_SQRTPI * s * erfc(-s); }

/* Z(S) = e^{-S^2} + sqrt(pi)(S + 1/(2S)) erf S: the denominator of g(phi|S)
 * (Sec. III.A.1).  Its S -> 0 limit is 2. */
double orc_Z(double S) {
  if (S < 1e-8) return 2.0;
  return exp(-S * S) + ORC_SQRTPI * (S + 0.5 / S) * erf(S);
}

/* Gamma / (n c_mp) = [sqrt(pi) e^{-S^2} + (pi/(2S) + pi S) erf S] r^2, the
 * number flux into a sphere of radius r (Sec. III.A.1, final Gamma result).
 * It equals sqrt(pi) r^2 Z(S); at S = 0 it is 2 sqrt(pi) r^2. */
double orc_gamma_hat(double S, double r) {
  if (S < 1e-8) return 2.0 * ORC_SQRTPI * r * r;
  return (ORC_SQRTPI * exp(-S * S) + (ORC_PI / (2.0 * S) + ORC_PI * S) * erf(S)) * r * r;
}

/* Unnormalised CDF of mu = sin(phi) under g(phi|S) (Sec. III.A.1):
 * with d(mu) = cos(phi) d(phi), the density of mu on [-1, 1] is chi(S mu) / Z(S),
 * so G(t) = integral_{-1}^{t} chi(S mu) d(mu) and G(1) = Z(S).  Antiderivative:
 *   H(t) = sqrt(pi)/(4S) erf(St) + sqrt(pi) S t^2 (1 + erf St) / 2 + t e^{-S^2 t^2} / 2,
 * evaluated as G(t) = H(t) - H(-1) term by term so that no term cancels. */
static double orc_G_mu(double t, double S) {
  double St = S * t;
  double e_diff; /* erf(S t) - erf(-S) */
  if (t < 0.0 && -St > 1.0) e_diff = erfc(-St) - erfc(S);
  else e_diff = erf(St) + erf(S);
  double term1 = ORC_SQRTPI / (4.0 * S) * e_diff;
  double term2 = 0.5 * ORC_SQRTPI * S * (t * t * erfc(-St) - erfc(S));
  double term3 = 0.5 * (t * exp(-St * St) + exp(-S * S));
  return term1 + term2 + term3;
}

double orc_F_mu(double t, double S) {
  if (t <= -1.0) return 0.0;
  if (t >= 1.0) return 1.0;
  if (S < 1e-8) return 0.5 * (t + 1.0); /* S -> 0: g -> cos(phi)/2, mu uniform */
  return orc_G_mu(t, S) / orc_Z(S);
}

/* Inverse of F_mu by bisection on [-1, 1] until the bracket stops shrinking. */
double orc_inv_F_mu(double u, double S) {
  if (S < 1e-8) return 2.0 * u - 1.0;
  double target = u * orc_Z(S);
  double lo = -1.0, hi = 1.0;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (orc_G_mu(mid, S) < target) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* CDF of the inward normal speed x = v_n / c_mp >= 0 of eq. vel_dist1, read as
 * p(x | s) = 2 x e^{-(x - s)^2} / chi(s) (the printed "2 v_i" taken as 2x in
 * units of c_mp, the only reading that integrates to 1):
 *   F_n(x|s) = [e^{-s^2} - e^{-(x-s)^2} + sqrt(pi) s (erf(x-s) + erf s)] / chi(s),
 * with erf(x-s) + erf(s) written as a difference of two small erfc values
 * wherever the plain sum would cancel. */
static double orc_Fn_num(double x, double s) {
  double a = x - s;
  double e_sum; /* erf(x - s) + erf(s) */
  if (s < 0.0) e_sum = erfc(-s) - erfc(a);
  else if (a < 0.0) e_sum = erfc(-a) - erfc(s);
  else e_sum = erf(a) + erf(s);
  return exp(-s * s) - exp(-a * a) + ORC_SQRTPI * s * e_sum;
}

double orc_F_n(double x, double s) {
  if (x <= 0.0) return 0.0;
  return orc_Fn_num(x, s) / orc_chi(s);
}

double orc_inv_F_n(double u, double s) {
  double target = u * orc_chi(s);
  double lo = 0.0, hi = (s > 0.0 ? s : 0.0) + 7.0;
  while (orc_Fn_num(hi, s) < target) hi *= 2.0;
  for (int it = 0; it < 400; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (orc_Fn_num(mid, s) < target) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------------------- */
/* Query constants.                                                            */
/* ------------------------------------------------------------------------- */
int orc_setup(const orc_query* q, const double* V, uint64_t nv, orc_consts* c) {
  memset(c, 0, sizeof(*c));
  double w = q->q_wxyz[0], x = q->q_wxyz[1], y = q->q_wxyz[2], z = q->q_wxyz[3];
  double n = sqrt(w * w + x * x + y * y + z * z);
  if (!(n > 0.0)) return 1;
  w /= n; x /= n; y /= n; z /= n;
  /* R(q) maps body to wind axes; its rows are the wind axes in the body frame:
   * U = R^T x_hat, e1 = R^T y_hat, e2 = R^T z_hat.  This frame replaces the
   * Rodrigues rotation of Sec. III.A.3 (same distribution, no degenerate axis). */
  c->U[0] = 1.0 - 2.0 * (y * y + z * z);
  c->U[1] = 2.0 * (x * y - w * z);
  c->U[2] = 2.0 * (x * z + w * y);
  c->e1[0] = 2.0 * (x * y + w * z);
  c->e1[1] = 1.0 - 2.0 * (x * x + z * z);
  c->e1[2] = 2.0 * (y * z - w * x);
  c->e2[0] = 2.0 * (x * z - w * y);
  c->e2[1] = 2.0 * (y * z + w * x);
  c->e2[2] = 1.0 - 2.0 * (x * x + y * y);

  c->S = q->S;
  c->s_zero = q->S < 1e-8;
  c->tau = sqrt(q->T_w / q->T_inf);
  c->alpha = q->alpha;
  c->N = q->n_particles;
  c->seed = q->seed;
  c->rmax = q->max_reflections;
  c->round_fp32 = q->round_fp32;
  c->eacc = q->energy_acc ? 1 : 0;
  c->alpha_E = q->energy_acc ? q->alpha_E : 1.0;

  if (q->cv_box) {
    /* Box control volume (the rectangular CV of Sec. III.A, seeded correctly):
     * the cube of half-side cv_radius about cv_center, or with cv_radius <= 0
     * the vertex box widened on every axis by 1e-3 of its half-diagonal.  The
     * inflow through face f (area A_f, inward normal n_f) is the one-sided
     * flux of the drifting Maxwellian, A_f chi(s_f) / (2 sqrt(pi)) per n c_mp
     * with s_f = S U.n_f (the sphere's flux density at latitude sin(phi) =
     * U.n), so Gamma_hat = sum_f A_f chi(s_f) / (2 sqrt(pi)). */
    c->box = 1;
    if (q->cv_radius > 0.0) {
      for (int k = 0; k < 3; ++k) {
        c->c0[k] = q->cv_center[k];
        c->h[k] = q->cv_radius;
      }
    } else {
      double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (uint64_t i = 0; i < nv; ++i)
        for (int k = 0; k < 3; ++k) {
          if (V[3 * i + k] < lo[k]) lo[k] = V[3 * i + k];
          if (V[3 * i + k] > hi[k]) hi[k] = V[3 * i + k];
        }
      double hd = 0.0;
      for (int k = 0; k < 3; ++k) {
        c->c0[k] = 0.5 * (lo[k] + hi[k]);
        c->h[k] = 0.5 * (hi[k] - lo[k]);
        hd += c->h[k] * c->h[k];
      }
      hd = sqrt(hd);
      for (int k = 0; k < 3; ++k) c->h[k] += 1e-3 * hd;
    }
    c->r = sqrt(c->h[0] * c->h[0] + c->h[1] * c->h[1] + c->h[2] * c->h[2]);
    double cum = 0.0;
    for (int f = 0; f < 6; ++f) {
      int k = f / 2, j = (k + 1) % 3, l = (k + 2) % 3;
      double n_k = (f % 2 == 0) ? 1.0 : -1.0; /* inward normal of the face at c0[k] -/+ h[k] */
      double s_f = c->s_zero ? 0.0 : q->S * c->U[k] * n_k;
      c->face_s[f] = s_f;
      cum += 4.0 * c->h[j] * c->h[l] * orc_chi(s_f);
      c->face_cum[f] = cum;
    }
    c->Z = orc_Z(c->S);
    c->Gamma_hat = cum / (2.0 * ORC_SQRTPI);
    return 0;
  }
  if (q->cv_radius > 0.0) {
    for (int k = 0; k < 3; ++k) c->c0[k] = q->cv_center[k];
    c->r = q->cv_radius;
  } else {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint64_t i = 0; i < nv; ++i)
      for (int k = 0; k < 3; ++k) {
        if (V[3 * i + k] < lo[k]) lo[k] = V[3 * i + k];
        if (V[3 * i + k] > hi[k]) hi[k] = V[3 * i + k];
      }
    for (int k = 0; k < 3; ++k) c->c0[k] = 0.5 * (lo[k] + hi[k]);
    double rr = 0.0;
    for (uint64_t i = 0; i < nv; ++i) {
      double d0 = V[3 * i] - c->c0[0], d1 = V[3 * i + 1] - c->c0[1], d2 = V[3 * i + 2] - c->c0[2];
      double d = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      if (d > rr) rr = d;
    }
    c->r = rr * (1.0 + 1e-3);
  }
  c->Z = orc_Z(c->S);
  c->Gamma_hat = orc_gamma_hat(c->S, c->r);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Seeding one particle, Sec. III.A.1-3.                                       */
/* ------------------------------------------------------------------------- */
/* Box CV: the face by its share of the inflow, the point uniform on the face,
 * the velocity from the same flux-weighted drifting distribution as on the
 * sphere with s_n = s_f, tangential components Gaussian about the tangential
 * drift S U_j, S U_l (face axes j, l). */
static void orc_seed_box(const orc_consts* c, const uint32_t r0[4], const uint32_t r1[4], double x[3],
                         double wv[3], double* mu_out) {
  double u0 = u64_of(r0[0]), u1 = u64_of(r0[1]), u2 = u64_of(r0[2]), u3 = u64_of(r0[3]);
  double u4 = u64_of(r1[0]), u5 = u64_of(r1[1]);
  double t = u0 * c->face_cum[5];
  int f = 0;
  while (f < 5 && !(t < c->face_cum[f])) ++f;
  int k = f / 2, j = (k + 1) % 3, l = (k + 2) % 3;
  double n_k = (f % 2 == 0) ? 1.0 : -1.0;
  x[k] = c->c0[k] - n_k * c->h[k];
  x[j] = c->c0[j] + (2.0 * u1 - 1.0) * c->h[j];
  x[l] = c->c0[l] + (2.0 * u5 - 1.0) * c->h[l];
  double wn = orc_inv_F_n(u2, c->face_s[f]);
  double rad = sqrt(-2.0 * log(u3));
  double g1 = rad * cos(2.0 * ORC_PI * u4);
  double g2 = rad * sin(2.0 * ORC_PI * u4);
  wv[k] = wn * n_k;
  wv[j] = c->S * c->U[j] + g1 / sqrt(2.0);
  wv[l] = c->S * c->U[l] + g2 / sqrt(2.0);
  if (c->round_fp32) {
    for (int m = 0; m < 3; ++m) {
      x[m] = (double)(float)x[m];
      wv[m] = (double)(float)wv[m];
    }
  }
  if (mu_out) *mu_out = c->U[k] * n_k;
}

static void orc_seed_one(const orc_consts* c, uint64_t pid, double x[3], double wv[3], double* mu_out) {
  uint32_t r0[4], r1[4];
  orc_stream(c->seed, pid, 0u, r0);
  orc_stream(c->seed, pid, 1u, r1);
  if (c->box) {
    orc_seed_box(c, r0, r1, x, wv, mu_out);
    return;
  }
  double u0 = u64_of(r0[0]), u1 = u64_of(r0[1]), u2 = u64_of(r0[2]), u3 = u64_of(r0[3]);
  double u4 = u64_of(r1[0]);

  /* Position: latitude from g(phi|S) via mu = sin(phi), longitude uniform. */
  double mu = c->s_zero ? 2.0 * u0 - 1.0 : orc_inv_F_mu(u0, c->S);
  double a = sqrt(fmax(0.0, 1.0 - mu * mu)); /* cos(phi) */
  double th = 2.0 * ORC_PI * u1;
  double ct = cos(th), st = sin(th);
  double cvec[3], dvec[3], nhat[3], t1[3], t2[3];
  for (int k = 0; k < 3; ++k) {
    cvec[k] = ct * c->e1[k] + st * c->e2[k];
    dvec[k] = -st * c->e1[k] + ct * c->e2[k];
  }
  /* Inward normal n = mu U - cos(phi) c, so that U.n = mu = sin(phi): the point
   * x = c0 - r n lies upstream for mu > 0.  t1 is the unit tangent along the
   * tangential part of U, t1 = (U - mu n)/cos(phi) = cos(phi) U + mu c, and
   * t2 = t1 x n = -(U x c) = -d. */
  for (int k = 0; k < 3; ++k) {
    nhat[k] = mu * c->U[k] - a * cvec[k];
    t1[k] = a * c->U[k] + mu * cvec[k];
    t2[k] = -dvec[k];
    x[k] = c->c0[k] - c->r * nhat[k];
  }

  /* Velocity, eqs. vel_dist1-3: the inward normal component from the
   * flux-weighted drifting distribution with S_n = S sin(phi), the tangential
   * components Gaussian (variance 1/2 in units of c_mp^2) about S_t1 = S cos(phi)
   * and S_t2 = 0. */
  double s_n = c->S * mu;
  double wn = orc_inv_F_n(u2, s_n);
  double rad = sqrt(-2.0 * log(u3));
  double g1 = rad * cos(2.0 * ORC_PI * u4);
  double g2 = rad * sin(2.0 * ORC_PI * u4);
  double wt1 = c->S * a + g1 / sqrt(2.0);
  double wt2 = g2 / sqrt(2.0);
  /* Back to body axes by the transpose of the local frame matrix (Sec. III.A.3). */
  for (int k = 0; k < 3; ++k) wv[k] = wn * nhat[k] + wt1 * t1[k] + wt2 * t2[k];

  if (c->round_fp32) {
    for (int k = 0; k < 3; ++k) {
      x[k] = (double)(float)x[k];
      wv[k] = (double)(float)wv[k];
    }
  }
  if (mu_out) *mu_out = mu;
}

void orc_seed_range(const orc_consts* c, uint64_t p0, uint64_t p1, double* x, double* w, double* mu) {
  for (uint64_t p = p0; p < p1; ++p) {
    uint64_t i = p - p0;
    orc_seed_one(c, p, x + 3 * i, w + 3 * i, mu ? mu + i : 0);
  }
}

/* ------------------------------------------------------------------------- */
/* Gas-surface interaction (Sec. II.A): Maxwell model, diffuse with            */
/* probability alpha, else specular.                                           */
/* ------------------------------------------------------------------------- */
void orc_reflect(const orc_consts* c, uint64_t pid, uint32_t b, const double w_in[3],
                 const double n_g[3], double w_out[3]) {
  uint32_t r[4];
  orc_stream(c->seed, pid, 2u + b, r);
  double ua = u32_of(r[0]), ub = u32_of(r[1]), uc = u32_of(r[2]), ud = u32_of(r[3]);
  double wn = w_in[0] * n_g[0] + w_in[1] * n_g[1] + w_in[2] * n_g[2];
  if (ua < c->alpha) {
    /* Diffuse: the particle leaves from the side it arrived on, with the
     * flux-weighted half-range Maxwellian of the wall temperature: normal
     * speed tau sqrt(-ln u) (eq. vel_dist1 with S_n = 0, c_mp -> c_w) and
     * Gaussian tangential components of variance tau^2 / 2. */
    double ns[3];
    double sg = wn < 0.0 ? 1.0 : -1.0;
    for (int k = 0; k < 3; ++k) ns[k] = sg * n_g[k];
    /* Orthonormal tangents of ns (Duff et al., JCGT 2017). */
    double sign = ns[2] >= 0.0 ? 1.0 : -1.0;
    double aa = -1.0 / (sign + ns[2]);
    double bb = ns[0] * ns[1] * aa;
    double b1[3] = {1.0 + sign * ns[0] * ns[0] * aa, sign * bb, -sign * ns[0]};
    double b2[3] = {bb, sign + ns[1] * ns[1] * aa, -ns[1]};
    /* With energy accommodation alpha_E (the "momentum and energy" exchange of
     * Sec. I; Sentman's definition alpha_E = (E_i - E_r)/(E_i - E_w)), the
     * molecule leaves diffusely at the temperature whose flux-weighted mean
     * energy 2kT_r is E_r = (1 - alpha_E) E_i + alpha_E 2kT_w, i.e.
     * tau_r^2 = alpha_E tau^2 + (1 - alpha_E) |w|^2 / 2 per molecule. */
    double tr = c->tau;
    if (c->eacc) {
      double e_in = w_in[0] * w_in[0] + w_in[1] * w_in[1] + w_in[2] * w_in[2];
      tr = sqrt(c->alpha_E * c->tau * c->tau + (1.0 - c->alpha_E) * 0.5 * e_in);
    }
    double vn = tr * sqrt(-log(ub));
    double rad = sqrt(-2.0 * log(uc));
    double g1 = rad * cos(2.0 * ORC_PI * ud), g2 = rad * sin(2.0 * ORC_PI * ud);
    double v1 = tr * g1 / sqrt(2.0), v2 = tr * g2 / sqrt(2.0);
    for (int k = 0; k < 3; ++k) w_out[k] = vn * ns[k] + v1 * b1[k] + v2 * b2[k];
  } else {
    /* Specular: mirror the normal component. */
    for (int k = 0; k < 3; ++k) w_out[k] = w_in[k] - 2.0 * wn * n_g[k];
  }
}

/* ------------------------------------------------------------------------- */
/* Ray-triangle test (Sec. II.A: closest intersection on a triangulation).     */
/* Watertight formulation of Woop, Benthin & Wald (JCGT 2013), two-sided.      */
/* ------------------------------------------------------------------------- */
int orc_intersect(const double o[3], const double d[3], const double v0[3], const double v1[3],
                  const double v2[3], double* t_out, double b[3]) {
  int kz = 0;
  if (fabs(d[1]) > fabs(d[kz])) kz = 1;
  if (fabs(d[2]) > fabs(d[kz])) kz = 2;
  if (d[kz] == 0.0) return 0;
  int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
  if (d[kz] < 0.0) { int tmp = kx; kx = ky; ky = tmp; }
  double Sx = d[kx] / d[kz], Sy = d[ky] / d[kz], Sz = 1.0 / d[kz];
  double A[3], B[3], C[3];
  for (int k = 0; k < 3; ++k) { A[k] = v0[k] - o[k]; B[k] = v1[k] - o[k]; C[k] = v2[k] - o[k]; }
  double Ax = A[kx] - Sx * A[kz], Ay = A[ky] - Sy * A[kz];
  double Bx = B[kx] - Sx * B[kz], By = B[ky] - Sy * B[kz];
  double Cx = C[kx] - Sx * C[kz], Cy = C[ky] - Sy * C[kz];
  double U = Cx * By - Cy * Bx;
  double Vv = Ax * Cy - Ay * Cx;
  double W = Bx * Ay - By * Ax;
  if ((U < 0.0 || Vv < 0.0 || W < 0.0) && (U > 0.0 || Vv > 0.0 || W > 0.0)) return 0;
  double det = U + Vv + W;
  if (det == 0.0) return 0;
  double T = U * (Sz * A[kz]) + Vv * (Sz * B[kz]) + W * (Sz * C[kz]);
  double t = T / det;
  if (!(t > 0.0)) return 0;
  *t_out = t;
  b[0] = U / det; b[1] = Vv / det; b[2] = W / det;
  return 1;
}

/* ------------------------------------------------------------------------- */
/* Closest hit on the triangulation (Sec. II.A), by brute force or through a   */
/* plain bounding-volume hierarchy.                                            */
/* ------------------------------------------------------------------------- */
/* Hierarchy: median split.  A node's triangles are split at the median of     */
/* their centroids along the axis where the centroids spread most (ties in the */
/* centroid go by triangle index); a leaf holds at most 4 triangles.  Every box */
/* is the union of its triangles' vertex boxes widened by a margin far above   */
/* FP64 rounding.  The hierarchy only prunes: a box is skipped when the ray    */
/* misses it or enters it beyond the best t found so far (with a relative      */
/* slack), and candidates are ranked by (t, index) exactly as the brute-force  */
/* loop ranks them, so both return the same triangle, t and barycentrics.      */
struct orc_bvh {
  uint64_t n_nodes;
  double* lo;        /* [n_nodes][3] widened box */
  double* hi;
  int64_t* child;    /* [n_nodes][2]: child node ids; {-1, -1} for a leaf */
  uint64_t* first;   /* leaf: first position in idx */
  uint32_t* count;   /* leaf: number of triangles */
  uint32_t* idx;     /* triangle indices in leaf order */
};

typedef struct {
  double key;
  uint32_t tri;
} orc_key;

static int orc_key_cmp(const void* a, const void* b) {
  const orc_key* x = (const orc_key*)a;
  const orc_key* y = (const orc_key*)b;
  if (x->key < y->key) return -1;
  if (x->key > y->key) return 1;
  return (x->tri > y->tri) - (x->tri < y->tri);
}

static uint64_t bvh_node(orc_bvh* h, const double* V, const uint32_t* T, orc_key* keys, uint64_t a, uint64_t b,
                         double pad) {
  uint64_t id = h->n_nodes++;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (uint64_t i = a; i < b; ++i) {
    uint32_t k = h->idx[i];
    for (int j = 0; j < 3; ++j) {
      double c = 0.0;
      for (int v = 0; v < 3; ++v) {
        double x = V[3 * (uint64_t)T[3 * (uint64_t)k + v] + j];
        if (x < lo[j]) lo[j] = x;
        if (x > hi[j]) hi[j] = x;
        c += x;
      }
      c /= 3.0;
      if (c < clo[j]) clo[j] = c;
      if (c > chi[j]) chi[j] = c;
    }
  }
  for (int j = 0; j < 3; ++j) {
    h->lo[3 * id + j] = lo[j] - pad;
    h->hi[3 * id + j] = hi[j] + pad;
  }
  if (b - a <= 4) {
    h->child[2 * id] = h->child[2 * id + 1] = -1;
    h->first[id] = a;
    h->count[id] = (uint32_t)(b - a);
    return id;
  }
  int axis = 0;
  for (int j = 1; j < 3; ++j)
    if (chi[j] - clo[j] > chi[axis] - clo[axis]) axis = j;
  for (uint64_t i = a; i < b; ++i) {
    uint32_t k = h->idx[i];
    double c = 0.0;
    for (int v = 0; v < 3; ++v) c += V[3 * (uint64_t)T[3 * (uint64_t)k + v] + axis];
    keys[i].key = c / 3.0;
    keys[i].tri = k;
  }
  qsort(keys + a, b - a, sizeof(orc_key), orc_key_cmp);
  for (uint64_t i = a; i < b; ++i) h->idx[i] = keys[i].tri;
  uint64_t m = a + (b - a) / 2;
  h->first[id] = 0;
  h->count[id] = 0;
  int64_t l = (int64_t)bvh_node(h, V, T, keys, a, m, pad);
  int64_t r = (int64_t)bvh_node(h, V, T, keys, m, b, pad);
  h->child[2 * id] = l;
  h->child[2 * id + 1] = r;
  return id;
}

orc_bvh* orc_bvh_build(const double* V, uint64_t nv, const uint32_t* T, uint64_t nt) {
  if (nt == 0) return NULL;
  orc_bvh* h = (orc_bvh*)calloc(1, sizeof(orc_bvh));
  uint64_t cap = 2 * nt;
  h->lo = (double*)malloc(3 * cap * sizeof(double));
  h->hi = (double*)malloc(3 * cap * sizeof(double));
  h->child = (int64_t*)malloc(2 * cap * sizeof(int64_t));
  h->first = (uint64_t*)malloc(cap * sizeof(uint64_t));
  h->count = (uint32_t*)malloc(cap * sizeof(uint32_t));
  h->idx = (uint32_t*)malloc(nt * sizeof(uint32_t));
  orc_key* keys = (orc_key*)malloc(nt * sizeof(orc_key));
  double amax = 0.0;
  for (uint64_t i = 0; i < 3 * nv; ++i)
    if (fabs(V[i]) > amax) amax = fabs(V[i]);
  for (uint64_t k = 0; k < nt; ++k) h->idx[k] = (uint32_t)k;
  bvh_node(h, V, T, keys, 0, nt, 1e-9 * (1.0 + amax));
  free(keys);
  return h;
}

void orc_bvh_free(orc_bvh* h) {
  if (!h) return;
  free(h->lo); free(h->hi); free(h->child); free(h->first); free(h->count); free(h->idx);
  free(h);
}

uint64_t orc_bvh_nodes(const orc_bvh* h) { return h ? h->n_nodes : 0; }

/* Whether the ray o + t d (t >= 0) meets box `id` no later than t_max. */
static int bvh_box_hit(const orc_bvh* h, uint64_t id, const double o[3], const double d[3], double t_max) {
  double tn = 0.0, tf = INFINITY;
  for (int j = 0; j < 3; ++j) {
    double lo = h->lo[3 * id + j], hi = h->hi[3 * id + j];
    if (d[j] == 0.0) {
      if (o[j] < lo || o[j] > hi) return 0;
      continue;
    }
    double t0 = (lo - o[j]) / d[j], t1 = (hi - o[j]) / d[j];
    if (t0 > t1) { double tmp = t0; t0 = t1; t1 = tmp; }
    if (t0 > tn) tn = t0;
    if (t1 < tf) tf = t1;
  }
  return tn <= tf && tn <= t_max * (1.0 + 1e-7);
}

static void tri_verts(const double* V, const uint32_t* T, uint64_t k, double v0[3], double v1[3], double v2[3]) {
  for (int j = 0; j < 3; ++j) {
    v0[j] = V[3 * (uint64_t)T[3 * k + 0] + j];
    v1[j] = V[3 * (uint64_t)T[3 * k + 1] + j];
    v2[j] = V[3 * (uint64_t)T[3 * k + 2] + j];
  }
}

/* Candidate k for the closest hit: t > 0, the triangle just left excluded;
 * a smaller t wins, equal t goes to the lower index. */
static void closest_consider(const double* V, const uint32_t* T, uint64_t k, int64_t prev, const double o[3],
                             const double d[3], int64_t* best, double* best_t, double best_b[3]) {
  if ((int64_t)k == prev) return;
  double v0[3], v1[3], v2[3], t, b[3];
  tri_verts(V, T, k, v0, v1, v2);
  if (!orc_intersect(o, d, v0, v1, v2, &t, b)) return;
  if (t < *best_t || (t == *best_t && (int64_t)k < *best)) {
    *best_t = t;
    *best = (int64_t)k;
    best_b[0] = b[0]; best_b[1] = b[1]; best_b[2] = b[2];
  }
}

int64_t orc_closest(const double* V, const uint32_t* T, uint64_t nt, const orc_bvh* bvh, const double o[3],
                    const double d[3], int64_t prev, double* t_out, double b_out[3]) {
  int64_t best = -1;
  double best_t = INFINITY;
  double best_b[3] = {0.0, 0.0, 0.0};
  if (!bvh) {
    for (uint64_t k = 0; k < nt; ++k) closest_consider(V, T, k, prev, o, d, &best, &best_t, best_b);
  } else {
    uint64_t stack[128];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
      uint64_t id = stack[--sp];
      if (!bvh_box_hit(bvh, id, o, d, best_t)) continue;
      if (bvh->child[2 * id] < 0) {
        for (uint32_t i = 0; i < bvh->count[id]; ++i)
          closest_consider(V, T, bvh->idx[bvh->first[id] + i], prev, o, d, &best, &best_t, best_b);
      } else {
        stack[sp++] = (uint64_t)bvh->child[2 * id + 1];
        stack[sp++] = (uint64_t)bvh->child[2 * id];
      }
    }
  }
  *t_out = best_t;
  b_out[0] = best_b[0]; b_out[1] = best_b[1]; b_out[2] = best_b[2];
  return best;
}

/* ------------------------------------------------------------------------- */
/* Trace, interact and tally (Sec. II.A; multiple reflections, Sec. I).        */
/* ------------------------------------------------------------------------- */
int orc_trace_range(const double* V, uint64_t nv, const uint32_t* T, uint64_t nt, const orc_bvh* bvh,
                    const orc_consts* c, uint64_t p0, uint64_t p1,
                    double* tri_sum, double* tri_comp, orc_scalars* sc, const orc_particle_out* po) {
  (void)nv;
  for (uint64_t pid = p0; pid < p1; ++pid) {
    double o[3], w[3];
    orc_seed_one(c, pid, o, w, 0);
    uint64_t i = pid - p0;
    if (po && po->w_entry)
      for (int k = 0; k < 3; ++k) po->w_entry[3 * i + k] = w[k];
    int64_t prev = -1;
    uint32_t hits = 0;
    double D = 0.0, E = 0.0;
    double dwp[3] = {0.0, 0.0, 0.0}, Lp[3] = {0.0, 0.0, 0.0};
    int32_t first = -1;
    sc->rays += 1;
    for (;;) {
      sc->segments += 1;
      double best_t, best_b[3];
      int64_t best = orc_closest(V, T, nt, bvh, o, w, prev, &best_t, best_b);
      if (best < 0) {
        if (hits == 0) sc->missed += 1;
        else sc->escaped += 1;
        break;
      }
      double v0[3], v1[3], v2[3], p[3], e1[3], e2[3], ng[3];
      tri_verts(V, T, (uint64_t)best, v0, v1, v2);
      for (int k = 0; k < 3; ++k) {
        p[k] = best_b[0] * v0[k] + best_b[1] * v1[k] + best_b[2] * v2[k];
        e1[k] = v1[k] - v0[k];
        e2[k] = v2[k] - v0[k];
      }
      ng[0] = e1[1] * e2[2] - e1[2] * e2[1];
      ng[1] = e1[2] * e2[0] - e1[0] * e2[2];
      ng[2] = e1[0] * e2[1] - e1[1] * e2[0];
      double nl = sqrt(ng[0] * ng[0] + ng[1] * ng[1] + ng[2] * ng[2]);
      for (int k = 0; k < 3; ++k) ng[k] /= nl;

      double wout[3];
      orc_reflect(c, pid, hits, w, ng, wout);
      /* Momentum given to the body by this hit (Sec. II.A): w - w', and its
       * moment about the body origin, p x (w - w'). */
      double dw[3] = {w[0] - wout[0], w[1] - wout[1], w[2] - wout[2]};
      double L[3] = {p[1] * dw[2] - p[2] * dw[1], p[2] * dw[0] - p[0] * dw[2], p[0] * dw[1] - p[1] * dw[0]};
      double* s = tri_sum + 7 * (uint64_t)best;
      double* cc = tri_comp + 7 * (uint64_t)best;
      for (int k = 0; k < 3; ++k) { nsum(s + k, cc + k, dw[k]); nsum(s + 3 + k, cc + 3 + k, L[k]); }
      s[6] += 1.0;
      for (int k = 0; k < 3; ++k) { dwp[k] += dw[k]; Lp[k] += L[k]; }
      D += dw[0] * c->U[0] + dw[1] * c->U[1] + dw[2] * c->U[2];
      /* energy given to the body by this hit, in units of m c_mp^2 / 2 */
      E += (w[0] * w[0] + w[1] * w[1] + w[2] * w[2]) - (wout[0] * wout[0] + wout[1] * wout[1] + wout[2] * wout[2]);
      if (hits == 0) first = (int32_t)best;
      hits += 1;
      sc->hits += 1;
      for (int k = 0; k < 3; ++k) { o[k] = p[k]; w[k] = wout[k]; }
      prev = best;
      if (hits >= c->rmax) { sc->capped += 1; break; }
    }
    nsum(&sc->D, &sc->D_c, D);
    nsum(&sc->D2, &sc->D2_c, D * D);
    nsum(&sc->E, &sc->E_c, E);
    nsum(&sc->E2, &sc->E2_c, E * E);
    if (po) {
      if (po->first_tri) po->first_tri[i] = first;
      if (po->nhits) po->nhits[i] = (int32_t)hits;
      if (po->D) po->D[i] = D;
      if (po->E) po->E[i] = E;
      for (int k = 0; k < 3; ++k) {
        if (po->w_exit) po->w_exit[3 * i + k] = w[k];
        if (po->dw) po->dw[3 * i + k] = dwp[k];
        if (po->L) po->L[3 * i + k] = Lp[k];
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Force, moment and drag coefficient (eq. drag; Sec. II.A effective mass).    */
/* Each particle carries the rate Gamma / N, so the force is                   */
/*   F = rho c_mp^2 (Gamma_hat / N) sum (w - w'),  q = rho S^2 c_mp^2 / 2,      */
/*   F / q = K sum (w - w') with K = 2 Gamma_hat / (N S^2); the moment likewise */
/*   (Mhat = M / (rho c_mp^2), finite at S = 0 like Fhat).                     */
/* ------------------------------------------------------------------------- */
void orc_finalize(const orc_consts* c, const double* tri_total, uint64_t nt, const orc_scalars* sc,
                  const double x_ref[3], double A_ref, orc_result* out) {
  memset(out, 0, sizeof(*out));
  double F[3] = {0, 0, 0}, Fc[3] = {0, 0, 0}, L[3] = {0, 0, 0}, Lc[3] = {0, 0, 0};
  for (uint64_t k = 0; k < nt; ++k)
    for (int j = 0; j < 3; ++j) {
      nsum(&F[j], &Fc[j], tri_total[7 * k + j]);
      nsum(&L[j], &Lc[j], tri_total[7 * k + 3 + j]);
    }
  for (int j = 0; j < 3; ++j) { F[j] += Fc[j]; L[j] += Lc[j]; }
  double N = (double)c->N;
  double K = c->s_zero ? NAN : 2.0 * c->Gamma_hat / (N * c->S * c->S);
  double M[3] = {L[0] - (x_ref[1] * F[2] - x_ref[2] * F[1]),
                 L[1] - (x_ref[2] * F[0] - x_ref[0] * F[2]),
                 L[2] - (x_ref[0] * F[1] - x_ref[1] * F[0])};
  for (int j = 0; j < 3; ++j) {
    out->F_over_q[j] = K * F[j];
    out->M_over_q[j] = K * M[j];
    out->Fhat[j] = c->Gamma_hat / N * F[j];
    out->Mhat[j] = c->Gamma_hat / N * M[j];
  }
  out->CD = (out->F_over_q[0] * c->U[0] + out->F_over_q[1] * c->U[1] + out->F_over_q[2] * c->U[2]) / A_ref;
  double meanD = (sc->D + sc->D_c) / N;
  double varD = (sc->D2 + sc->D2_c) / N - meanD * meanD;
  if (varD < 0.0) varD = 0.0;
  out->CD_sigma = c->s_zero ? NAN : 2.0 * c->Gamma_hat / (c->S * c->S * A_ref) * sqrt(varD / N);
  out->Gamma_hat = c->Gamma_hat;
  /* Energy: each particle carries the rate Gamma / N, so the power to the body
   * is Q = n c_mp (m c_mp^2 / 2) (Gamma_hat / N) sum E; C_H = Q / (rho U^3 A_ref / 2)
   * = Gamma_hat sum E / (N S^3 A_ref). */
  double sumE = sc->E + sc->E_c;
  double meanE = sumE / N;
  double varE = (sc->E2 + sc->E2_c) / N - meanE * meanE;
  if (varE < 0.0) varE = 0.0;
  out->Qhat = c->Gamma_hat * meanE;
  out->CH = c->s_zero ? NAN : c->Gamma_hat * meanE / (c->S * c->S * c->S * A_ref);
  out->CH_sigma = c->s_zero ? NAN : c->Gamma_hat / (c->S * c->S * c->S * A_ref) * sqrt(varE / N);
  out->rays = sc->rays; out->hits = sc->hits; out->segments = sc->segments;
  out->missed = sc->missed; out->escaped = sc->escaped; out->capped = sc->capped;
}
