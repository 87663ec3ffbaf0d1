// tpmc_device.hpp -- device building blocks of the TPMC hot path for gfx950:
// Philox streams, FP64 boundary seeding, FP32 watertight ray-triangle and
// ray-box tests, Maxwell re-emission, fixed-point quantisation, wave reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tpmc_internal.h"
#include "tpmc_math.hpp"

// Contraction into FMA only within one source expression, so every kernel that
// inlines these functions rounds them identically (plain and batched paths
// must agree bit for bit).
#pragma clang fp contract(on)

namespace tpmc {

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.77245385090551602730;
constexpr double kInvSqrt2 = 0.70710678118654752440;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Stream of particle p at
// step s: counter (p lo, p hi, s, 0), key (seed lo, seed hi).  Steps 0-1 feed
// the seeding, step 2 + b the b-th re-emission.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t a, b, c, d;
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // full 64-bit products: one v_mad_u64_u32 gives both halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ U4 stream(const QueryDev& q, uint64_t pid, uint32_t step) {
  return philox4x32_10((uint32_t)pid, (uint32_t)(pid >> 32), step, 0u, q.key0, q.key1);
}

// Uniform variates in (0, 1), exact in their type:
// FP64 u = (k + 1/2) 2^-32; FP32 u = (floor(k / 2^9) + 1/2) 2^-23.
__device__ __forceinline__ double unif64(uint32_t k) { return ((double)k + 0.5) * 0x1p-32; }
__device__ __forceinline__ float unif32(uint32_t k) { return ((float)(k >> 9) + 0.5f) * 0x1p-23f; }

// ---------------------------------------------------------------------------
// Boundary seeding in FP64 (Sec. III.A).
//
// Latitude: mu = sin(phi) has density chi(S mu) / Z(S) on [-1, 1], from
// g(phi|S) with d(mu) = cos(phi) d(phi); chi(s) = e^{-s^2} + sqrt(pi) s (1 + erf s).
// Its CDF numerator G(t) = int_{-1}^t chi(S m) dm is the difference of the
// antiderivative sqrt(pi)/(4S) erf(St) + sqrt(pi) S t^2 (1 + erf St)/2 + t e^{-S^2 t^2}/2
// at t and -1, arranged so that no term cancels.  G' = chi(S t) > 0 and
// G'' = S sqrt(pi) (1 + erf St), so the equation G(mu) = u Z is solved by
// Halley's method inside a shrinking bracket.  Every evaluation costs one exp
// and one erfc: the alternative forms below are selected values, not calls.
//
// Mixed precision: the iterations that only approach the root run in FP32
// (cheap exp / erfc) until a step is below 1e-3 (by the cubic convergence the
// error after such a step is near 1e-9); then FP64 Halley steps take over and
// end after a step below 1e-5, which leaves an error far below the FP64
// resolution of the result (usually one FP64 evaluation).  The result is an FP64 root either way; FP32
// only chooses where the FP64 iteration starts.
// ---------------------------------------------------------------------------
// Besides G and its derivatives, returns e = exp(-(S t)^2) and ta = erfc(|S t|),
// which the normal-speed law at s = S mu reuses (normal_speed_consts_near).
// Both come from the shifted table ee (exp_erfc_grid).
__device__ __forceinline__ void latitude_G(const QueryDev& q, const double* __restrict__ ee, double t, double& G,
                                           double& dG, double& d2G, double& e, double& ta) {
  const double S = q.S;
  const double St = S * t;
  exp_erfc_grid(ee, fabs(St), e, ta);
  const double c = St >= 0.0 ? 2.0 - ta : ta;  // erfc(-S t) = 1 + erf(S t)
  double E;                                     // erf(S t) + erf(S)
  if (S < 0.25) E = erf(St) + q.erfS;  // uniform branch: small S keeps erf(St) exact
  else E = St < -1.0 ? c - q.erfcS : (c - 1.0) + q.erfS;
  G = q.lat_k * E + 0.5 * kSqrtPi * S * (t * t * c - q.erfcS) + 0.5 * (t * e + q.expmS2);
  dG = e + kSqrtPi * St * c;
  d2G = S * kSqrtPi * c;
}

// FP32 form of G for the approaching iterations (constants rounded to FP32).
struct LatConst32 {
  float S, erfS, erfcS, expmS2;
  bool small;
};

__device__ __forceinline__ void latitude_G32(const LatConst32& c, float t, float& G, float& dG, float& d2G) {
  const float St = c.S * t;
  const float e = __expf(-St * St);  // exp2 of x log2(e): relative error up to ~|x| 2^-24, ample here
  const float ey = e * erfcx32(fabsf(St));    // erfc(|S t|)
  const float cc = St >= 0.0f ? 2.0f - ey : ey;  // erfc(-S t)
  const float E = c.small ? erff(St) + c.erfS : (St < -1.0f ? cc - c.erfcS : (cc - 1.0f) + c.erfS);
  G = (float)kSqrtPi / (4.0f * c.S) * E + 0.5f * (float)kSqrtPi * c.S * (t * t * cc - c.erfcS) +
      0.5f * (t * e + c.expmS2);
  dG = e + (float)kSqrtPi * St * cc;
  d2G = c.S * (float)kSqrtPi * cc;
}

// One Halley step inside the bracket [lo, hi], bisection when the step leaves
// it.  x_new = x - 2 f f' / (2 f'^2 - f f''), or the Newton step f / f' when
// the Halley factor 1 - f f'' / (2 f'^2) leaves (1/2, 2); one reciprocal either
// way.  Returns |step| of a Halley (or Newton) step, or +inf after a
// bisection, so that only a genuine iteration step can end a solve.  The
// bounds are inclusive: a step below one ulp leaves x unchanged.
// The quotient uses the hardware reciprocal (plus one Newton step in FP64):
// the step only corrects x, so its relative accuracy (1 ulp in FP32, ~2^-50
// in FP64) is ample, and a zero or non-finite denominator still sends the
// iterate out of the bracket into bisection.
__device__ __forceinline__ float step_quotient(float n, float d) { return n * __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double step_quotient(double n, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return n * r;
}

template <class T>
__device__ __forceinline__ T halley_step(T& x, T f, T df, T d2f, T& lo, T& hi) {
  if (f < T(0)) lo = x;
  else hi = x;
  const T df2 = df * df;
  const T D = T(2) * df2 - f * d2f;
  const bool hal = D > df2 && D < T(4) * df2;
  const T xn = x - step_quotient(hal ? T(2) * f * df : f, hal ? D : df);
  if (xn >= lo && xn <= hi) {
    const T dx = fabs(xn - x);
    x = xn;
    return dx;
  }
  x = T(0.5) * (lo + hi);
  return (T)__builtin_inf();
}

// Starting points of the latitude solve: a table of the root mu of
// G(mu) = u Z(S) over ln S = ln kLatS0 + i kLatDL (S from 0.05 to 10.02) and
// the logit t = ln(u / (1 - u)) = kLatT0 + j kLatDT, bilinear in (ln S, t).
// The law depends on S alone, so one table serves every query; rows are
// spaced in ln S because the root bends fastest in S below S ~ 1.  Filled once
// per device by FP64 bisection (lat_table_kernel); a bilinear start is within
// 1e-3 of the root, so one FP32 step usually ends the approach.  Outside the
// table the start is a blend of the S -> 0 law (uniform mu) and the S -> inf
// law (density 2 mu).  It only chooses where the iteration starts, and only
// where the fine table below does not reach (S < 0.25 or S > 10).
constexpr int kLatNS = 107, kLatNT = 257;
constexpr float kLatS0 = 0.05f, kLatDL = 0.05f, kLatT0 = -24.0f, kLatDT = 0.1875f;

__device__ __forceinline__ float unif32_hi(uint32_t k) { return ((float)k + 0.5f) * 0x1p-32f; }  // ~unif64(k)

// FP32 natural logarithm by the hardware log2 (starting points and the
// seeding estimate only; the exact solves keep their own logarithm).
__device__ __forceinline__ float hw_ln(float x) { return 0.69314718f * __builtin_amdgcn_logf(x); }

// The same root from the fine table (layout kLatF* in tpmc_internal.h, filled
// by lat_fine_kernel) at the draw u = ua, 1 - u = uam: the four rows and
// cubic weights in ln S that the host set for the query (q.lat_f0 >= 0, i.e.
// S in [0.25, 10]), linear in the logit.  Within 6e-6 of the root for every u
// (a dense host evaluation against FP64 roots, poles included), so the exact
// solve starts from it with no FP32 step, and the seeding estimate takes it as
// it is.
__device__ __forceinline__ float latitude_fine(const QueryDev& q, const float* __restrict__ tab, float ua,
                                               float uam) {
  const float t = hw_ln(ua) - hw_ln(uam);
  const float ft = fminf(fmaxf((t - kLatFT0) * (1.0f / kLatFDT), 0.0f), (float)(kLatFNT - 1));
  const int j = min((int)ft, kLatFNT - 2);
  const float b = ft - (float)j;
  const float* r = tab + q.lat_f0 * kLatFNT + j;
  float m = 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) m += q.lat_fw[k] * ((1.0f - b) * r[k * kLatFNT] + b * r[k * kLatFNT + 1]);
  return fminf(fmaxf(m, -1.0f), 1.0f);
}

__device__ __forceinline__ float latitude_start(const float* __restrict__ tab, float S, double u) {
  const float fs = logf(S * (1.0f / kLatS0)) * (1.0f / kLatDL);
  const float uf = (float)u;
  if (fs >= 0.0f && fs <= (float)(kLatNS - 1)) {
    const float t = logf(uf) - logf((float)(1.0 - u));
    const float ft = fminf(fmaxf((t - kLatT0) * (1.0f / kLatDT), 0.0f), (float)(kLatNT - 1));
    const int i = min((int)fs, kLatNS - 2), j = min((int)ft, kLatNT - 2);
    const float a = fs - (float)i, b = ft - (float)j;
    const float* r0 = tab + i * kLatNT + j;
    const float* r1 = r0 + kLatNT;
    return (1.0f - a) * ((1.0f - b) * r0[0] + b * r0[1]) + a * ((1.0f - b) * r1[0] + b * r1[1]);
  }
  const float wgt = S * S / (1.0f + S * S);
  return (1.0f - wgt) * (2.0f * uf - 1.0f) + wgt * sqrtf(uf);
}

// The last FP64 evaluation of a latitude solve: point t, exp(-(S t)^2), erfc(|S t|).
struct LatEval {
  double t, e, ta;
  bool valid;
};

__device__ inline double sample_latitude(const QueryDev& q, const float* __restrict__ lat_tab,
                                        const float* __restrict__ lat_fine, const double* __restrict__ ee,
                                        uint32_t k, LatEval& le) {
  const double u = unif64(k);
  le.valid = false;
  if (q.s_zero) return 2.0 * u - 1.0;  // S -> 0: g -> cos(phi)/2, mu uniform
  const double target = u * q.Z;
  float xf;
  if (q.lat_f0 >= 0) {
    // one FP64 step from here ends the solve (start error ~6e-6 < 1e-5)
    xf = latitude_fine(q, lat_fine, unif32_hi(k), unif32_hi(~k));
  } else {
    const LatConst32 c{(float)q.S, (float)q.erfS, (float)q.erfcS, (float)q.expmS2, q.S < 0.25};
    xf = fminf(fmaxf(latitude_start(lat_tab, c.S, u), -1.0f), 1.0f);
    float lof = -1.0f, hif = 1.0f;
    const float tf = (float)target;
#pragma unroll 1
    for (int it = 0; it < 5; ++it) {
      float G, dG, d2G;
      latitude_G32(c, xf, G, dG, d2G);
      const float dx = halley_step(xf, G - tf, dG, d2G, lof, hif);
      if (dx <= 1e-3f || hif - lof <= 1e-3f) break;
    }
  }
  double x = (double)xf;
  double lo = -1.0, hi = 1.0;
  le.valid = true;
#pragma unroll 1
  for (int it = 0; it < 100; ++it) {
    double G, dG, d2G;
    le.t = x;
    latitude_G(q, ee, x, G, dG, d2G, le.e, le.ta);
    const double dx = halley_step(x, G - target, dG, d2G, lo, hi);
    // cubic convergence: after a step below 1e-5 the remaining error is far
    // below the FP64 resolution of mu
    if (dx <= 1e-5 || hi - lo <= 1e-15) break;
  }
  return x;
}

// Inward normal speed x = v_n / c_mp >= 0 of eq. vel_dist1, p(x|s) = 2x e^{-(x-s)^2} / chi(s).
// CDF numerator F(x) = e^{-s^2} - e^{-(x-s)^2} + sqrt(pi) s (erf(x-s) + erf s),
// F' = 2x e^{-(x-s)^2}, F'' = 2 e^{-(x-s)^2} (1 - 2x(x-s)).
struct NormalSpeedConsts {
  double s, es2, erfs, erfcs, erfcms, chi;
};

__device__ __forceinline__ NormalSpeedConsts normal_speed_consts(const double* __restrict__ ee, double s) {
  NormalSpeedConsts k;
  k.s = s;
  double t;  // the small one of erfc(s), erfc(-s)
  exp_erfc_grid(ee, fabs(s), k.es2, t);
  k.erfcs = s >= 0.0 ? t : 2.0 - t;
  k.erfcms = s >= 0.0 ? 2.0 - t : t;  // 1 + erf(s)
  k.erfs = s >= 0.0 ? 1.0 - t : t - 1.0;
  k.chi = k.es2 + kSqrtPi * s * k.erfcms;
  return k;
}

// The same constants at s from exp(-s0^2) and erfc(|s0|) at a nearby s0 of
// the same sign (the latitude solve's last evaluation point, S times a point
// within one Halley step of mu).  With y = |s0|, h = |s| - y:
//   exp(-s^2)  = exp(-y^2) sum_n H_n(-y) h^n / n!,
//   erfc(|s|)  = erfc(y) - 2/sqrt(pi) exp(-y^2) sum_n H_n(-y) h^(n+1) / (n+1)!,
// H_n the physicists' Hermite polynomials (generating function
// exp(2xh - h^2) = sum_n H_n(x) h^n / n!).  For |h| (y + 1) <= 1e-4 the terms
// fall by at least ~2e-4 each, so six terms leave a relative error near 1e-21;
// otherwise (or across s = 0) the constants are evaluated directly.
__device__ __forceinline__ NormalSpeedConsts normal_speed_consts_near(const double* __restrict__ ee, double s,
                                                                     double s0, double e0, double ta0) {
  const double y = fabs(s0);
  const double h = fabs(s) - y;
  if (!((s >= 0.0) == (s0 >= 0.0) && fabs(h) * (y + 1.0) <= 1e-4)) return normal_speed_consts(ee, s);
  constexpr double kInv[7] = {1.0, 1.0, 1.0 / 2, 1.0 / 3, 1.0 / 4, 1.0 / 5, 1.0 / 6};
  const double x = -y;
  double Hm = 1.0, Hn = 2.0 * x;          // H_0, H_1
  double hp = h;                          // h^n / n! at n = 1
  double E = 1.0 + Hn * hp;               // sum_n H_n h^n / n!
  double I = h + Hn * hp * h * kInv[2];  // sum_n H_n h^(n+1) / (n+1)!
#pragma unroll
  for (int n = 1; n < 5; ++n) {
    const double Hp = 2.0 * x * Hn - 2.0 * n * Hm;  // H_{n+1}
    Hm = Hn;
    Hn = Hp;
    hp *= h * kInv[n + 1];            // h^(n+1) / (n+1)!
    E += Hn * hp;
    I += Hn * hp * h * kInv[n + 2];  // h^(n+2) / (n+2)!
  }
  NormalSpeedConsts k;
  k.s = s;
  k.es2 = e0 * E;
  const double t = ta0 - 2.0 / kSqrtPi * e0 * I;  // erfc(|s|)
  k.erfcs = s >= 0.0 ? t : 2.0 - t;
  k.erfcms = s >= 0.0 ? 2.0 - t : t;
  k.erfs = s >= 0.0 ? 1.0 - t : t - 1.0;
  k.chi = k.es2 + kSqrtPi * s * k.erfcms;
  return k;
}

__device__ __forceinline__ void normal_speed_F(const double* __restrict__ ee, const NormalSpeedConsts& k, double x,
                                               double& F, double& dF, double& d2F) {
  const double a = x - k.s;
  double ea, t;
  exp_erfc_grid(ee, fabs(a), ea, t);
  // erf(x - s) + erf(s) as a difference of small erfc values wherever a sum would cancel
  const double esum = k.s < 0.0 ? k.erfcms - t : (a < 0.0 ? t - k.erfcs : (1.0 - t) + k.erfs);
  F = k.es2 - ea + kSqrtPi * k.s * esum;
  dF = 2.0 * x * ea;
  d2F = 2.0 * ea * (1.0 - 2.0 * x * a);
}

__device__ __forceinline__ void normal_speed_F32(float s, float es2, float erfs, float erfcs, float erfcms, float x,
                                                 float& F, float& dF, float& d2F) {
  const float a = x - s;
  const float ea = __expf(-a * a);
  const float t = ea * erfcx32(fabsf(a));  // erfc(|a|)
  const float esum = s < 0.0f ? erfcms - t : (a < 0.0f ? t - erfcs : (1.0f - t) + erfs);
  F = es2 - ea + (float)kSqrtPi * s * esum;
  dF = 2.0f * x * ea;
  d2F = 2.0f * ea * (1.0f - 2.0f * x * a);
}

// Starting points of the normal-speed solve: a table of the root x of
// F(x | s) = u chi(s) over s in [kVnS0, kVnS0 + (kVnNS - 1) kVnDS] and the logit
// t = ln(u / (1 - u)) in [kVnT0, kVnT0 + (kVnNT - 1) kVnDT], bilinear in (s, t).
// The law depends on s alone, so one table serves every query; it is filled
// once per device by FP64 bisection (vn_table_kernel).  It only chooses where
// the iteration starts.
constexpr int kVnNS = 225, kVnNT = 385;
constexpr float kVnS0 = -4.0f, kVnDS = 0.0625f, kVnT0 = -24.0f, kVnDT = 0.125f;

__device__ __forceinline__ float normal_speed_start(const float* __restrict__ tab, double s, double u) {
  const float sf = (float)s;
  if (sf >= kVnS0 && sf <= kVnS0 + (kVnNS - 1) * kVnDS) {
    const float t = logf((float)u) - logf((float)(1.0 - u));
    const float fs = (sf - kVnS0) * (1.0f / kVnDS);
    const float ft = fminf(fmaxf((t - kVnT0) * (1.0f / kVnDT), 0.0f), (float)(kVnNT - 1));
    const int i = min((int)fs, kVnNS - 2), j = min((int)ft, kVnNT - 2);
    const float a = fs - (float)i, b = ft - (float)j;
    const float* r0 = tab + i * kVnNT + j;
    const float* r1 = r0 + kVnNT;
    return (1.0f - a) * ((1.0f - b) * r0[0] + b * r0[1]) + a * ((1.0f - b) * r1[0] + b * r1[1]);
  }
  // outside the table: near-Gaussian about s for large s, the Rayleigh law otherwise
  const float uf = (float)u;
  return sf > 1.0f ? sf + 0.5f / sf + erfinvf(2.0f * uf - 1.0f) : sqrtf(-log1pf(-uf));
}

__device__ inline double sample_normal_speed(const float* __restrict__ tab, const double* __restrict__ ee,
                                             const NormalSpeedConsts& k, double u) {
  const double s = k.s;
  const double target = u * k.chi;
  // The root lies below max(s, 0) + 7: the upper tail there is below e^{-49},
  // far under the smallest 1 - u the variates produce (2^-33).
  const double hi0 = (s > 0.0 ? s : 0.0) + 7.0;
  // FP32 approach from the tabulated start.  Below s = -9 the FP32 density
  // underflows; such s are never drawn in practice, and FP64 then starts there.
  const float sf = (float)s;
  float xf = normal_speed_start(tab, s, u);
  float lof = 0.0f, hif = (float)hi0;
  if (!(xf > lof && xf < hif)) xf = 0.5f * (lof + hif);
  if (s > -9.0) {
    const float es2 = (float)k.es2, erfs = (float)k.erfs, erfcs = (float)k.erfcs, erfcms = (float)k.erfcms;
    const float tf = (float)target;
#pragma unroll 1
    for (int it = 0; it < 5; ++it) {
      float F, dF, d2F;
      normal_speed_F32(sf, es2, erfs, erfcs, erfcms, xf, F, dF, d2F);
      const float dx = halley_step(xf, F - tf, dF, d2F, lof, hif);
      if (dx <= 1e-3f * xf || hif - lof <= 1e-3f * xf) break;
    }
  }
  double x = (double)xf;
  double lo = 0.0, hi = hi0;
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
#pragma unroll 1
  for (int it = 0; it < 100; ++it) {
    double F, dF, d2F;
    normal_speed_F(ee, k, x, F, dF, d2F);
    const double dx = halley_step(x, F - target, dF, d2F, lo, hi);
    if (dx <= 1e-5 * x || hi - lo <= 1e-15 * x) break;
  }
  return x;
}

// One seeded particle (Sec. III.A.1-3): position on the CV and velocity, FP64.
// Both control volumes give a point x, an inward unit normal n, unit tangents
// t1, t2, a tangential drift (d1, d2) and the normal drift s_n; the normal
// speed (eq. vel_dist1) and the Gaussian tangentials (eqs. vel_dist2-3) are
// drawn the same way, w = w_n n + (d1 + g1/sqrt2) t1 + (d2 + g2/sqrt2) t2.
//  * Sphere: mu = sin(phi) from g(phi|S), theta uniform; n = mu U - cos(phi) c
//    with c = cos(th) e1 + sin(th) e2, t1 = cos(phi) U + mu c (along the
//    tangential part of U), t2 = t1 x n = sin(th) e1 - cos(th) e2;
//    x = c0 - r n; d1 = S cos(phi), d2 = 0; s_n = S mu.
//  * Box (query flag): face f by its share A_f chi(s_f) of the inflow, a
//    uniform point on it; n = n_a e_a (a = f/2, n_a = +1 on the low face),
//    t1 = e_j, t2 = e_l (j = a+1, l = a+2 mod 3); d1 = S U_j, d2 = S U_l;
//    s_n = s_f.
// Only the few scalars that fix the frame stay live across the normal-speed
// solve (the frame is expanded afterwards), which keeps the persistent kernel
// inside its register budget.
__device__ inline void seed_particle(const QueryDev& q, const float* __restrict__ lat_tab,
                                     const float* __restrict__ lat_fine, const float* __restrict__ vn_tab, const double* __restrict__ sc_tab,
                                     const double* __restrict__ ee, uint64_t pid, double x[3], double w[3]) {
  const U4 r0 = stream(q, pid, 0u);
  const U4 r1 = stream(q, pid, 1u);
  double p0, p1, p2, p3;  // sphere: mu, cos(phi), sin(th), cos(th); box: n_a, position on the face (2)
  int fa = 0;             // box: the face's normal axis
  NormalSpeedConsts k;
  if (q.box) {
    const double t = unif64(r0.a) * q.face_cum[5];
    int f = 0;
    while (f < 5 && !(t < q.face_cum[f])) ++f;
    fa = f >> 1;
    p0 = (f & 1) ? -1.0 : 1.0;
    p1 = 2.0 * unif64(r0.b) - 1.0;
    p2 = 2.0 * unif64(r1.b) - 1.0;
    p3 = 0.0;
    k = normal_speed_consts(ee, q.face_s[f]);
  } else {
    LatEval le;
    p0 = sample_latitude(q, lat_tab, lat_fine, ee, r0.a, le);
    p1 = sqrt(fmax(0.0, 1.0 - p0 * p0));
    sincos_2pi_draw(sc_tab, r0.b, p2, p3);  // of 2 pi unif64(r0.b)
    const double s_n = q.S * p0;
    k = le.valid ? normal_speed_consts_near(ee, s_n, q.S * le.t, le.e, le.ta) : normal_speed_consts(ee, s_n);
  }
  const double wn = sample_normal_speed(vn_tab, ee, k, unif64(r0.c));
  const double rad = sqrt(-2.0 * log_draw(r0.d));  // ln unif64(r0.d)
  double sb, cb;
  sincos_2pi_draw(sc_tab, r1.a, sb, cb);  // of 2 pi unif64(r1.a)
  const double g1 = rad * cb * kInvSqrt2, g2 = rad * sb * kInvSqrt2;
  if (q.box) {
    const int j = fa == 2 ? 0 : fa + 1;  // t1 axis; the remaining axis is t2's
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      x[i] = i == fa ? q.c0[i] - p0 * q.h[i] : q.c0[i] + (i == j ? p1 : p2) * q.h[i];
      w[i] = i == fa ? wn * p0 : q.S * q.U[i] + (i == j ? g1 : g2);
    }
  } else {
    const double mu = p0, cphi = p1, sth = p2, cth = p3;
    const double wt1 = q.S * cphi + g1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double ci = cth * q.e1[i] + sth * q.e2[i];
      const double di = -sth * q.e1[i] + cth * q.e2[i];
      const double ni = mu * q.U[i] - cphi * ci;
      const double t1i = cphi * q.U[i] + mu * ci;
      x[i] = q.c0[i] - q.r * ni;
      w[i] = wn * ni + wt1 * t1i - g2 * di;
    }
  }
}

// ---------------------------------------------------------------------------
// Ray set-up for the watertight test of Woop, Benthin & Wald (JCGT 2013):
// permute so that z is the dominant direction axis, shear so the ray is +z.
// ---------------------------------------------------------------------------
struct Ray {
  float ox, oy, oz;
  float dx, dy, dz;
  float idx, idy, idz;  // 1 / d for the slab test
  float Sx, Sy, Sz;
  int kx, ky, kz;
};

__device__ __forceinline__ float comp(float x, float y, float z, int k) { return k == 0 ? x : (k == 1 ? y : z); }

__device__ __forceinline__ void make_ray(Ray& r, float ox, float oy, float oz, float dx, float dy, float dz) {
  r.ox = ox; r.oy = oy; r.oz = oz;
  r.dx = dx; r.dy = dy; r.dz = dz;
  // Hardware reciprocals (1 ulp); the slab test's far-bound margin covers
  // them, and the shear only has to be the same for every triangle of a ray.
  r.idx = __builtin_amdgcn_rcpf(dx); r.idy = __builtin_amdgcn_rcpf(dy); r.idz = __builtin_amdgcn_rcpf(dz);
  const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
  int kz = 0;
  if (ay > ax) kz = 1;
  if (az > fmaxf(ax, ay)) kz = 2;
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  const float dkz = comp(dx, dy, dz, kz);
  if (dkz < 0.0f) {
    const int t = kx;
    kx = ky;
    ky = t;
  }
  r.kx = kx; r.ky = ky; r.kz = kz;
  r.Sz = __builtin_amdgcn_rcpf(dkz);
  r.Sx = comp(dx, dy, dz, kx) * r.Sz;
  r.Sy = comp(dx, dy, dz, ky) * r.Sz;
}

// Two-sided closest-hit candidate test.  Returns true with t and barycentrics
// when the ray meets the triangle at 0 < t <= t_max.  Watertight test of Woop,
// Benthin & Wald (JCGT 2013): translate to the ray origin, permute so the
// dominant direction component is z, shear so the ray is +z, and take the
// three 2-D edge functions; exactly-zero edge functions are recomputed in FP64
// so that an edge shared by two triangles is never missed by both.  Apart from
// that rare fallback the test is branch-free.
__device__ __forceinline__ bool intersect_tri(const Ray& r, const TriRec& tr, float t_max, float& t_out,
                                              float& b0, float& b1, float& b2) {
#pragma clang fp contract(off)
  const float Ax0 = tr.v0x - r.ox, Ay0 = tr.v0y - r.oy, Az0 = tr.v0z - r.oz;
  const float Bx0 = tr.v1x - r.ox, By0 = tr.v1y - r.oy, Bz0 = tr.v1z - r.oz;
  const float Cx0 = tr.v2x - r.ox, Cy0 = tr.v2y - r.oy, Cz0 = tr.v2z - r.oz;
  const float Akx = comp(Ax0, Ay0, Az0, r.kx), Aky = comp(Ax0, Ay0, Az0, r.ky), Akz = comp(Ax0, Ay0, Az0, r.kz);
  const float Bkx = comp(Bx0, By0, Bz0, r.kx), Bky = comp(Bx0, By0, Bz0, r.ky), Bkz = comp(Bx0, By0, Bz0, r.kz);
  const float Ckx = comp(Cx0, Cy0, Cz0, r.kx), Cky = comp(Cx0, Cy0, Cz0, r.ky), Ckz = comp(Cx0, Cy0, Cz0, r.kz);
  const float Ax = Akx - r.Sx * Akz, Ay = Aky - r.Sy * Akz;
  const float Bx = Bkx - r.Sx * Bkz, By = Bky - r.Sy * Bkz;
  const float Cx = Ckx - r.Sx * Ckz, Cy = Cky - r.Sy * Ckz;
  float U = Cx * By - Cy * Bx;
  float V = Ax * Cy - Ay * Cx;
  float W = Bx * Ay - By * Ax;
  if (U == 0.0f || V == 0.0f || W == 0.0f) {
    U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
    V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
    W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
  }
  const bool mixed = (U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f);
  const float det = U + V + W;
  const float T = U * (r.Sz * Akz) + V * (r.Sz * Bkz) + W * (r.Sz * Ckz);
  // Hardware reciprocal (1 ulp): t and the barycentrics only place the hit;
  // which side of every edge the ray passes was settled exactly above.
  const float inv = __builtin_amdgcn_rcpf(det);
  const float t = T * inv;
  t_out = t;
  b0 = U * inv;
  b1 = V * inv;
  b2 = W * inv;
  return !mixed && det != 0.0f && t > 0.0f && t <= t_max && t < __builtin_inff();
}

// Slab test of a child box; conservative far bound per Ize (JCGT 2013), so a
// box whose triangle is hit is never culled by rounding.
__device__ __forceinline__ bool slab(const Ray& r, float lox, float loy, float loz, float hix, float hiy, float hiz,
                                     float t_max, float& t_near) {
  const float tx0 = (lox - r.ox) * r.idx, tx1 = (hix - r.ox) * r.idx;
  const float ty0 = (loy - r.oy) * r.idy, ty1 = (hiy - r.oy) * r.idy;
  const float tz0 = (loz - r.oz) * r.idz, tz1 = (hiz - r.oz) * r.idz;
  const float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
  const float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), t_max));
  t_near = tn;
  // 1 + 5 * 2^-23 >= 1 + 8u (u = 2^-24): two roundings per t value plus the
  // 1-ulp reciprocal, for both bounds (Ize, JCGT 2013).
  return tn <= tf * 1.0000006f;
}

// ---------------------------------------------------------------------------
// Seeding in two stages.  A particle whose ray misses both boxes of the BVH
// root is a miss whatever its exact state, so its exact FP64 seeding (above)
// is work without effect; on small or flat bodies most particles are such.
// precull_may_enter estimates the particle's ray from the same variates in
// FP32 (the latitude from a fine table without iteration, the normal speed
// from its tabulated start and two FP32 Halley steps, the hardware exp, log,
// sine and cosine, the frame in FP32) and tests it against the root's two
// boxes grown by kPrecullMargin CV radii on every side.  Returns false only if
// that grown test fails, i.e. only for particles whose exact ray misses the
// root's boxes:
//  * the fine latitude table (cubic in ln S, linear in the logit) leaves an
//    error d in mu of about 1e-5; the speed's Halley steps leave about C dx^3
//    after a second step dx, and the estimate gives up (the particle is
//    seeded exactly) unless that step is below 1e-5 of the speed; it also
//    gives up outside the tables' ranges of S and s;
//  * a latitude error d moves cos(phi) by d |mu| / cos(phi), so the estimate
//    gives up for cos(phi) < 0.05 (mu within 1.25e-3 of +-1); elsewhere the
//    point and the direction move by at most ~20 d, relative to r and to |w|;
//  * along the at most 2 r of path inside the CV, the estimated ray then stays
//    within ~60 d r of the exact one: a few hundredths of the margin (0.02 r)
//    for the table's d, and far less for the rounding of the FP32 solves and
//    the hardware sine, cosine and logarithm.
// tpmc_precull_check measures the distance between estimated and exact rays.
// Box control volumes are not estimated (always true).
// ---------------------------------------------------------------------------
constexpr float kPrecullMargin = 0.02f;


// fs in [0, ns - 1], ft in [0, nt - 1]
__device__ __forceinline__ float bilinear_start(const float* __restrict__ tab, int ns, int nt, float fs, float ft) {
  const int i = min((int)fs, ns - 2), j = min((int)ft, nt - 2);
  const float a = fs - (float)i, b = ft - (float)j;
  const float* r0 = tab + i * nt + j;
  const float* r1 = r0 + nt;
  return (1.0f - a) * ((1.0f - b) * r0[0] + b * r0[1]) + a * ((1.0f - b) * r1[0] + b * r1[1]);
}

// The estimated ray (o, w); false when the estimate gives up.  The per-particle
// conditions are gathered into one flag rather than taken as early returns, so
// that the lanes stay converged (table lookups use clamped indices throughout;
// what a given-up particle computes is discarded).
__device__ inline bool precull_estimate(const QueryDev& q, const float* __restrict__ lat_tab,
                                        const float* __restrict__ vn_tab, uint64_t pid, float o[3], float w[3]) {
  if (q.box) return false;
  const U4 r0 = stream(q, pid, 0u);
  const U4 r1 = stream(q, pid, 1u);
  // latitude mu = sin(phi)
  const float ua = unif32_hi(r0.a), uam = unif32_hi(~r0.a);  // u and 1 - u
  float mu;
  bool ok = true;
  if (q.s_zero) {
    mu = 2.0f * ua - 1.0f;
  } else {
    // from the fine table, inside its S range only (the host sets lat_f0 = -1 outside)
    if (q.lat_f0 < 0) return false;
    mu = latitude_fine(q, lat_tab, ua, uam);
  }
  const float cphi = sqrtf(fmaxf(0.0f, 1.0f - mu * mu));
  ok = ok && cphi >= 0.05f;
  // inward normal speed at s = S mu
  const float s = q.s_zero ? 0.0f : q.Sf * mu;
  const float es2 = __expf(-s * s);
  const float ta = es2 * erfcx32(fabsf(s));  // erfc(|s|)
  const float erfcs = s >= 0.0f ? ta : 2.0f - ta, erfcms = s >= 0.0f ? 2.0f - ta : ta;
  const float erfs = s >= 0.0f ? 1.0f - ta : ta - 1.0f;
  const float chi = es2 + (float)kSqrtPi * s * erfcms;
  const float uc = unif32_hi(r0.c), ucm = unif32_hi(~r0.c);
  const float hi0 = fmaxf(s, 0.0f) + 7.0f;
  const float fs = (s - kVnS0) * (1.0f / kVnDS);
  ok = ok && s > -9.0f && fs >= 0.0f && fs <= (float)(kVnNS - 1);  // inside the table's s range only
  const float tv = hw_ln(uc) - hw_ln(ucm);
  float wn = bilinear_start(vn_tab, kVnNS, kVnNT, fminf(fmaxf(fs, 0.0f), (float)(kVnNS - 1)),
                            fminf(fmaxf((tv - kVnT0) * (1.0f / kVnDT), 0.0f), (float)(kVnNT - 1)));
  ok = ok && wn > 0.0f && wn < hi0;
  {
    float lo = 0.0f, hi = hi0, F, dF, d2F, dx = 0.0f;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      normal_speed_F32(s, es2, erfs, erfcs, erfcms, wn, F, dF, d2F);
      dx = halley_step(wn, F - uc * chi, dF, d2F, lo, hi);
    }
    ok = ok && dx <= 1e-5f * wn;
  }
  // tangential Gaussians (Box-Muller) and the angles; v_sin / v_cos take revolutions
  const float rad = sqrtf(-2.0f * hw_ln(unif32_hi(r0.d)));
  const float ub = unif32_hi(r1.a), uth = unif32_hi(r0.b);
  const float g1 = rad * __builtin_amdgcn_cosf(ub) * (float)kInvSqrt2;
  const float g2 = rad * __builtin_amdgcn_sinf(ub) * (float)kInvSqrt2;
  const float sth = __builtin_amdgcn_sinf(uth), cth = __builtin_amdgcn_cosf(uth);
  const float wt1 = q.Sf * cphi + g1;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float ci = cth * q.e1f[i] + sth * q.e2f[i];
    const float di = -sth * q.e1f[i] + cth * q.e2f[i];
    const float ni = mu * q.Uf[i] - cphi * ci;
    const float t1i = cphi * q.Uf[i] + mu * ci;
    o[i] = q.c0f[i] - q.rf * ni;
    w[i] = wn * ni + wt1 * t1i - g2 * di;
  }
  return ok;
}

__device__ inline bool precull_may_enter(const QueryDev& q, const float* __restrict__ lat_tab,
                                         const float* __restrict__ vn_tab, const Node* __restrict__ nodes,
                                         uint64_t pid) {
  float o[3] = {0.0f, 0.0f, 0.0f}, w[3] = {0.0f, 0.0f, 0.0f};
  const bool ok = precull_estimate(q, lat_tab, vn_tab, pid, o, w);
  Ray r;
  r.ox = o[0]; r.oy = o[1]; r.oz = o[2];
  r.idx = __builtin_amdgcn_rcpf(w[0]);
  r.idy = __builtin_amdgcn_rcpf(w[1]);
  r.idz = __builtin_amdgcn_rcpf(w[2]);
  const float m = kPrecullMargin * q.rf;
  const Node& nd = nodes[0];
  const float inf = __builtin_inff();
  float tn;
  const bool h0 = slab(r, nd.lo0x - m, nd.lo0y - m, nd.lo0z - m, nd.hi0x + m, nd.hi0y + m, nd.hi0z + m, inf, tn);
  const bool h1 = slab(r, nd.lo1x - m, nd.lo1y - m, nd.lo1z - m, nd.hi1x + m, nd.hi1y + m, nd.hi1z + m, inf, tn);
  return !ok || h0 || h1;  // a given-up estimate keeps the particle
}

// ---------------------------------------------------------------------------
// Gas-surface interaction (Sec. II.A), FP32.  Maxwell model: diffuse with
// probability alpha -- the particle leaves the side it arrived on with the
// flux-weighted half-range Maxwellian of T_w (normal speed tau sqrt(-ln u),
// tangential components N(0, tau^2/2)) -- else specular.  Returns whether
// the kernel's bound on the re-emission temperature (tr_cap2, which keeps the
// fixed-point tallies in range) had to limit tau_r: the model itself has no
// such bound, so a result with any such event departs from it.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool reemit(const QueryDev& q, uint64_t pid, uint32_t bounce, float nx, float ny, float nz,
                                       float& wx, float& wy, float& wz) {
  const U4 r = stream(q, pid, 2u + bounce);
  const float wn = wx * nx + wy * ny + wz * nz;
  bool limited = false;
  if (unif32(r.a) < q.alpha) {
    // temperature of the re-emitted Maxwellian: tau, or with energy
    // accommodation tau_r^2 = alpha_E tau^2 + (1 - alpha_E) |w|^2 / 2
    float tr = q.tau;
    if (q.eacc) {
      const float e_in = wx * wx + wy * wy + wz * wz;
      const float tr2 = q.alpha_E * q.tau * q.tau + (1.0f - q.alpha_E) * 0.5f * e_in;
      limited = tr2 > q.tr_cap2;
      tr = sqrtf(fminf(tr2, q.tr_cap2));
    }
    const float sg = wn < 0.0f ? 1.0f : -1.0f;
    const float sx = sg * nx, sy = sg * ny, sz = sg * nz;
    // orthonormal tangents of (sx, sy, sz) (Duff et al., JCGT 2017)
    const float sign = sz >= 0.0f ? 1.0f : -1.0f;
    const float a = -1.0f / (sign + sz);
    const float b = sx * sy * a;
    const float b1x = 1.0f + sign * sx * sx * a, b1y = sign * b, b1z = -sign * sx;
    const float b2x = b, b2y = sign + sy * sy * a, b2z = -sy;
    const float vn = tr * sqrtf(-logf(unif32(r.b)));
    const float rad = tr * sqrtf(-2.0f * logf(unif32(r.c))) * (float)kInvSqrt2;
    float sn, cs;
    sincospif(2.0f * unif32(r.d), &sn, &cs);
    const float v1 = rad * cs, v2 = rad * sn;
    wx = vn * sx + v1 * b1x + v2 * b2x;
    wy = vn * sy + v1 * b1y + v2 * b2y;
    wz = vn * sz + v1 * b1z + v2 * b2z;
  } else {
    const float k = 2.0f * wn;
    wx -= k * nx;
    wy -= k * ny;
    wz -= k * nz;
  }
  return limited;
}

// ---------------------------------------------------------------------------
// Fixed point and wave-level reductions.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long fx(float v, float scale) { return __float2ll_rn(v * scale); }
// The same for |v * scale| < 2^31: round to nearest even, then a 32-bit
// conversion (3 instructions instead of 12).
__device__ __forceinline__ long long fx32(float v, float scale) { return (long long)(int)rintf(v * scale); }
__device__ __forceinline__ long long fxd(double v, double scale) { return __double2ll_rn(v * scale); }

__device__ __forceinline__ long long wave_sum(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// The wave's total in scalar registers (the same value in every lane).
__device__ __forceinline__ long long wave_sum_uniform(long long v) {
  const long long t = wave_sum(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)t);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((unsigned long long)t >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ void atomic_add_i64(long long* p, long long v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}

}  // namespace tpmc
