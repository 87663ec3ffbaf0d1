// tpmc_math.hpp -- FP64 logarithm, sine and cosine of the seeding draws.
//
// The seeding draws are u = (k + 1/2) 2^-32 for a 32-bit integer k (unif64 in
// tpmc_device.hpp), so u = n 2^-33 with n = 2k + 1 odd, and the reduction is
// exact in integer arithmetic: ln u = ln n - 33 ln 2 with n = m 2^e exactly,
// m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...),
// s = (m - 1)/(m + 1), |s| <= 0.1716, series to s^21 (first omitted term
// below 1e-18 relative); e ln 2 is split as e ln2_hi (exact: ln2_hi has 46
// significant bits) plus e ln2_lo.  The result stays within 1.5 ulp of ln u
// over every k (a CPU test compares it with 40-digit values; the largest
// errors sit near u = 0.7, where -ln 2 and ln m partly cancel), with about
// 30 % fewer instructions than a general-argument log.  The coefficients 2/(2j+1)
// are rounded to the nearest double.
#ifndef TPMC_MATH_HPP
#define TPMC_MATH_HPP

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpmc {

// ln(u) for u = (k + 1/2) 2^-32.
__host__ __device__ inline double log_draw(uint32_t k) {
  const uint64_t n = 2ull * k + 1ull;  // u = n 2^-33
  int e = 63 - __builtin_clzll(n);     // n = m 2^e, m in [1, 2)
  double m = ldexp((double)n, -e);
  if (m > 0x1.6a09e667f3bcdp+0) {      // sqrt(2)
    m *= 0.5;
    ++e;
  }
  // s = (m - 1)/(m + 1) without the general division's scaling and fix-up
  // steps (its operands are far from every special case): a reciprocal, two
  // Newton steps, and the remainder correction that rounds the quotient
  const double num = m - 1.0, den = m + 1.0;
#ifdef __HIP_DEVICE_COMPILE__
  double r = __builtin_amdgcn_rcp(den);
#else
  double r = 1.0 / den;
#endif
  r = fma(fma(-den, r, 1.0), r, r);
  r = fma(fma(-den, r, 1.0), r, r);
  const double q0 = num * r;
  const double s = fma(fma(-den, q0, num), r, q0);
  const double w = s * s;
  double p = 0x1.8618618618618p-4;  // 2/21
  p = fma(p, w, 0x1.af286bca1af28p-4);
  p = fma(p, w, 0x1.e1e1e1e1e1e1ep-4);
  p = fma(p, w, 0x1.1111111111111p-3);
  p = fma(p, w, 0x1.3b13b13b13b14p-3);
  p = fma(p, w, 0x1.745d1745d1746p-3);
  p = fma(p, w, 0x1.c71c71c71c71cp-3);
  p = fma(p, w, 0x1.2492492492492p-2);
  p = fma(p, w, 0x1.999999999999ap-2);
  p = fma(p, w, 0x1.5555555555555p-1);  // 2/3
  const double lm = fma(s * w, p, 2.0 * s);  // ln m = 2s + s w P(w)
  const double E = (double)(e - 33);
  return fma(E, 0x1.62e42fefa3980p-1, fma(E, 0x1.bcd5e4f1d9cc0p-47, lm));
}

// sin(2 pi u) and cos(2 pi u) for u = (k + 1/2) 2^-32, from a table of
// sin and cos at the 256 angles 2 pi j / 256 (tab[2j], tab[2j + 1]) and the
// angle addition formulas: with n = 2k + 1 the angle is pi n 2^-32, its top
// eight bits j = n >> 25 pick the table angle a = 2 pi j / 256, and the rest
// delta = pi (n mod 2^25) 2^-32 in [0, 2 pi / 256) is exact up to the rounding
// of pi 2^-32; sin(delta) to delta^7 and cos(delta) to delta^6 (first omitted
// terms below 1e-17 absolute).  Within two ulps of the exact values when the
// table entries are within one (a CPU test compares with 40-digit values).
__host__ __device__ inline void sincos_2pi_draw(const double* __restrict__ tab, uint32_t k, double& s, double& c) {
  const uint64_t n = 2ull * k + 1ull;
  const uint32_t j = (uint32_t)(n >> 25);                       // 0..255
  const double d = (double)(uint32_t)(n & 0x1FFFFFFull) * 0x1.921fb54442d18p-31;  // pi 2^-32 per unit
  const double z = d * d;
  const double sd = d * fma(z, fma(z, fma(z, -0x1.a01a01a01a01ap-13, 0x1.1111111111111p-7), -0x1.5555555555555p-3), 1.0);
  const double cd = fma(z, fma(z, fma(z, -0x1.6c16c16c16c17p-10, 0x1.5555555555555p-5), -0.5), 1.0);
  const double sa = tab[2 * j], ca = tab[2 * j + 1];
  s = fma(sa, cd, ca * sd);
  c = fma(ca, cd, -(sa * sd));
}

// exp(-y^2) and erfc(y) for y >= 0 from a table of both at the grid points
// y_j = j / 256 (tab[2j] = exp(-y_j^2), tab[2j + 1] = erfc(y_j), j = 0 ..
// kExpErfcN - 1, so y_j up to 27.5) and a Taylor shift by h = y - y_j,
// |h| <= 1/512 (exact: y_j has eight fractional bits).  With the physicists'
// Hermite polynomials H_n (generating function exp(2xh - h^2) = sum_n H_n(x)
// h^n / n!) and a_n = H_n(-y_j) h^n / n!,
//   exp(-(y_j + h)^2) = exp(-y_j^2) sum_n a_n,
//   erfc(y_j + h)     = erfc(y_j) - 2/sqrt(pi) exp(-y_j^2) sum_n a_n h / (n + 1),
// and H_{n+1}(x) = 2x H_n(x) - 2n H_{n-1}(x) gives
// a_{n+1} = (-2 y_j h a_n - 2 h^2 a_{n-1}) / (n + 1).  The terms fall at least
// as fast as (2 y_j |h|)^n / n! <= 0.11^n / n!, so kExpErfcTerms terms leave a
// truncation error below 1e-17 relative to the leading term over the whole
// table; a CPU test compares both results with 40-digit values.  Above the
// table both values underflow to zero.  About 70 FP64 operations and one
// 16-byte load, against about 180 for a library exp and erfc.
constexpr int kExpErfcN = 7041;
constexpr double kExpErfcYmax = 27.5;  // (kExpErfcN - 1) / 256
constexpr int kExpErfcTerms = 10;

template <int NTERMS = kExpErfcTerms>
__host__ __device__ inline void exp_erfc_grid(const double* __restrict__ tab, double y, double& e, double& ta) {
  const bool inside = y < kExpErfcYmax;
  const double yc = fmin(y, kExpErfcYmax);  // computed for every y, selected below
  const double jf = rint(yc * 256.0);
  const int j = (int)jf;
  const double h = yc - jf * 0x1p-8;
  const double p = -2.0 * (jf * 0x1p-8) * h;
  const double q = -2.0 * h * h;
  // the terms after a_0 are summed on their own (small first to large last
  // does not matter here: each is below 0.11 of the one before), so that the
  // leading 1 enters once, in the final fma
  double am = 1.0, a = p;  // a_0, a_1
  double se = a;           // sum_{n>=1} a_n
  double si = 0.5 * a;     // sum_{n>=1} a_n / (n + 1)
#pragma unroll
  for (int n = 1; n < NTERMS - 1; ++n) {
    const double an = fma(q, am, p * a) * (1.0 / (double)(n + 1));
    am = a;
    a = an;
    se += a;
    si = fma(a, 1.0 / (double)(n + 2), si);
#ifdef __HIP_DEVICE_COMPILE__
    // keep each term's sums in its iteration: scheduled after the whole
    // recurrence, every term would stay live until the end (16 more VGPRs)
    __asm__ volatile("" : "+v"(se), "+v"(si), "+v"(a), "+v"(am));
#endif
  }
  const double e0 = tab[2 * j], t0 = tab[2 * j + 1];
  e = inside ? fma(e0, se, e0) : 0.0;
  ta = inside ? fma(-0x1.20dd750429b6dp+0 * e0, fma(h, si, h), t0) : 0.0;  // 2/sqrt(pi)
}

// erfcx(y) = exp(y^2) erfc(y) for y >= 0 in FP32, for the FP32 approach of the
// seeding solves (which have exp(-y^2) already, so erfc(y) = exp(-y^2) erfcx(y)
// costs a dozen operations instead of a library erfcf).  (1 + 2y) erfcx(y) is a
// smooth function of t = (y - 2)/(y + 2) on [-1, 1) (the change of variable of
// Schonfelder's and of Shepherd and Laframboise's erfc expansions), here a
// degree-10 polynomial interpolating 40-digit values at the Chebyshev nodes,
// rounded to FP32: within 3e-7 relative over [0, inf) (a CPU test checks it).
// The reciprocals are the hardware's on the device (1 ulp).
__host__ __device__ inline float erfcx32(float y) {
#ifdef __HIP_DEVICE_COMPILE__
  const float t = (y - 2.0f) * __builtin_amdgcn_rcpf(y + 2.0f);
#else
  const float t = (y - 2.0f) / (y + 2.0f);
#endif
  float p = 0x1.5bd97ap-13f;
  p = fmaf(p, t, -0x1.7eaf24p-13f);
  p = fmaf(p, t, -0x1.71314ap-10f);
  p = fmaf(p, t, 0x1.10c17cp-10f);
  p = fmaf(p, t, 0x1.1d16b6p-7f);
  p = fmaf(p, t, -0x1.04337ap-7f);
  p = fmaf(p, t, -0x1.bc22fcp-5f);
  p = fmaf(p, t, 0x1.4ff1bap-3f);
  p = fmaf(p, t, -0x1.5407dap-3f);
  p = fmaf(p, t, -0x1.7bf518p-4f);
  p = fmaf(p, t, 0x1.46e80ep+0f);
#ifdef __HIP_DEVICE_COMPILE__
  return p * __builtin_amdgcn_rcpf(fmaf(2.0f, y, 1.0f));
#else
  return p / fmaf(2.0f, y, 1.0f);
#endif
}

}  // namespace tpmc

#endif  // TPMC_MATH_HPP
