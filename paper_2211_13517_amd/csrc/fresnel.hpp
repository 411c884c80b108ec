// FP64 Fresnel integrals and the accelerated-sinusoid response rho(q, z).
//
// F(x) = C(x) + i S(x) = int_0^x exp(i pi t^2 / 2) dt.
//  * |x| < 2: power series F(x) = sum_n (i pi/2)^n x^(2n+1) / (n! (2n+1)).
//  * |x| >= 2: F(x) = sgn(x) (1+i)/2 + exp(i pi x^2/2) Phi(x) with
//    Phi(x) = -sgn(x) (1+i)/(2 sqrt(pi)) K(w), w = (sqrt(pi)/2)(1-i)|x|, where
//    K(w) = sqrt(pi) exp(w^2) erfc(w) = 1/(w + (1/2)/(w + (2/2)/(w + (3/2)/(w + ...))))
//    is Laplace's continued fraction for erfc, evaluated backwards at a fixed
//    depth (60 terms at |x| < 3, 32 below 6, 16 beyond: converged to rounding).
//    This follows from F(x) = (1+i)/2 erf((sqrt(pi)/2)(1-i) x).
//
// rho(q, z) = int_0^1 exp(-2 pi i q u + i pi z (u-1/2)^2) du = e^{-i pi q} R(q, z);
// for z > 0, with y+- = sqrt(2/z)(+-z/2 - q),
//   R = exp(-i pi q^2/z)/sqrt(2z) [F(y+) - F(y-)].
// Substituting the decomposition of F removes the large phase q^2/z exactly
// (pi y+-^2/2 = pi (z/4 -+ q + q^2/z)):
//   R = (1/sqrt(2z)) [ (sgn y+ - sgn y-)(1+i)/2 e^{-i pi q^2/z}
//                      + e^{i pi (z/4 - q)} Phi(y+) - e^{i pi (z/4 + q)} Phi(y-) ].
// When y+ and y- are non-zero with the same sign (|q| > z/2) the first term
// vanishes and no phase grows with q^2/z; otherwise |q| <= z/2, the phase
// q^2/z is at most z/4 and the direct form F(y+) - F(y-) (a sum of same-sign
// terms, one of them zero when |q| = z/2) is used.
// z < 0 uses R(q, z) = conj R(-q, -z); z = 0 gives R = sinc q.
#pragma once

#include <hip/hip_runtime.h>

namespace fdas {

struct c64 {
  double re, im;
};

__host__ __device__ inline c64 c64add(c64 a, c64 b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ inline c64 c64sub(c64 a, c64 b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ inline c64 c64mul(c64 a, c64 b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline c64 c64scale(c64 a, double s) { return {a.re * s, a.im * s}; }
__host__ __device__ inline c64 c64conj(c64 a) { return {a.re, -a.im}; }
__host__ __device__ inline c64 c64div(c64 a, c64 b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

__device__ inline c64 cispi64(double x) {
  double s, c;
  sincospi(x, &s, &c);
  return {c, s};
}

constexpr double kPi64 = 3.141592653589793238462643383279502884;
constexpr double kSqrtPi = 1.772453850905516027298167483341145183;

__device__ inline c64 fresnel_series(double x) {
  const double a = 0.5 * kPi64 * x * x;
  c64 t = {x, 0.0};
  c64 s = {0.0, 0.0};
  for (int n = 0; n < 80; ++n) {
    s = c64add(s, c64scale(t, 1.0 / (2 * n + 1)));
    const double f = a / (n + 1);
    t = {-t.im * f, t.re * f};  // t *= i a / (n+1)
    if (fabs(t.re) + fabs(t.im) < 1e-18 * (fabs(s.re) + fabs(s.im))) break;
  }
  return s;
}

// Phi(|x|) for |x| >= 2 (positive-argument branch).
__device__ inline c64 fresnel_phi_big(double ax) {
  const int depth = ax < 3.0 ? 60 : (ax < 6.0 ? 32 : 16);
  const double h = 0.5 * kSqrtPi * ax;
  const c64 w = {h, -h};
  c64 f = w;
  for (int n = depth; n >= 1; --n) f = c64add(w, c64div({0.5 * n, 0.0}, f));
  const c64 k = c64div({1.0, 0.0}, f);
  return c64scale(c64mul({1.0, 1.0}, k), -0.5 / kSqrtPi);
}

// F(x) = sgn(x)(1+i)/2 + exp(i pi x^2/2) Phi(x)
__device__ inline c64 fresnel_phi(double t) {
  if (t == 0.0) return {0.0, 0.0};
  const double sg = t > 0 ? 1.0 : -1.0;
  const double at = fabs(t);
  if (at >= 2.0) return c64scale(fresnel_phi_big(at), sg);
  const c64 f = fresnel_series(t);
  const c64 d = {f.re - 0.5 * sg, f.im - 0.5 * sg};
  return c64mul(d, cispi64(-0.5 * t * t));
}

__device__ inline c64 fresnel_F(double x) {
  const double ax = fabs(x);
  if (ax < 2.0) return fresnel_series(x);
  const double sg = x > 0 ? 1.0 : -1.0;
  const c64 p = c64mul(cispi64(0.5 * ax * ax), fresnel_phi_big(ax));
  return c64scale({0.5 + p.re, 0.5 + p.im}, sg);
}

// rho(q, z) in FP64.
__device__ inline c64 response64(double q, double z) {
  if (z == 0.0) {
    const double sinc = (q == 0.0) ? 1.0 : sinpi(q) / (kPi64 * q);
    return c64scale(cispi64(-q), sinc);
  }
  const bool neg = z < 0.0;
  const double qq = neg ? -q : q;
  const double za = fabs(z);
  const double s = sqrt(2.0 / za);
  const double yp = s * (0.5 * za - qq), ym = s * (-0.5 * za - qq);
  const double inv = 1.0 / sqrt(2.0 * za);
  c64 r;
  if ((yp > 0.0 && ym > 0.0) || (yp < 0.0 && ym < 0.0)) {
    const c64 a = c64mul(cispi64(0.25 * za - qq), fresnel_phi(yp));
    const c64 b = c64mul(cispi64(0.25 * za + qq), fresnel_phi(ym));
    r = c64scale(c64sub(a, b), inv);
  } else {
    const c64 d = c64sub(fresnel_F(yp), fresnel_F(ym));
    r = c64scale(c64mul(cispi64(-qq * qq / za), d), inv);
  }
  if (neg) r = c64conj(r);
  return c64mul(cispi64(-q), r);
}

}  // namespace fdas
