// Fourier-interpolated power P(r, z) at off-grid candidates, its
// adjoint, and gradient-ascent refinement.
//
// y(r, z) = sum_{k = k0-w+1}^{k0+w} A_k conj(rho(k - r, z)),  k0 = floor(r),
// w = m + ceil(|z|/2) (A_k = 0 outside the spectrum), P = |y|^2.
// dy/dr = -sum A_k conj(d rho/dq), dy/dz = sum A_k conj(d rho/dz),
// dP/dr = 2 Re(conj(y) dy/dr), dP/dz = 2 Re(conj(y) dy/dz), and the gradient
// with respect to A_k (as d/dRe + i d/dIm) is 2 y rho(k - r, z).
//
// Derivatives of rho (phi(u) = -2 pi q u + pi z (u-1/2)^2):
//  * |z| >= 0.05: integrating phi'(u) e^{i phi} by parts,
//      I1 = int (u-1/2) e^{i phi} = (q rho + (e1 - e0)/(2 pi i)) / z,
//      I2 = int (u-1/2)^2 e^{i phi} = (q I1 + ((e1 + e0)/2 - rho)/(2 pi i)) / z,
//    e0 = e^{i phi(0)}, e1 = e^{i phi(1)}; d rho/dq = -2 pi i (I1 + rho/2), d rho/dz = i pi I2.
//  * |z| < 0.05 (where those quotients cancel): expanding e^{i pi z v^2},
//      rho = e^{-i pi q} sum_n c_n M_{2n},  c_n = (i pi z)^n / n!,
//      d rho/dq = e^{-i pi q} sum_n c_n (-i pi M_{2n} - 2 pi i M_{2n+1}),
//      d rho/dz = e^{-i pi q} i pi sum_n c_n M_{2n+2},
//    with the moments M_k(q) = int_{-1/2}^{1/2} v^k e^{-2 pi i q v} dv from their
//    Taylor series in 2 pi q (|2 pi q| < 10) or the upward recurrence of
//    integration by parts.
// All of this runs in FP64: on CDNA4 the FP64 vector rate equals the
// unpacked FP32 rate, so FP64 costs no extra issue slots here.
#include "fresnel.hpp"
#include "launch.hpp"

namespace fdas {

constexpr double kZTaylor = 0.05;
constexpr int kTaylorTerms = 9;           // n = 0..8
constexpr int kMoments = 2 * kTaylorTerms + 2;

__device__ inline void moments(double q, c64* M) {
  const double c = 2.0 * kPi64 * q;
  if (fabs(c) < 10.0) {
    // M_k = sum_j (-i c)^j / j! mu_{k+j},  mu_n = 2^-n/(n+1) for even n, 0 for odd n
    for (int k = 0; k < kMoments; ++k) {
      c64 acc = {0.0, 0.0};
      c64 t = {1.0, 0.0};  // (-i c)^j / j!
      for (int j = 0; j < 60; ++j) {
        const int n = k + j;
        if ((n & 1) == 0) {
          const double mu = ldexp(1.0, -n) / (n + 1);
          acc = c64add(acc, c64scale(t, mu));
        }
        t = c64scale(c64mul(t, {0.0, -c}), 1.0 / (j + 1));
        if (fabs(t.re) + fabs(t.im) < 1e-30) break;
      }
      M[k] = acc;
    }
  } else {
    const c64 ep = cispi64(-q), em = cispi64(q);  // e^{-i c/2}, e^{+i c/2}
    M[0] = {2.0 * sinpi(q) / c, 0.0};
    const c64 inv_mic = {0.0, 1.0 / c};            // 1/(-i c) = i/c
    double h = 1.0;
    for (int k = 1; k < kMoments; ++k) {
      h *= 0.5;
      const double sg = (k & 1) ? -1.0 : 1.0;      // (-1/2)^k = sg * 2^-k
      const c64 b = c64scale(c64sub(ep, c64scale(em, sg)), h);
      // M_k = b/(-ic) + (k/(ic)) M_{k-1} = (b - k M_{k-1}) / (-ic)
      M[k] = c64mul(c64sub(b, c64scale(M[k - 1], (double)k)), inv_mic);
    }
  }
}

struct RhoD {
  c64 rho, dq, dz;
};

__device__ inline RhoD response_d64(double q, double z) {
  RhoD o;
  if (fabs(z) >= kZTaylor) {
    o.rho = response64(q, z);
    const c64 e0 = cispi64(0.25 * z);
    const c64 e1 = cispi64(0.25 * z - 2.0 * q);
    const c64 inv2pii = {0.0, -1.0 / (2.0 * kPi64)};  // 1/(2 pi i)
    const c64 i1 = c64scale(c64add(c64scale(o.rho, q), c64mul(c64sub(e1, e0), inv2pii)), 1.0 / z);
    const c64 mid = c64sub(c64scale(c64add(e1, e0), 0.5), o.rho);
    const c64 i2 = c64scale(c64add(c64scale(i1, q), c64mul(mid, inv2pii)), 1.0 / z);
    const c64 s = c64add(i1, c64scale(o.rho, 0.5));
    o.dq = c64mul({0.0, -2.0 * kPi64}, s);
    o.dz = c64mul({0.0, kPi64}, i2);
    return o;
  }
  c64 M[kMoments];
  moments(q, M);
  c64 r = {0.0, 0.0}, dq1 = {0.0, 0.0}, dz1 = {0.0, 0.0};
  c64 cn = {1.0, 0.0};
  for (int n = 0; n < kTaylorTerms; ++n) {
    r = c64add(r, c64mul(cn, M[2 * n]));
    dq1 = c64add(dq1, c64mul(cn, M[2 * n + 1]));
    dz1 = c64add(dz1, c64mul(cn, M[2 * n + 2]));
    cn = c64scale(c64mul(cn, {0.0, kPi64 * z}), 1.0 / (n + 1));
  }
  const c64 ph = cispi64(-q);
  o.rho = c64mul(ph, r);
  o.dq = c64mul(ph, c64add(c64mul({0.0, -kPi64}, r), c64mul({0.0, -2.0 * kPi64}, dq1)));
  o.dz = c64mul(ph, c64mul({0.0, kPi64}, dz1));
  return o;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int SDT>
__device__ inline c64 spec_at(const void* spec, int64_t nb, int64_t k) {
  using SS = Store<SDT>;
  if (k < 0 || k >= nb) return {0.0, 0.0};
  const c32 v = SS::unpack(reinterpret_cast<const typename SS::cplx_t*>(spec)[k]);
  return {(double)v.re, (double)v.im};
}

struct RzEval {
  c64 y, dydr, dydz;
};

// Positions the evaluation accepts: finite, |r| < 2^52 (so floor(r) is exact
// in int64) and |z| <= 2^17 (a window of at most 2^17 + 2 margin bins).
// Anything else evaluates to NaN without touching the spectrum, so that no
// input can make the window loop run away.
constexpr double kMaxAbsZ = 131072.0, kMaxAbsR = 4503599627370496.0;
__device__ inline bool rz_valid(double r, double z) { return fabs(r) < kMaxAbsR && fabs(z) <= kMaxAbsZ; }

// One wavefront evaluates y (and optionally its r, z derivatives) at (r, z).
template <int SDT, bool GRAD>
__device__ inline RzEval rz_eval(const void* spec, int64_t nb, double r, double z, int margin) {
  if (!rz_valid(r, z)) {  // also false for NaN
    const double q = __builtin_nan("");
    return RzEval{{q, q}, {q, q}, {q, q}};
  }
  const int64_t k0 = (int64_t)floor(r);
  const int w = margin + (int)ceil(fabs(z) * 0.5);
  const int lane = threadIdx.x & 63;
  c64 y = {0, 0}, dr = {0, 0}, dz = {0, 0};
  for (int t = lane; t < 2 * w; t += 64) {
    const int64_t k = k0 - w + 1 + t;
    const c64 a = spec_at<SDT>(spec, nb, k);
    if (a.re == 0.0 && a.im == 0.0) continue;
    if (GRAD) {
      const RhoD d = response_d64((double)k - r, z);
      y = c64add(y, c64mul(a, c64conj(d.rho)));
      dr = c64sub(dr, c64mul(a, c64conj(d.dq)));
      dz = c64add(dz, c64mul(a, c64conj(d.dz)));
    } else {
      y = c64add(y, c64mul(a, c64conj(response64((double)k - r, z))));
    }
  }
  RzEval e;
  e.y = {wave_sum(y.re), wave_sum(y.im)};
  if (GRAD) {
    e.dydr = {wave_sum(dr.re), wave_sum(dr.im)};
    e.dydz = {wave_sum(dz.re), wave_sum(dz.im)};
  }
  return e;
}

template <int SDT>
__global__ __launch_bounds__(256) void k_rz_power(const void* spec, int64_t nb, const double* r, const double* z, int64_t n,
                                                  int margin, double* p, c64* y_out) {
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  const RzEval e = rz_eval<SDT, false>(spec, nb, r[c], z[c], margin);
  if ((threadIdx.x & 63) == 0) {
    p[c] = e.y.re * e.y.re + e.y.im * e.y.im;
    if (y_out) y_out[c] = e.y;
  }
}

// The spectrum gradient dP/dA_k = sum_c 2 g_c y_c rho(k - r_c, z_c) is summed
// in fixed point with 64-bit integer atomics: integer addition is
// associative, so the sum does not depend on the arrival order.  Its unit
// 2^-s is chosen per call from a bound on the terms, so that no partial sum
// can overflow: |rho| <= 1 (an average of unit-modulus values), hence every
// term of candidate c is at most b_c = 2 |g_c| |y_c| and every partial sum at
// most n max_c b_c; s is the largest integer <= 40 with
// n max_c b_c 2^s <= 2^61 (one bit of slack for rounding).  The maximum is
// taken with an integer atomic on the (non-negative) doubles' bit patterns,
// so it too is order-independent.  Terms that are not finite are skipped and
// latched (status bit 2).
constexpr int kFixMaxShift = 40;

template <int SDT>
__global__ __launch_bounds__(256) void k_grad_bound(const void* spec, int64_t nb, const double* r, const double* z,
                                                    const c64* y_in, const double* gp, int64_t n, int margin,
                                                    unsigned long long* max_bits, int32_t* status) {
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  const double rr = r[c], zz = z[c];
  if (!rz_valid(rr, zz)) return;  // such a candidate adds nothing to the spectrum gradient
  const c64 y = y_in ? y_in[c] : rz_eval<SDT, false>(spec, nb, rr, zz, margin).y;
  if ((threadIdx.x & 63) != 0) return;
  const double b = 2.0 * fabs(gp[c]) * sqrt(y.re * y.re + y.im * y.im);
  if (!isfinite(b)) {
    atomicOr(status, 2);
    return;
  }
  atomicMax(max_bits, (unsigned long long)__double_as_longlong(b));
}

__global__ void k_grad_scale(const unsigned long long* max_bits, int64_t n, double* scale) {
  const double t = (double)n * __longlong_as_double((long long)*max_bits);
  int sh = kFixMaxShift;
  if (!(t < 1e300)) sh = -1000;  // absurd terms: every partial sum stays far below 2^61
  else if (t > 0.0) sh = min(kFixMaxShift, 61 - (ilogb(t) + 1));  // t < 2^(ilogb(t) + 1)
  *scale = ldexp(1.0, sh);
}

template <int SDT>
__global__ __launch_bounds__(256) void k_rz_grad(const void* spec, int64_t nb, const double* r, const double* z,
                                                 const c64* y_in, const double* gp, int64_t n, int margin,
                                                 double* gr, double* gz, unsigned long long* acc,
                                                 const double* scale_p, int32_t* status) {
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  const double rr = r[c], zz = z[c];
  const RzEval e = rz_eval<SDT, true>(spec, nb, rr, zz, margin);
  const c64 y = y_in ? y_in[c] : e.y;
  const double g = gp[c];
  if ((threadIdx.x & 63) == 0) {
    gr[c] = g * 2.0 * (y.re * e.dydr.re + y.im * e.dydr.im);
    gz[c] = g * 2.0 * (y.re * e.dydz.re + y.im * e.dydz.im);
  }
  if (!acc || !rz_valid(rr, zz)) return;
  const double scale = *scale_p;
  const int64_t k0 = (int64_t)floor(rr);
  const int w = margin + (int)ceil(fabs(zz) * 0.5);
  for (int t = threadIdx.x & 63; t < 2 * w; t += 64) {
    const int64_t k = k0 - w + 1 + t;
    if (k < 0 || k >= nb) continue;
    const c64 v = c64scale(c64mul(y, response64((double)k - rr, zz)), 2.0 * g);
    const double a = v.re * scale, b = v.im * scale;
    if (!(fabs(a) <= 4611686018427387904.0 && fabs(b) <= 4611686018427387904.0)) {  // 2^62; also NaN
      atomicOr(status, 2);
      continue;
    }
    atomicAdd(acc + 2 * k, (unsigned long long)(long long)llrint(a));
    atomicAdd(acc + 2 * k + 1, (unsigned long long)(long long)llrint(b));
  }
}

__global__ void k_fix_clear(unsigned long long* acc, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc[i] = 0ull;
}

__global__ void k_fix_to_float(const unsigned long long* acc, float* out, int64_t n, const double* scale_p) {
  const double inv = 1.0 / *scale_p;  // a power of two: exact
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)((double)(long long)acc[i] * inv);
}

// Preconditioned gradient ascent: near a peak P ~ P0 (1 - a dr^2 - b dz^2)
// with a = pi^2/3 (sinc main lobe) and b = pi^2/180 (quadratic-phase
// mismatch), so the step (g_r / (2 a P), g_z / (2 b P)) is Newton's step for
// that model; it is clamped and halved until P increases.
template <int SDT>
__global__ __launch_bounds__(256) void k_refine(const void* spec, int64_t nb, double* r, double* z, int64_t n, int iters,
                                                int margin, double* p_final) {
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  constexpr double A = kPi64 * kPi64 / 3.0, B = kPi64 * kPi64 / 180.0;
  double rr = r[c], zz = z[c];
  RzEval e = rz_eval<SDT, true>(spec, nb, rr, zz, margin);
  double P = e.y.re * e.y.re + e.y.im * e.y.im;
  for (int it = 0; it < iters && P > 0.0; ++it) {
    const double gr = 2.0 * (e.y.re * e.dydr.re + e.y.im * e.dydr.im);
    const double gz = 2.0 * (e.y.re * e.dydz.re + e.y.im * e.dydz.im);
    double sr = fmin(fmax(gr / (2.0 * A * P), -0.25), 0.25);
    double sz = fmin(fmax(gz / (2.0 * B * P), -2.0), 2.0);
    bool moved = false;
    for (int ls = 0; ls < 8; ++ls) {
      const RzEval t = rz_eval<SDT, true>(spec, nb, rr + sr, zz + sz, margin);
      const double Pt = t.y.re * t.y.re + t.y.im * t.y.im;
      if (Pt > P) {
        rr += sr;
        zz += sz;
        P = Pt;
        e = t;
        moved = true;
        break;
      }
      sr *= 0.5;
      sz *= 0.5;
    }
    if (!moved || (fabs(sr) < 1e-7 && fabs(sz) < 1e-6)) break;
  }
  // final FP64 evaluation at the returned position
  const RzEval f = rz_eval<SDT, false>(spec, nb, rr, zz, margin);
  if ((threadIdx.x & 63) == 0) {
    r[c] = rr;
    z[c] = zz;
    p_final[c] = f.y.re * f.y.re + f.y.im * f.y.im;
  }
}

// Sum over harmonics k = 1..H of a fundamental (r, z): S = sum_k P(k r, k z),
// dS/dr = sum_k k dP/dr(k r, k z), likewise in z, and the curvature weight
// sum_k k^2 P_k of the peak model P_k ~ P_k0 (1 - a (k dr)^2 - b (k dz)^2).
struct HarmEval {
  double S, gr, gz, curv;
};

template <int SDT, bool GRAD>
__device__ inline HarmEval harm_eval(const void* spec, int64_t nb, double r, double z, int H, int margin) {
  HarmEval h = {0.0, 0.0, 0.0, 0.0};
  for (int k = 1; k <= H; ++k) {
    const double kd = (double)k;
    const RzEval e = rz_eval<SDT, GRAD>(spec, nb, kd * r, kd * z, margin);
    const double P = e.y.re * e.y.re + e.y.im * e.y.im;
    h.S += P;
    if (GRAD) {
      h.gr += kd * (2.0 * (e.y.re * e.dydr.re + e.y.im * e.dydr.im));
      h.gz += kd * (2.0 * (e.y.re * e.dydz.re + e.y.im * e.dydz.im));
      h.curv += kd * kd * P;
    }
  }
  return h;
}

// The same sums with four harmonics evaluated at once: the wavefront splits
// into four groups of 16 lanes, group g taking harmonics g + 1, g + 5, ...;
// each group reduces its harmonic over its 16 lanes, then the four groups'
// partial sums are added.  Short windows (32-40 bins at small z) keep all
// 64 lanes busy this way instead of about half of them.
template <int SDT, bool GRAD>
__device__ inline HarmEval harm_eval4(const void* spec, int64_t nb, double r, double z, int H, int margin) {
  constexpr int GL = 16;
  const int lane = threadIdx.x & 63, g = lane / GL, gl = lane % GL;
  HarmEval h = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 1; k0 <= H; k0 += 64 / GL) {
    const int k = k0 + g;
    const double kd = (double)k, kr = kd * r, kz = kd * z;
    c64 y = {0.0, 0.0}, dr = {0.0, 0.0}, dz = {0.0, 0.0};
    if (k <= H && rz_valid(kr, kz)) {
      const int64_t b0 = (int64_t)floor(kr);
      const int w = margin + (int)ceil(fabs(kz) * 0.5);
      for (int t = gl; t < 2 * w; t += GL) {
        const int64_t b = b0 - w + 1 + t;
        const c64 a = spec_at<SDT>(spec, nb, b);
        if (a.re == 0.0 && a.im == 0.0) continue;
        if (GRAD) {
          const RhoD d = response_d64((double)b - kr, kz);
          y = c64add(y, c64mul(a, c64conj(d.rho)));
          dr = c64sub(dr, c64mul(a, c64conj(d.dq)));
          dz = c64add(dz, c64mul(a, c64conj(d.dz)));
        } else {
          y = c64add(y, c64mul(a, c64conj(response64((double)b - kr, kz))));
        }
      }
    } else if (k <= H) {
      y.re = __builtin_nan("");  // an invalid harmonic makes S NaN
    }
#pragma unroll
    for (int o = GL / 2; o > 0; o >>= 1) {
      y.re += __shfl_xor(y.re, o, 64);
      y.im += __shfl_xor(y.im, o, 64);
      if (GRAD) {
        dr.re += __shfl_xor(dr.re, o, 64);
        dr.im += __shfl_xor(dr.im, o, 64);
        dz.re += __shfl_xor(dz.re, o, 64);
        dz.im += __shfl_xor(dz.im, o, 64);
      }
    }
    if (k <= H) {
      const double P = y.re * y.re + y.im * y.im;
      h.S += P;
      if (GRAD) {
        h.gr += kd * (2.0 * (y.re * dr.re + y.im * dr.im));
        h.gz += kd * (2.0 * (y.re * dz.re + y.im * dz.im));
        h.curv += kd * kd * P;
      }
    }
  }
  // every lane of a group holds its group's sums: add the four groups
#pragma unroll
  for (int o = GL; o < 64; o <<= 1) {
    h.S += __shfl_xor(h.S, o, 64);
    if (GRAD) {
      h.gr += __shfl_xor(h.gr, o, 64);
      h.gz += __shfl_xor(h.gz, o, 64);
      h.curv += __shfl_xor(h.curv, o, 64);
    }
  }
  return h;
}

// One harmonic: the single-harmonic evaluation itself (so that H = 1 is
// fdas_refine step for step); more: four at a time.
template <int SDT, bool GRAD>
__device__ inline HarmEval harm_sum(const void* spec, int64_t nb, double r, double z, int H, int margin) {
  return H == 1 ? harm_eval<SDT, GRAD>(spec, nb, r, z, H, margin) : harm_eval4<SDT, GRAD>(spec, nb, r, z, H, margin);
}

// Ascent of S at the fundamental with the Newton step of the summed peak
// model, (dS/dr / (2 a sum k^2 P_k), dS/dz / (2 b sum k^2 P_k)), clamped to
// 0.25/H bin and 2/H z (a quarter bin at the top harmonic) and halved until S
// grows.  For H = 1 this is exactly the single-harmonic refinement.
template <int SDT>
__global__ __launch_bounds__(256) void k_refine_harm(const void* spec, int64_t nb, double* r, double* z,
                                                     const int32_t* harm, int64_t n, int iters, int margin,
                                                     double* p_final) {
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  const int H = harm[c];
  if (H < 1 || H > 32) {  // invalid count: position untouched, result NaN
    if ((threadIdx.x & 63) == 0) p_final[c] = __builtin_nan("");
    return;
  }
  constexpr double A = kPi64 * kPi64 / 3.0, B = kPi64 * kPi64 / 180.0;
  const double hd = (double)H;
  double rr = r[c], zz = z[c];
  HarmEval e = harm_sum<SDT, true>(spec, nb, rr, zz, H, margin);
  for (int it = 0; it < iters && e.S > 0.0; ++it) {
    double sr = fmin(fmax(e.gr / (2.0 * A * e.curv), -0.25 / hd), 0.25 / hd);
    double sz = fmin(fmax(e.gz / (2.0 * B * e.curv), -2.0 / hd), 2.0 / hd);
    bool moved = false;
    for (int ls = 0; ls < 8; ++ls) {
      const HarmEval t = harm_sum<SDT, true>(spec, nb, rr + sr, zz + sz, H, margin);
      if (t.S > e.S) {
        rr += sr;
        zz += sz;
        e = t;
        moved = true;
        break;
      }
      sr *= 0.5;
      sz *= 0.5;
    }
    if (!moved || (fabs(sr) < 1e-7 / hd && fabs(sz) < 1e-6 / hd)) break;
  }
  const HarmEval f = harm_sum<SDT, false>(spec, nb, rr, zz, H, margin);
  if ((threadIdx.x & 63) == 0) {
    r[c] = rr;
    z[c] = zz;
    p_final[c] = f.S;
  }
}

hipError_t launch_refine_harmonics(int sdt, const void* spec, int64_t nb, double* r, double* z, const int32_t* harm,
                                   int64_t n, int iters, int margin, double* p_final, hipStream_t st) {
  const dim3 g((unsigned)((n + 3) / 4));
  switch (sdt) {
    case FDAS_F32:
      hipLaunchKernelGGL((k_refine_harm<FDAS_F32>), g, dim3(256), 0, st, spec, nb, r, z, harm, n, iters, margin, p_final);
      break;
    case FDAS_BF16:
      hipLaunchKernelGGL((k_refine_harm<FDAS_BF16>), g, dim3(256), 0, st, spec, nb, r, z, harm, n, iters, margin, p_final);
      break;
    case FDAS_F16:
      hipLaunchKernelGGL((k_refine_harm<FDAS_F16>), g, dim3(256), 0, st, spec, nb, r, z, harm, n, iters, margin, p_final);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rz_power(int sdt, const void* spec, int64_t nb, const double* r, const double* z, int64_t n, int margin,
                           double* p, c64* y, hipStream_t st) {
  const dim3 g((unsigned)((n + 3) / 4));
  switch (sdt) {
    case FDAS_F32: hipLaunchKernelGGL((k_rz_power<FDAS_F32>), g, dim3(256), 0, st, spec, nb, r, z, n, margin, p, y); break;
    case FDAS_BF16: hipLaunchKernelGGL((k_rz_power<FDAS_BF16>), g, dim3(256), 0, st, spec, nb, r, z, n, margin, p, y); break;
    case FDAS_F16: hipLaunchKernelGGL((k_rz_power<FDAS_F16>), g, dim3(256), 0, st, spec, nb, r, z, n, margin, p, y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rz_grad(int sdt, const void* spec, int64_t nb, const double* r, const double* z, const c64* y,
                          const double* gp, int64_t n, int margin, double* gr, double* gz, float* gspec,
                          unsigned long long* acc, unsigned long long* max_bits, double* scale, int32_t* status,
                          hipStream_t st) {
  const dim3 g((unsigned)((n + 3) / 4));
  if (gspec) {
    hipLaunchKernelGGL(k_fix_clear, dim3(1024), dim3(256), 0, st, acc, 2 * nb);
    hipLaunchKernelGGL(k_fix_clear, dim3(1), dim3(64), 0, st, max_bits, (int64_t)1);
    switch (sdt) {
      case FDAS_F32: hipLaunchKernelGGL((k_grad_bound<FDAS_F32>), g, dim3(256), 0, st, spec, nb, r, z, y, gp, n, margin, max_bits, status); break;
      case FDAS_BF16: hipLaunchKernelGGL((k_grad_bound<FDAS_BF16>), g, dim3(256), 0, st, spec, nb, r, z, y, gp, n, margin, max_bits, status); break;
      case FDAS_F16: hipLaunchKernelGGL((k_grad_bound<FDAS_F16>), g, dim3(256), 0, st, spec, nb, r, z, y, gp, n, margin, max_bits, status); break;
      default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_grad_scale, dim3(1), dim3(1), 0, st, max_bits, n, scale);
  }
  unsigned long long* a = gspec ? acc : nullptr;
  switch (sdt) {
    case FDAS_F32: hipLaunchKernelGGL((k_rz_grad<FDAS_F32>), g, dim3(256), 0, st, spec, nb, r, z, y, gp, n, margin, gr, gz, a, scale, status); break;
    case FDAS_BF16: hipLaunchKernelGGL((k_rz_grad<FDAS_BF16>), g, dim3(256), 0, st, spec, nb, r, z, y, gp, n, margin, gr, gz, a, scale, status); break;
    case FDAS_F16: hipLaunchKernelGGL((k_rz_grad<FDAS_F16>), g, dim3(256), 0, st, spec, nb, r, z, y, gp, n, margin, gr, gz, a, scale, status); break;
    default: return hipErrorInvalidValue;
  }
  if (gspec) hipLaunchKernelGGL(k_fix_to_float, dim3(1024), dim3(256), 0, st, acc, gspec, 2 * nb, scale);
  return hipGetLastError();
}

hipError_t launch_refine(int sdt, const void* spec, int64_t nb, double* r, double* z, int64_t n, int iters, int margin,
                         double* p_final, hipStream_t st) {
  const dim3 g((unsigned)((n + 3) / 4));
  switch (sdt) {
    case FDAS_F32: hipLaunchKernelGGL((k_refine<FDAS_F32>), g, dim3(256), 0, st, spec, nb, r, z, n, iters, margin, p_final); break;
    case FDAS_BF16: hipLaunchKernelGGL((k_refine<FDAS_BF16>), g, dim3(256), 0, st, spec, nb, r, z, n, iters, margin, p_final); break;
    case FDAS_F16: hipLaunchKernelGGL((k_refine<FDAS_F16>), g, dim3(256), 0, st, spec, nb, r, z, n, iters, margin, p_final); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fdas
