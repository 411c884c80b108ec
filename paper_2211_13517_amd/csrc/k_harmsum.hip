// Rows a9-a10: nested incoherent harmonic sums over the power plane,
// thresholds and candidate compaction.
//
// Cell (R, j) holds the sum for a signal whose H-th harmonic sits at bin R and
// acceleration trial j (m = j - j0 trials from z = 0).  Harmonic k of H lies at
//   r_k = floor((2 k R + H) / (2 H)),  m_k = sgn(m) floor((2 k |m| + H) / (2 H)),
// i.e. k R / H and k m / H rounded half up (half away from zero in m, which
// keeps +z and -z symmetric), so r_H = R and m_H = m.  With H the top stage,
// the stage H' = H / s sums the terms k = s, 2s, ..., H exactly, hence one
// pass of H reads gives every stage.  A stage is searched where its
// fundamental R/H' is at least r_lo and R < N/2 - h_max, passes when
// S_H' >= tau_H', and a cell reports only its most significant passing stage
// (smallest noise tail probability P(Gamma(H', 1) > S), evaluated in FP64 for
// the few passing cells).
#include "launch.hpp"

namespace fdas {

constexpr int kHarmThreads = 256;

// ln P(Gamma(h, 1) > s) = -s + ln sum_{k<h} s^k / k!, integer h.
__device__ inline double log_tail_gamma(double s, int h) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < h; ++k) {
    term *= s / k;
    sum += term;
  }
  return -s + log(sum);
}

// Gaussian-equivalent significance: sigma with ln P(N(0,1) > sigma) = lq,
// by Newton steps on ln(erfcx(sigma/sqrt2)/2) - sigma^2/2.
__device__ inline double sigma_from_log_tail(double lq) {
  double x = sqrt(fmax(-2.0 * lq, 1.0));
  for (int it = 0; it < 30; ++it) {
    const double ex = erfcx(x * 0.70710678118654752440);
    const double f = log(0.5 * ex) - 0.5 * x * x - lq;
    const double fp = -0.79788456080286535588 / ex;  // -sqrt(2/pi)/erfcx
    const double dx = f / fp;
    x -= dx;
    if (fabs(dx) < 1e-12 * fmax(1.0, x)) break;
  }
  return x;
}

template <int PDT, int H>
__global__ __launch_bounds__(kHarmThreads) void k_harmsum(HarmArgs a) {
  using PS = Store<PDT>;
  using RT = typename PS::real_t;
  constexpr int NST = ilog2(H) + 1;
  const SeriesDesc d = a.desc[blockIdx.z];
  const int nb = d.nbins;
  const int R = blockIdx.x * kHarmThreads + threadIdx.x;
  if (R >= nb - a.hmax) return;
  const RT* plane = reinterpret_cast<const RT*>(a.plane) + d.plane_off;
  int rk[H];
#pragma unroll
  for (int k = 1; k <= H; ++k) rk[k - 1] = (2 * k * R + H) / (2 * H);
  const int jbeg = blockIdx.y * a.Z / gridDim.y, jend = (blockIdx.y + 1) * a.Z / gridDim.y;
  for (int j = jbeg; j < jend; ++j) {
    const int m = j - a.j0;
    const int am = m < 0 ? -m : m;
    float tk[H];
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      const int mk = (2 * k * am + H) / (2 * H);
      const int jk = a.j0 + (m < 0 ? -mk : mk);
      tk[k - 1] = PS::unpack_real(plane[(size_t)jk * nb + rk[k - 1]]);
    }
    float S[NST];
    bool any = false;
#pragma unroll
    for (int i = 0; i < NST; ++i) {
      const int step = H >> i;  // stage H' = 2^i uses k = step, 2 step, ..., H
      float sum = 0.f;
#pragma unroll
      for (int k = step; k <= H; k += step) sum += tk[k - 1];
      S[i] = sum;
      any |= (R >= (1 << i) * a.r_lo) && (sum >= a.tau[i]);
    }
    if (!any) continue;
    double best = 0.0;
    int bi = -1;
    for (int i = 0; i < NST; ++i) {
      if (!((R >= (1 << i) * a.r_lo) && (S[i] >= a.tau[i]))) continue;
      const double lq = log_tail_gamma((double)S[i], 1 << i);
      if (bi < 0 || lq < best) {
        best = lq;
        bi = i;
      }
    }
    const unsigned long long slot = atomicAdd(a.count, 1ull);
    if ((int64_t)slot < a.capacity) {
      const int hh = 1 << bi;
      fdas_candidate c;
      c.series = (int)blockIdx.z;
      c.harm = hh;
      c.R = R;
      c.j = j;
      c.r = (float)((double)R / hh);
      c.z = (float)((a.z_min + a.z_step * j) / hh);
      c.power = S[bi];
      c.sigma = (float)sigma_from_log_tail(best);
      a.cands[slot] = c;
    }
  }
}

template <int PDT, int H>
static void hs_launch(const HarmArgs& a, dim3 g, hipStream_t st) {
  hipLaunchKernelGGL((k_harmsum<PDT, H>), g, dim3(kHarmThreads), 0, st, a);
}

template <int PDT>
static hipError_t hs_h(const HarmArgs& a, dim3 g, hipStream_t st) {
  switch (a.n_harm) {
    case 1: hs_launch<PDT, 1>(a, g, st); break;
    case 2: hs_launch<PDT, 2>(a, g, st); break;
    case 4: hs_launch<PDT, 4>(a, g, st); break;
    case 8: hs_launch<PDT, 8>(a, g, st); break;
    case 16: hs_launch<PDT, 16>(a, g, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The x-grid covers the longest series; blocks past a shorter series' end exit.
hipError_t launch_harmonic_sum(int pdt, const HarmArgs& a, int max_bins, hipStream_t st) {
  const int rows_per_block = 200;  // one block walks (up to) all acceleration trials of its columns
  const int ychunks = (a.Z + rows_per_block - 1) / rows_per_block;
  const dim3 g((max_bins + kHarmThreads - 1) / kHarmThreads, ychunks, a.n_series);
  switch (pdt) {
    case FDAS_F32: return hs_h<FDAS_F32>(a, g, st);
    case FDAS_BF16: return hs_h<FDAS_BF16>(a, g, st);
    case FDAS_F16: return hs_h<FDAS_F16>(a, g, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fdas
