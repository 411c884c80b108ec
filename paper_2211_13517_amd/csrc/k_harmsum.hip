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
#include <algorithm>

#include "fft.hpp"
#include "launch.hpp"

namespace fdas {


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

// Tiling: a block owns CW consecutive cells R in [R0, R0 + CW) (R0 a multiple
// of CW) for JT consecutive acceleration trials.  For R0 + i, harmonic k reads
// bin r_k = k R0 / H + floor((2 k i + H) / (2 H)), so the tile needs, for each
// k, the strip of bins [k R0 / H, k R0 / H + CW k / H] of the rows j_k(j) of
// its trials, which form a contiguous range of at most floor(k (JT-1)/H) + 2
// rows (j_k is monotone in j).  The block copies every such strip into LDS in
// one burst of aligned 16-byte loads (raw storage type), synchronises once and
// evaluates its CW x JT cells from LDS.
constexpr int kCells = 256;

template <int H, int CW, int JT, int CH>
struct HarmTile {
  static constexpr int rows(int k) { return (k * (JT - 1)) / H + 2; }             // max distinct rows of harmonic k
  static constexpr int chunks(int k) { return (CW * k / H + 1 + 2 * CH - 2) / CH; } // 16-byte chunks per strip row
  static constexpr int pitch(int k) { return chunks(k) * CH; }                      // elements per strip row
  static constexpr int off(int k) { return k <= 1 ? 0 : off(k - 1) + rows(k - 1) * pitch(k - 1); }
  static constexpr int SIZE = off(H + 1);                                            // elements of LDS
};

template <int PDT>
struct HarmCfg {
  static constexpr int JT = Store<PDT>::RBYTES == 2 ? 8 : 4;
  // Tile order: groups of GROUP bands (about 48 trials) are swept over all
  // column tiles, the bands of a group interleaved.  Bands that are close in
  // z share the rows of the low harmonics, and a sweep's working set then
  // stays in the L2/MALL (a cache model of this access pattern gives ~1.3
  // plane reads from HBM, against ~4 when every column tile walks all bands).
  static constexpr int GROUP = 48 / JT;
};

__device__ __forceinline__ int harm_row(int j0, int m, int k, int H) {
  const int am = m < 0 ? -m : m;
  const int mk = (2 * k * am + H) / (2 * H);
  return j0 + (m < 0 ? -mk : mk);
}

template <int PDT, int H>
__global__ __launch_bounds__(kCells) void k_harmsum(HarmArgs a) {
  using PS = Store<PDT>;
  using RT = typename PS::real_t;
  constexpr int NST = ilog2(H) + 1;
  constexpr int CH = 16 / (int)sizeof(RT);
  constexpr int CW = kCells, JT = HarmCfg<PDT>::JT;
  using HT = HarmTile<H, CW, JT, CH>;
  __shared__ __align__(16) RT strip[HT::SIZE];

  const SeriesDesc d = a.desc[blockIdx.z];
  const int nb = d.nbins;
  constexpr int G = HarmCfg<PDT>::GROUP;
  const int nbx = (a.max_bins + CW - 1) / CW;  // column tiles of the longest series
  const int grp = blockIdx.x / (nbx * G), inner = blockIdx.x % (nbx * G);
  const int R0 = (inner / G) * CW;
  const int jt0 = (grp * G + inner % G) * JT;
  if (R0 >= nb - a.hmax || jt0 >= a.Z) return;  // whole tile outside the searched band
  const int jt1 = min(jt0 + JT, a.Z);
  const int tid = threadIdx.x;
  const RT* plane = reinterpret_cast<const RT*>(a.plane) + d.plane_off;

  // copy the strips
  static_for<1, H + 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int NCH = HT::chunks(k), ITEMS = HT::rows(k) * NCH;
    const int rlo = harm_row(a.j0, jt0 - a.j0, k, H);
    const int rhi = harm_row(a.j0, jt1 - 1 - a.j0, k, H);
    const int nitems = (rhi - rlo + 1) * NCH;
    const int cs = (k * (R0 / H)) & ~(CH - 1);
#pragma unroll
    for (int f0 = 0; f0 < ITEMS; f0 += CW) {
      const int f = f0 + tid;
      if (f < nitems) {
        const int r = f / NCH, c = f - r * NCH;
        const int e0 = cs + c * CH;
        if (e0 < nb) {
          const uint4 v = *reinterpret_cast<const uint4*>(plane + (size_t)(rlo + r) * nb + e0);
          *reinterpret_cast<uint4*>(strip + HT::off(k) + r * HT::pitch(k) + c * CH) = v;
        }
      }
    }
  });
  __syncthreads();

  const int R = R0 + tid;
  if (R >= nb - a.hmax) return;
  int roff[H];
  static_for<1, H + 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    roff[k - 1] = HT::off(k) + ((k * (R0 / H)) & (CH - 1)) + (2 * k * tid + H) / (2 * H);
  });
  for (int j = jt0; j < jt1; ++j) {
    const int m = j - a.j0;
    float tk[H];
    static_for<1, H + 1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const int rel = harm_row(a.j0, m, k, H) - harm_row(a.j0, jt0 - a.j0, k, H);
      tk[k - 1] = PS::unpack_real(strip[roff[k - 1] + rel * HT::pitch(k)]);
    });
    float S[NST];
    bool any = false;
#pragma unroll
    for (int st = 0; st < NST; ++st) {
      const int step = H >> st;  // stage H' = 2^st uses k = step, 2 step, ..., H
      float sum = 0.f;
#pragma unroll
      for (int k = step; k <= H; k += step) sum += tk[k - 1];
      S[st] = sum;
      any |= (R >= (1 << st) * a.r_lo) && (sum >= a.tau[st]);
    }
    if (!any) continue;
    double best = 0.0;
    int bi = -1;
    for (int st = 0; st < NST; ++st) {
      if (!((R >= (1 << st) * a.r_lo) && (S[st] >= a.tau[st]))) continue;
      const double lq = log_tail_gamma((double)S[st], 1 << st);
      if (bi < 0 || lq < best) {
        best = lq;
        bi = st;
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
      c.sigma = 0.f;  // filled in by k_cand_sigma
      a.cands[slot] = c;
    }
  }
}

// Gaussian-equivalent significance of every stored record (FP64).
__global__ __launch_bounds__(256) void k_cand_sigma(fdas_candidate* __restrict__ cands,
                                                    const unsigned long long* __restrict__ count, int64_t capacity) {
  const int64_t n = min((int64_t)*count, capacity);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    fdas_candidate c = cands[i];
    c.sigma = (float)sigma_from_log_tail(log_tail_gamma((double)c.power, c.harm));
    cands[i] = c;
  }
}

template <int PDT, int H>
static void hs_launch(const HarmArgs& a, dim3 g, hipStream_t st) {
  constexpr int JT = HarmCfg<PDT>::JT, G = HarmCfg<PDT>::GROUP;
  const int nby = (a.Z + JT - 1) / JT;
  const int ngroups = (nby + G - 1) / G;
  const int nbx = (a.max_bins + kCells - 1) / kCells;
  g.x = (unsigned)((int64_t)ngroups * G * nbx);
  hipLaunchKernelGGL((k_harmsum<PDT, H>), g, dim3(kCells), 0, st, a);
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
  HarmArgs b = a;
  b.max_bins = max_bins;
  const dim3 g(1, 1, a.n_series);
  hipError_t e;
  switch (pdt) {
    case FDAS_F32: e = hs_h<FDAS_F32>(b, g, st); break;
    case FDAS_BF16: e = hs_h<FDAS_BF16>(b, g, st); break;
    case FDAS_F16: e = hs_h<FDAS_F16>(b, g, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess || a.capacity == 0) return e;
  const int64_t blocks = std::min<int64_t>((a.capacity + 255) / 256, 1024);
  hipLaunchKernelGGL(k_cand_sigma, dim3((unsigned)blocks), dim3(256), 0, st, a.cands, a.count, a.capacity);
  return hipGetLastError();
}

}  // namespace fdas
