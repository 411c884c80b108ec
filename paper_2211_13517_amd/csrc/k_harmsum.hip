// Nested incoherent harmonic sums over the power plane,
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
// the few passing cells).  On a half-bin plane (two columns per bin) the same
// rules run over columns: R, r_lo and h_max count half bins.
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

// Tiling.  A block owns CW consecutive cells R in [R0, R0 + CW) (R0 a
// multiple of CW) for the 16 trials of one band m in [16u, 16u + 16), bands
// aligned to z = 0.  Because m_k(m + H) = m_k(m) + k for m >= 0 (and the
// mirror image below zero), the harmonic-k row used by trial t of band u is
//   base_k + rel_k(t),  base_k = j0 + 16 k u / H,
// with rel_k(t) = floor((2kt + H)/(2H)) for u >= 0 and ceil((2kt - H)/(2H))
// for u < 0: a compile-time pattern.  Likewise harmonic k of cell R0 + i
// reads bin k R0 / H + floor((2ki + H)/(2H)).  The block copies, for every
// k below the top two, the rows base_k .. base_k + rows(k) - 1 of the bin
// strip it needs into LDS with aligned 16-byte loads, synchronises once, and
// then evaluates its CW x 16 cells with LDS reads whose offsets are all
// immediates.  The top two harmonics use (nearly) one value per cell, so
// each thread loads those straight into registers; that keeps a tile's LDS
// at 34 KB (four blocks per CU instead of three).
constexpr int kBand = 16;

template <int H, int CW, int CH, int ND>
struct HarmTile {
  static constexpr int KL = H - ND;  // harmonics staged in LDS (the top ND are read directly)
  static constexpr int rows(int k) { return (2 * k * (kBand - 1) + H) / (2 * H) + 1; }
  // bins of harmonic k read by the tile: 0 .. floor((2k(CW-1) + H)/(2H))
  static constexpr int span(int k) { return (2 * k * (CW - 1) + H) / (2 * H) + 1; }
  static constexpr int chunks(int k) { return (span(k) + CH - 1) / CH; }          // 16-byte chunks per strip row
  static constexpr int pitch(int k) { return chunks(k) * CH; }                     // elements per strip row
  static constexpr int off(int k) { return k <= 1 ? 0 : off(k - 1) + rows(k - 1) * pitch(k - 1); }
  static constexpr int SIZE = off(KL + 1);                                          // elements of LDS
  // strip row of harmonic k for trial t of a band below (neg) or above z = 0
  static constexpr int rel(int k, int t, bool neg) {
    return neg ? (2 * k * t - H <= 0 ? 0 : (2 * k * t - H + 2 * H - 1) / (2 * H)) : (2 * k * t + H) / (2 * H);
  }
};

template <int PDT>
struct HarmCfg {
  static constexpr int CW = Store<PDT>::RBYTES == 2 ? 256 : 128;  // cells per tile = threads per block
  // Tile order: groups of GROUP bands (48 trials) are swept over all column
  // tiles, the bands of a group interleaved.  Bands that are close in z
  // share the rows of the low harmonics, and a sweep's working set then
  // stays in the L2/MALL (a cache model of this access pattern gives ~1.3
  // plane reads from HBM, against ~4 when every column tile walks all bands).
  static constexpr int GROUP = 3;
};

// Blocks are dispatched round-robin over the 8 XCDs (block b to XCD b % 8).
// The launch order is remapped so that each XCD takes runs of kXcdRun
// consecutive tiles (neighbouring columns, whose strips share their edge
// cache lines in that XCD's L2) while all XCDs advance through one common
// front of the tile sequence.
constexpr int kXcds = 8, kXcdRun = 16;
__device__ __forceinline__ int xcd_tile(int b) {
  constexpr int W = kXcds * kXcdRun;
  const int r = b % W;
  return b - r + (r % kXcds) * kXcdRun + r / kXcds;
}

__device__ __forceinline__ int floordiv(int a, int b) { return (a >= 0 ? a : a - b + 1) / b; }

// Nested stage sums: stage 0 is harmonic H alone; stage st adds the odd
// multiples of H / 2^st, so the sum handed to sink(st, S) covers
// k = H/2^st, 2 H/2^st, ..., H.
//  * FP32 planes: plain FP32 additions in that order.
//  * 16-bit planes: the values are read in pairs into one register (stage 1
//    pairs H with H/2; later stages pair consecutive odd multiples) and each
//    pair is added to the running sum by one FP32-accumulating two-term dot
//    product with (1, 1), the products being exact.
// The H values of one cell, as read from LDS (16-bit planes: the raw bits,
// zero-extended; FP32 planes: the float bits).
template <int H>
struct HarmVals {
  uint32_t v[H];
};

template <int PDT, int H, int KL, typename OFF, typename DIR>
__device__ __forceinline__ HarmVals<H> load_vals(const char* lds, const int* boff, OFF off, DIR dir) {
  HarmVals<H> r;
  static_for<1, H + 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (k > KL) {
      r.v[k - 1] = dir(kc);
    } else {
      const char* p = lds + boff[k - 1] + off(kc);
      if constexpr (Store<PDT>::RBYTES == 4)
        r.v[k - 1] = *reinterpret_cast<const uint32_t*>(p);
      else
        r.v[k - 1] = *reinterpret_cast<const uint16_t*>(p);
    }
  });
  return r;
}

template <int PDT, int H, typename SINK>
__device__ __forceinline__ void stage_sums(const HarmVals<H>& x, SINK sink) {
  using PS = Store<PDT>;
  using RT = typename PS::real_t;
  constexpr int NST = ilog2(H) + 1;
  if constexpr (PS::RBYTES == 4) {
    float s = __uint_as_float(x.v[H - 1]);
    sink(0, s);
    static_for<1, NST>([&](auto sc) {
      constexpr int st = decltype(sc)::value;
      constexpr int step = H >> st;
      static_for<0, (1 << st) / 2>([&](auto ic) {
        constexpr int k = step * (2 * decltype(ic)::value + 1);
        s += __uint_as_float(x.v[k - 1]);
      });
      sink(st, s);
    });
  } else {
    auto pair = [&](int ka, int kb) { return x.v[ka - 1] | (x.v[kb - 1] << 16); };
    auto dot = [](uint32_t w, float acc) {
      if constexpr (PDT == FDAS_BF16) {
        typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf2, w), __builtin_bit_cast(bf2, 0x3f803f80u), acc,
                                               false);
      } else {
        typedef _Float16 h2 __attribute__((ext_vector_type(2)));
        return __builtin_amdgcn_fdot2(__builtin_bit_cast(h2, w), __builtin_bit_cast(h2, 0x3c003c00u), acc, false);
      }
    };
    if constexpr (H == 1) {
      sink(0, PS::unpack_real((RT)x.v[0]));
    } else {
      const uint32_t w1 = pair(H / 2, H);
      sink(0, PS::unpack_real((RT)(w1 >> 16)));
      float s = dot(w1, 0.f);
      sink(1, s);
      static_for<2, NST>([&](auto sc) {
        constexpr int st = decltype(sc)::value;
        constexpr int step = H >> st;
        static_for<0, (1 << st) / 4>([&](auto ic) {
          constexpr int ka = step * (4 * decltype(ic)::value + 1), kb = ka + 2 * step;
          s = dot(pair(ka, kb), s);
        });
        sink(st, s);
      });
    }
  }
}

// Wave-wide pass mask of one trial: the OR over stages of the ballots
// S_st >= thr[st], each ballot the compare's own lane mask.  On 16-bit planes
// stage 0 (harmonic H alone, a stored value) is tested on its raw bits: for
// non-negative values the bit patterns order like the values, so
// x >= thr[0]  <=>  bits(x) >= thr0_bits, the smallest pattern whose value is
// at least thr[0].  (A NaN pattern also passes this test; the exact stage
// tests of the reporting pass then reject it, as the float compare does.)
template <int PDT, int H>
__device__ __forceinline__ unsigned long long pass_mask(const HarmVals<H>& x, const float* thr, uint32_t thr0_bits) {
  unsigned long long m = 0;
  if constexpr (Store<PDT>::RBYTES == 2) {
    m = __builtin_amdgcn_ballot_w64(x.v[H - 1] >= thr0_bits);
    stage_sums<PDT, H>(x, [&](int st, float S) {
      if (st > 0) m |= __builtin_amdgcn_ballot_w64(S >= thr[st]);
    });
  } else {
    stage_sums<PDT, H>(x, [&](int st, float S) { m |= __builtin_amdgcn_ballot_w64(S >= thr[st]); });
  }
  return m;
}

// Smallest 16-bit pattern of the plane type whose value is >= v (v > 0, or +inf).
template <int PDT>
__device__ __forceinline__ uint32_t ceil_bits16(float v) {
  if constexpr (PDT == FDAS_BF16) {
    uint32_t b = __float_as_uint(v) >> 16;
    if (__uint_as_float(b << 16) < v) ++b;
    return b;
  } else if constexpr (PDT == FDAS_F16) {
    const _Float16 h = (_Float16)v;
    uint32_t b = __builtin_bit_cast(uint16_t, h);
    if ((float)h < v) ++b;
    return b;
  } else {
    return 0u;
  }
}

template <int PDT, int H>
__global__ __launch_bounds__(HarmCfg<PDT>::CW) void k_harmsum(HarmArgs a) {
  using PS = Store<PDT>;
  using RT = typename PS::real_t;
  constexpr int NST = ilog2(H) + 1;
  constexpr int CH = 16 / (int)sizeof(RT);
  constexpr int CW = HarmCfg<PDT>::CW, G = HarmCfg<PDT>::GROUP;
  // The top ND harmonics read (nearly) one value per cell: they bypass LDS
  // and are loaded by each thread straight into registers.
  constexpr int ND = H >= 4 ? 2 : 0;
  using HT = HarmTile<H, CW, CH, ND>;
  __shared__ __align__(16) RT strip[HT::SIZE];

  const SeriesDesc d = a.desc[blockIdx.z];
  const int nb = d.nbins << a.res_shift;  // plane columns of the series
  const int ncol = (a.max_bins + CW - 1) / CW;  // column tiles of the longest series
  const int tile = xcd_tile(blockIdx.x);
  const int grp = tile / (ncol * G), inner = tile % (ncol * G);
  const int R0 = (inner / G) * CW;
  const int u = floordiv(-a.j0, kBand) + grp * G + inner % G;
  const int jt0 = a.j0 + kBand * u;  // trial of t = 0
  if (R0 >= nb - a.hmax || jt0 >= a.Z) return;  // whole tile outside the searched region
  const int t_lo = max(0, -jt0), t_hi = min(kBand, a.Z - jt0);
  const int tid = threadIdx.x;
  const RT* plane = reinterpret_cast<const RT*>(a.plane) + d.plane_off;

  // Copy the strips with direct global-to-LDS 16-byte loads: item f of
  // harmonic k (row f / NCH, chunk f % NCH) lands at byte off(k) * sizeof(RT)
  // + 16 f, so a wave's 64 items are contiguous in LDS from a wave-uniform
  // base, and every load of the block is in flight before the one wait at
  // the barrier.  Rows outside the plane are never read by a valid trial.
  const int wave0 = __builtin_amdgcn_readfirstlane(tid & ~63);
  static_for<1, HT::KL + 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int NCH = HT::chunks(k), ITEMS = HT::rows(k) * NCH;
    const int base = a.j0 + (kBand / H) * k * u;
    const int cs = k * (R0 / H);
    // wave-uniform 64-bit base (row base_k, bin cs) plus a 32-bit byte offset
    // per lane, the form the load's scalar-base addressing takes
    const char* src = reinterpret_cast<const char*>(plane + ((int64_t)base * nb + cs));
#pragma unroll
    for (int f0 = 0; f0 < ITEMS; f0 += CW) {
      if (f0 + wave0 >= ITEMS) continue;  // wave-uniform
      const int f = f0 + tid;
      const int r = f / NCH, c = f - r * NCH;
      const int row = base + r, e0 = cs + c * CH;
      if (f < ITEMS && row >= 0 && row < a.Z && e0 < nb)
        load_lds16(src + (uint32_t)((r * nb + c * CH) * (int)sizeof(RT)),
                   reinterpret_cast<char*>(strip) + HT::off(k) * (int)sizeof(RT) + (f0 + wave0) * 16);
    }
  });
  // The directly read harmonics: this thread's bin of each of their rows
  // (rows outside the plane and bins past the series are clamped: their
  // values only reach cells that are not searched).
  auto raw = [](const RT* p) -> uint32_t {
    if constexpr (sizeof(RT) == 4)
      return *reinterpret_cast<const uint32_t*>(p);
    else
      return *reinterpret_cast<const uint16_t*>(p);
  };
  auto direct_ptr = [&](int k, int rel) {
    const int cs = k * (R0 / H);
    const int row = min(max(a.j0 + (kBand / H) * k * u + rel, 0), a.Z - 1);  // uniform
    const int pos = min((2 * k * tid + H) / (2 * H), nb - 1 - cs);
    return reinterpret_cast<const RT*>(reinterpret_cast<const char*>(plane + ((int64_t)row * nb + cs)) +
                                       (uint32_t)(pos * (int)sizeof(RT)));
  };
  uint32_t dv[ND > 0 ? ND : 1][kBand];
  auto dload = [&](auto negc) {
    constexpr bool NEG = decltype(negc)::value;
    static_for<0, ND>([&](auto dc) {
      constexpr int k = H - decltype(dc)::value;
      static_for<0, kBand>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        dv[decltype(dc)::value][t] = raw(direct_ptr(k, HT::rel(k, t, NEG)));
      });
    });
  };
  if (u < 0)
    dload(std::true_type{});
  else
    dload(std::false_type{});
  __syncthreads();

  const int R = R0 + tid;
  if (R >= nb - a.hmax) return;
  // byte offset of this cell's harmonic-k bin in row 0 of strip k; kept
  // opaque so that the compiler holds it in a register and folds every row
  // offset into the LDS instruction's immediate
  const char* lds = reinterpret_cast<const char*>(strip);
  int boff[H];
  static_for<1, HT::KL + 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    int b = (HT::off(k) + (2 * k * tid + H) / (2 * H)) * (int)sizeof(RT);
    asm volatile("" : "+v"(b));
    boff[k - 1] = b;
  });
  // per-cell thresholds: a stage whose fundamental R / 2^st lies below r_lo
  // is not searched (threshold +inf)
  bool en[NST];
  float thr[NST];
#pragma unroll
  for (int st = 0; st < NST; ++st) {
    en[st] = R >= (1 << st) * a.r_lo;
    thr[st] = en[st] ? a.tau[st] : __builtin_inff();
  }
  const uint32_t thr0_bits = ceil_bits16<PDT>(thr[0]);
  // wave-wide pass masks per trial (scalar registers)
  unsigned long long bal[kBand];
  auto band = [&](auto negc) {
    constexpr bool NEG = decltype(negc)::value;
    auto offs = [](auto tc) {
      return [](auto kc) {
        constexpr int k = decltype(kc)::value, t = decltype(tc)::value;
        return HT::rel(k, t, NEG) * HT::pitch(k) * (int)sizeof(RT);
      };
    };
    // software pipeline: the LDS reads of trial t + 1 are issued before the
    // sums of trial t (every trial's reads stay inside the strips)
    auto dir = [&](auto tc) {
      return [&](auto kc) { return dv[H - decltype(kc)::value][decltype(tc)::value]; };
    };
    HarmVals<H> cur = load_vals<PDT, H, HT::KL>(lds, boff, offs(std::integral_constant<int, 0>{}),
                                               dir(std::integral_constant<int, 0>{}));
    static_for<0, kBand>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      HarmVals<H> nxt;
      if constexpr (t + 1 < kBand)
        nxt = load_vals<PDT, H, HT::KL>(lds, boff, offs(std::integral_constant<int, t + 1>{}),
                                        dir(std::integral_constant<int, t + 1>{}));
      bal[t] = 0;
      if (t >= t_lo && t < t_hi) bal[t] = pass_mask<PDT, H>(cur, thr, thr0_bits);
      if constexpr (t + 1 < kBand) cur = nxt;
    });
  };
  if (u < 0)
    band(std::true_type{});
  else
    band(std::false_type{});

  // rare: cells with a passing stage report their most significant one
  unsigned long long any = 0;
#pragma unroll
  for (int t = 0; t < kBand; ++t) any |= bal[t];
  if (!any) return;
  const int lane = threadIdx.x & 63;
  uint32_t mask = 0;
#pragma unroll
  for (int t = 0; t < kBand; ++t) mask |= (uint32_t)((bal[t] >> lane) & 1ull) << t;
  const bool neg = u < 0;
  while (mask) {
    const int t = __builtin_ctz(mask);
    mask &= mask - 1;
    const int j = jt0 + t;
    float S[NST];
    const HarmVals<H> x = load_vals<PDT, H, HT::KL>(
        lds, boff,
        [&](auto kc) {
          constexpr int k = decltype(kc)::value;
          return HT::rel(k, t, neg) * HT::pitch(k) * (int)sizeof(RT);
        },
        [&](auto kc) {
          constexpr int k = decltype(kc)::value;
          return raw(direct_ptr(k, HT::rel(k, t, neg)));
        });
    stage_sums<PDT, H>(x, [&](int st, float v) { S[st] = v; });
    double best = 0.0;
    int bi = -1;
    for (int st = 0; st < NST; ++st) {
      if (!(en[st] && S[st] >= thr[st])) continue;
      const double lq = log_tail_gamma((double)S[st], 1 << st);
      if (bi < 0 || lq < best) {
        best = lq;
        bi = st;
      }
    }
    if (bi < 0) continue;  // only an infinite sum at an unsearched stage gets here
    const unsigned long long slot = atomicAdd(a.count, 1ull);
    if ((int64_t)slot < a.capacity) {
      const int hh = 1 << bi;
      fdas_candidate c;
      c.series = (int)blockIdx.z + a.series_base;
      c.harm = hh;
      c.R = R;
      c.j = j;
      c.r = (float)((double)R / (hh << a.res_shift));
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
  constexpr int CW = HarmCfg<PDT>::CW, G = HarmCfg<PDT>::GROUP;
  const int fd = [](int x, int y) { return (x >= 0 ? x : x - y + 1) / y; }(-a.j0, kBand);
  const int nbands = [](int x, int y) { return (x >= 0 ? x : x - y + 1) / y; }(a.Z - 1 - a.j0, kBand) - fd + 1;
  const int ngroups = (nbands + G - 1) / G;
  const int ncol = (a.max_bins + CW - 1) / CW;
  constexpr int W = kXcds * kXcdRun;
  g.x = (unsigned)(((int64_t)ngroups * G * ncol + W - 1) / W * W);  // tiles past the last group exit
  hipLaunchKernelGGL((k_harmsum<PDT, H>), g, dim3(CW), 0, st, a);
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
hipError_t launch_harmonic_sum(int pdt, const HarmArgs& a, hipStream_t st) {
  const HarmArgs& b = a;
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
