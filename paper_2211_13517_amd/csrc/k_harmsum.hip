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


// ln P(Gamma(h, 1) > s) = -s + ln sum_{k<h} s^k / k!, integer h.  Not
// inlined: the harmonic sum calls it only for passing cells, and inline its
// FP64 logarithm would raise the kernel's register count (and lower the
// blocks per CU) for every cell.
__device__ __noinline__ double log_tail_gamma(double s, int h) {
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
// reads bin k R0 / H + floor((2ki + H)/(2H)).
//
// Bound first, exact sums where the bound passes.  The plane buffer carries
// the column maxima M[j][c] = max_{q < 8} P[j][8c + q] after its data.  The
// block copies into LDS, for the lower half of the harmonics (k <= H/2), the
// strip of plane values it reads, and for the upper half (k > H/2, whose
// strips are the largest: together they hold 5/6 of the tile's reads at
// H = 16) the strip of column maxima covering theirs, 8 times smaller.  With
// each upper-half value replaced by the maximum of its run of 8 columns, the
// stage sums S'_H' are upper bounds of the exact S_H': the terms only grow
// and every operation of the sum (FP32 additions, and products by 1 in the
// two-term dot products of 16-bit planes) is monotone in each operand.  So
// a cell whose bounds all stay below their thresholds passes no stage, and
// only the few cells with a bound at or above one (about 3e-5 of them on
// pure noise at H = 16) load their upper-half values from the plane and sum
// exactly, in the same order as everywhere, and are tested and reported
// from those exact sums.  Every strip is copied with aligned 16-byte loads
// and read back with LDS offsets that are immediates.
constexpr int kBand = 16;
constexpr int kMaxCols = kPlaneMaxCols;

template <int H, int CW, int CH>
struct HarmTile {
  static constexpr int KX = H / 2;  // k <= KX: plane values; k > KX: column maxima
  static constexpr int rows(int k) { return (2 * k * (kBand - 1) + H) / (2 * H) + 1; }
  // bins of harmonic k read by the tile: 0 .. floor((2k(CW-1) + H)/(2H)),
  // from bin k R0 / H, a multiple of kMaxCols and of CH
  static constexpr int span(int k) { return (2 * k * (CW - 1) + H) / (2 * H) + 1; }
  // column maxima covering the span
  static constexpr int mspan(int k) { return (span(k) - 1) / kMaxCols + 1; }
  // 16-byte chunks per strip row; a maxima strip starts at the aligned
  // element at or below its first maximum, up to CH - 1 elements early
  static constexpr int chunks(int k) {
    return k <= KX ? (span(k) + CH - 1) / CH : (mspan(k) + 2 * CH - 2) / CH;
  }
  static constexpr int pitch(int k) { return chunks(k) * CH; }  // elements per strip row
  static constexpr int off(int k) { return k <= 1 ? 0 : off(k - 1) + rows(k - 1) * pitch(k - 1); }
  static constexpr int SIZE = off(H + 1);  // elements of LDS
  // strip row of harmonic k for trial t of a band below (neg) or above z = 0
  static constexpr int rel(int k, int t, bool neg) {
    return neg ? (2 * k * t - H <= 0 ? 0 : (2 * k * t - H + 2 * H - 1) / (2 * H)) : (2 * k * t + H) / (2 * H);
  }
};

template <int PDT>
struct HarmCfg {
  static constexpr int CW = 256;  // cells per tile = threads per block
  // wavefronts per SIMD asked of the register allocation (64 VGPRs for
  // eight): eight blocks of a 16-bit plane fit in LDS (15.7 KB each at
  // H = 16), five of an FP32 plane.  7 blocks per CU (72 VGPRs) ran 3 %
  // slower, 5 (87 VGPRs, with the Gamma tail inlined) 10 % slower.
  static constexpr int WAVES = Store<PDT>::RBYTES == 2 ? 8 : 5;
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

// f / D for 0 <= f < 2^11 and D <= 64, exactly, by a full-rate 24-bit
// multiply: with M = ceil(2^20 / D), f M / 2^20 exceeds f / D by less than
// f (D - 1) / (2^20 D) < 1 / D, which cannot reach the next integer.
template <int D>
__device__ __forceinline__ int div_small(int f) {
  constexpr unsigned M = ((1u << 20) + D - 1) / D;
  return (int)(__umul24((unsigned)f, M) >> 20);
}

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

// 16-bit planes: the H values of a cell held as the H/2 pairs that the
// stage sums add by two-term dot products (pair 0 = (H/2, H); at stage
// st >= 2 the pairs (ka, ka + 2 step), ka = step (4i + 1), step = H / 2^st),
// each pair in one register.  Over the 16 trials of a band, a value is read
// from LDS only when its strip row changes, straight into its half of the
// pair's register.
template <int H>
struct PairSlot {
  static constexpr int step(int k) { return k & -k; }
  static constexpr int stage(int k) { return ilog2(H) - ilog2(step(k)); }
  static constexpr int index(int k) {
    return k == H || k == H / 2 ? 0 : (1 << (stage(k) - 2)) + (k / step(k) - 1) / 4;
  }
  static constexpr int half(int k) { return k == H ? 1 : k == H / 2 ? 0 : ((k / step(k) - 1) / 2) & 1; }
};

template <int PDT, int H, bool NEG, typename HT>
__device__ __forceinline__ void band_pairs(const char* lds, const int* boff, const float* thr, uint32_t thr0_bits,
                                           int t_lo, int t_hi, unsigned long long* bal) {
  typedef unsigned short us2 __attribute__((ext_vector_type(2)));
  constexpr int NST = ilog2(H) + 1;
  us2 P[H / 2];
  const uint32_t thr0_hi = thr0_bits << 16;
  auto dot = [](us2 w, float acc) {
    if constexpr (PDT == FDAS_BF16) {
      typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
      return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf2, w), __builtin_bit_cast(bf2, 0x3f803f80u), acc,
                                             false);
    } else {
      typedef _Float16 h2 __attribute__((ext_vector_type(2)));
      return __builtin_amdgcn_fdot2(__builtin_bit_cast(h2, w), __builtin_bit_cast(h2, 0x3c003c00u), acc, false);
    }
  };
  static_for<0, kBand>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    static_for<1, H + 1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr int row = HT::rel(k, t, NEG);
      if constexpr (t == 0 || row != HT::rel(k, t - 1, NEG)) {
        const uint16_t v = *reinterpret_cast<const uint16_t*>(lds + boff[k - 1] + row * HT::pitch(k) * 2);
        if constexpr (PairSlot<H>::half(k) == 0)
          P[PairSlot<H>::index(k)].x = v;
        else
          P[PairSlot<H>::index(k)].y = v;
      }
    });
    {
      // stage 0 on the raw bits of harmonic H, the high half of pair 0
      unsigned long long m = __builtin_amdgcn_ballot_w64(__builtin_bit_cast(uint32_t, P[0]) >= thr0_hi);
      float s = dot(P[0], 0.f);
      m |= __builtin_amdgcn_ballot_w64(s >= thr[1]);
      static_for<2, NST>([&](auto sc) {
        constexpr int st = decltype(sc)::value;
        static_for<0, (1 << st) / 4>([&](auto ic) { s = dot(P[(1 << (st - 2)) + decltype(ic)::value], s); });
        m |= __builtin_amdgcn_ballot_w64(s >= thr[st]);
      });
      // trials outside the band's valid range: computed, then dropped
      bal[t] = (t >= t_lo && t < t_hi) ? m : 0ull;
    }
  });
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
__global__ __launch_bounds__(HarmCfg<PDT>::CW) __attribute__((amdgpu_waves_per_eu(HarmCfg<PDT>::WAVES)))
void k_harmsum(HarmArgs a) {
  using PS = Store<PDT>;
  using RT = typename PS::real_t;
  constexpr int NST = ilog2(H) + 1;
  constexpr int ES = (int)sizeof(RT);
  constexpr int CH = 16 / ES;
  constexpr int CW = HarmCfg<PDT>::CW, G = HarmCfg<PDT>::GROUP;
  using HT = HarmTile<H, CW, CH>;
  static_assert(HT::SIZE * ES <= 32768, "strips of one tile");
  __shared__ __align__(16) RT strip[HT::SIZE];

  const SeriesDesc d = a.desc[blockIdx.z];
  const int nb = d.nbins << a.res_shift;  // plane columns of the series
  const int nm = nb / kMaxCols;           // column maxima per row
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
  const RT* maxima = reinterpret_cast<const RT*>(a.maxima) + d.plane_off / kMaxCols;

  // Copy the strips with direct global-to-LDS 16-byte loads: item f of
  // harmonic k (row f / NCH, chunk f % NCH) lands at byte off(k) * ES + 16 f,
  // so a wave's 64 items are contiguous in LDS from a wave-uniform base, and
  // every load of the block is in flight before the one wait at the barrier.
  // Rows outside the plane are never read by a valid trial, nor chunks past
  // the row's end by a searched cell.
  // The item arithmetic uses full-rate 24-bit multiplies; on an interior
  // tile (every trial valid, the strips' last chunks well inside the rows)
  // every item is loaded without bounds tests.
  const int wave0 = __builtin_amdgcn_readfirstlane(tid & ~63);
  const bool interior = t_lo == 0 && t_hi == kBand && R0 + 2 * CW <= nb;
  // interior tiles (every strip row and column inside the plane) copy with
  // no bounds tests: a uniform branch between two instances of the copy
  auto copy = [&](auto intc) {
  constexpr bool INTERIOR = decltype(intc)::value;
  static_for<1, H + 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int NCH = HT::chunks(k), ITEMS = HT::rows(k) * NCH;
    static_assert(ITEMS < 2048 && NCH <= 64, "item index arithmetic");
    const int base = a.j0 + (kBand / H) * k * u;
    const int cs = k * (R0 / H);
    const bool ex = k <= HT::KX;
    const int c0 = ex ? cs : (cs / kMaxCols) & ~(CH - 1);  // first element of the strip's rows
    const int len = ex ? nb : nm;                           // elements per source row
    // wave-uniform 64-bit base (row base_k, element c0) plus a 32-bit byte
    // offset per lane, the form the load's scalar-base addressing takes
    const char* src = reinterpret_cast<const char*>((ex ? plane : maxima) + ((int64_t)base * len + c0));
#pragma unroll
    for (int f0 = 0; f0 < ITEMS; f0 += CW) {
      if (f0 + wave0 >= ITEMS) continue;  // wave-uniform
      const int f = f0 + tid;
      const int r = div_small<NCH>(f), c = f - (int)__umul24(r, NCH);
      bool ok = f < ITEMS;
      if constexpr (!INTERIOR) ok = ok && (unsigned)(base + r) < (unsigned)a.Z && c0 + c * CH < len;
      if (ok) {
        uint32_t e = __umul24(r, len) + c * CH;  // element offset (< 2^27)
        asm volatile("" : "+v"(e));              // (keeps the 24-bit multiply)
        load_lds16(src + e * ES, reinterpret_cast<char*>(strip) + HT::off(k) * ES + (f0 + wave0) * 16);
      }
    }
  });
  };
  if (interior)
    copy(std::true_type{});
  else
    copy(std::false_type{});
  __syncthreads();

  const int R = R0 + tid;
  if (R >= nb - a.hmax) return;
  // byte offset of this cell's harmonic-k value (plane value or column
  // maximum) in row 0 of strip k; kept opaque so that the compiler holds it
  // in a register and folds every row offset into the LDS instruction's
  // immediate
  const char* lds = reinterpret_cast<const char*>(strip);
  int boff[H];
  static_for<1, H + 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const int e = (2 * k * tid + H) / (2 * H);
    int b;
    if constexpr (k <= HT::KX) {
      b = (HT::off(k) + e) * ES;
    } else {
      const int ms = k * (R0 / H) / kMaxCols;
      b = (HT::off(k) + (ms & (CH - 1)) + e / kMaxCols) * ES;
    }
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
  // wave-wide masks per trial (scalar registers) of the cells whose bound
  // passes a stage
  unsigned long long bal[kBand];
  auto none = [](auto) { return 0u; };
  auto band = [&](auto negc) {
    constexpr bool NEG = decltype(negc)::value;
    auto offs = [](auto tc) {
      return [](auto kc) {
        constexpr int k = decltype(kc)::value, t = decltype(tc)::value;
        return HT::rel(k, t, NEG) * HT::pitch(k) * ES;
      };
    };
    if constexpr (Store<PDT>::RBYTES == 2 && H > 1) {
      band_pairs<PDT, H, NEG, HT>(lds, boff, thr, thr0_bits, t_lo, t_hi, bal);
      return;
    }
    // software pipeline: the LDS reads of trial t + 1 are issued before the
    // sums of trial t (every trial's reads stay inside the strips)
    HarmVals<H> cur = load_vals<PDT, H, H>(lds, boff, offs(std::integral_constant<int, 0>{}), none);
    static_for<0, kBand>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      HarmVals<H> nxt;
      if constexpr (t + 1 < kBand) nxt = load_vals<PDT, H, H>(lds, boff, offs(std::integral_constant<int, t + 1>{}), none);
      bal[t] = 0;
      if (t >= t_lo && t < t_hi) bal[t] = pass_mask<PDT, H>(cur, thr, thr0_bits);
      if constexpr (t + 1 < kBand) cur = nxt;
    });
  };
  if (u < 0)
    band(std::true_type{});
  else
    band(std::false_type{});

  // rare: cells whose bound passes sum exactly (upper-half values from the
  // plane) and report their most significant passing stage
  unsigned long long any = 0;
#pragma unroll
  for (int t = 0; t < kBand; ++t) any |= bal[t];
  if (!any) return;
  const int lane = threadIdx.x & 63;
  uint32_t mask = 0;
#pragma unroll
  for (int t = 0; t < kBand; ++t) mask |= (uint32_t)((bal[t] >> lane) & 1ull) << t;
  const bool neg = u < 0;
  // the lane's bin offsets of the upper harmonics are recomputed here from an
  // opaque copy of tid, not kept alive from the set-up over the band
  int tid_x = tid;
  asm volatile("" : "+v"(tid_x));
  auto raw = [](const RT* p) -> uint32_t {
    if constexpr (ES == 4)
      return *reinterpret_cast<const uint32_t*>(p);
    else
      return *reinterpret_cast<const uint16_t*>(p);
  };
  while (mask) {
    const int t = __builtin_ctz(mask);
    mask &= mask - 1;
    const int j = jt0 + t;
    float S[NST];
    const HarmVals<H> x = load_vals<PDT, H, HT::KX>(
        lds, boff,
        [&](auto kc) {
          constexpr int k = decltype(kc)::value;
          return HT::rel(k, t, neg) * HT::pitch(k) * ES;
        },
        [&](auto kc) {
          constexpr int k = decltype(kc)::value;
          // a valid trial's row and a searched cell's bin are inside the
          // plane: the strip's first row and bin (uniform) plus a 32-bit
          // byte offset (fewer than 16 rows of at most 2^23 columns)
          const RT* base = plane + ((int64_t)(a.j0 + (kBand / H) * k * u) * nb + k * (R0 / H));
          const uint32_t off = (uint32_t)(HT::rel(k, t, neg) * nb + (2 * k * tid_x + H) / (2 * H)) * (uint32_t)ES;
          return raw(reinterpret_cast<const RT*>(reinterpret_cast<const char*>(base) + off));
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
    if (bi < 0) continue;  // the bound passed, the exact sums do not
    const unsigned long long slot = atomicAdd(a.count, 1ull);
    if ((int64_t)slot < a.capacity) {
      const int hh = 1 << bi;
      fdas_candidate c;
      c.series = (int)blockIdx.z + a.series_base;
      c.harm = hh;
      c.R = R;
      c.j = j;
      // division by the power of two hh 2^res_shift, exactly
      c.r = ldexpf((float)R, -(bi + a.res_shift));
      c.z = (float)ldexp(a.z_min + a.z_step * j, -bi);
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

// Column maxima of a packed plane: M[j][c] is the largest of P[j][8c + q],
// q < 8, a NaN or negative value counting as +inf (see capped_bits).
// Maximum i of a series is row i / nm, column i % nm, and its run is the 8
// consecutive plane elements from 8 i.
template <int PDT>
__global__ __launch_bounds__(256) void k_plane_maxima(const void* __restrict__ plane, void* __restrict__ maxima,
                                                      const SeriesDesc* __restrict__ desc, int Z, int res_shift) {
  using RT = typename Store<PDT>::real_t;
  constexpr int V = 16 / (int)sizeof(RT);  // elements per 16-byte load
  const SeriesDesc d = desc[blockIdx.y];
  const int64_t n = (int64_t)Z * ((int64_t)(d.nbins << res_shift) / kMaxCols);
  const RT* p = reinterpret_cast<const RT*>(plane) + d.plane_off;
  RT* m = reinterpret_cast<RT*>(maxima) + d.plane_off / kMaxCols;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    uint32_t v = 0;
#pragma unroll
    for (int h = 0; h < kMaxCols / V; ++h) {
      const uint4 w = *reinterpret_cast<const uint4*>(p + kMaxCols * i + V * h);
      const RT* e = reinterpret_cast<const RT*>(&w);
#pragma unroll
      for (int q = 0; q < V; ++q) v = max(v, capped_bits<PDT>(e[q]));
    }
    m[i] = from_bits<PDT>(v);
  }
}

hipError_t launch_plane_maxima(int pdt, const void* plane, void* maxima, const SeriesDesc* desc, int n_series, int Z,
                               int res_shift, int64_t max_bins, int cus, hipStream_t st) {
  const int64_t per_series = (int64_t)Z * ((max_bins << res_shift) / kMaxCols);
  const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((per_series + 255) / 256, (int64_t)cus * 16)),
               (unsigned)n_series);
  switch (pdt) {
    case FDAS_F32: hipLaunchKernelGGL(k_plane_maxima<FDAS_F32>, g, dim3(256), 0, st, plane, maxima, desc, Z, res_shift); break;
    case FDAS_BF16: hipLaunchKernelGGL(k_plane_maxima<FDAS_BF16>, g, dim3(256), 0, st, plane, maxima, desc, Z, res_shift); break;
    case FDAS_F16: hipLaunchKernelGGL(k_plane_maxima<FDAS_F16>, g, dim3(256), 0, st, plane, maxima, desc, Z, res_shift); break;
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
