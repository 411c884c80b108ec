// Overlap-save correlation with every template and the power plane,
// fused in one kernel so that the complex products never leave the chip.
//
// Work unit ("tile"): one segment of one series and one group of templates.
// Segment s of a series covers spectrum bins [s U - h', s U - h' + L) (zero
// outside [0, N/2)), h' = h_max rounded up to a multiple of 8.  The tile
// loads it once, runs the forward FFT and keeps the result F in registers;
// then, for each template j of its group, multiplies F by the template
// spectrum T_j (read from L2, it is shared by every tile), runs the inverse
// FFT and stores |y|^2 of U outputs free of wrap-around (U the largest
// multiple of 8 <= L - 2 h'), at plane[j][s U + i], and the maximum of each
// aligned run of 8 of them in the column-maxima section of the plane buffer.
//
// Half-bin plane: h' and U are multiples of 4 and U <= L - 2 h' - 1, so
// output i + 1 is free of wrap-around too, and each output stores the pair
// (|y_i|^2, |y_i - y_{i+1}|^2 / 2) at columns 2(s U + i) and 2(s U + i) + 1
// of a row twice as long; a column maximum covers 4 outputs.  Output i sits
// in thread i mod NT, register i / NT; its successor is the next lane's
// register (a cross-lane shuffle), for the last lane of a wavefront the first
// lane of the next wavefront (through LDS in block tiles), and for the last
// thread of the tile the first thread's next register.
//
// Every FFT holds 16 points per thread.  L = 1024: one wavefront owns a tile
// and exchanges through its private LDS buffer, so the four wavefronts of a
// block never wait for each other; with a 16-bit plane its inverse FFTs run
// in FP16 on the matrix cores (fft_mfma.hpp).  L = 2048, 4096, 8192: a block of L/16
// threads (2, 4 or 8 wavefronts) owns a tile and synchronises.
// Tiles are dealt round-robin to wavefronts (resp. blocks) of a grid sized to
// the machine, so every unit runs the same number of tiles to within one.
#include "fft.hpp"
#include "fft_mfma.hpp"
#include "launch.hpp"

namespace fdas {

__device__ __forceinline__ int find_series(const SeriesDesc* __restrict__ desc, int n, int64_t tile) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].tile_begin <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// y at output i + 1 for each of this thread's outputs i = tid + NT c (zero
// past the tile's last point, which no valid output needs).
template <class FS, bool BLOCK>
__device__ __forceinline__ void next_outputs(const c32 (&v)[FS::P], c32 (&nx)[FS::P], c32* edge, int tid) {
  constexpr int P = FS::P, NW = FS::NT / 64;
  const int lane = tid & 63, wave = tid >> 6;
  const int src = (lane + 1) & 63;
  c32 w[P];
  static_for<0, P>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    w[c] = {__shfl(v[c].re, src, 64), __shfl(v[c].im, src, 64)};
  });
  if constexpr (!BLOCK) {
    // lane 63's successor is lane 0 at the next register: w[c + 1] of lane 63
    static_for<0, P>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      c32 last = {0.f, 0.f};
      if constexpr (c + 1 < P) last = w[c + 1];
      nx[c] = lane == 63 ? last : w[c];
    });
  } else {
    if (lane == 0) {
      static_for<0, P>([&](auto cc) { edge[wave * P + decltype(cc)::value] = v[decltype(cc)::value]; });
    }
    __syncthreads();
    static_for<0, P>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      c32 last = {0.f, 0.f};
      if (lane == 63) {
        if (wave + 1 < NW) last = edge[(wave + 1) * P + c];
        else if constexpr (c + 1 < P) last = edge[c + 1];
      }
      nx[c] = lane == 63 ? last : w[c];
    });
    // the next write to `edge` follows the barriers of the next inverse FFT
  }
}

// Column maxima (on capped bit patterns, see capped_bits) of aligned groups
// of G lanes (4 or 8), over every register at once so that the DPP steps of
// different registers interleave: lane swaps within quads give every lane of
// a quad its quad's maximum; for G = 8 a shift by 4 lanes within each row of
// 16 then gives lanes 4..7 of each group the group's maximum (lanes 0..3 of
// a row read 0 and keep theirs).  The group's lane G/2 holds it.
template <int G, int P>
__device__ __forceinline__ void group_max(uint32_t (&v)[P]) {
  auto step = [&](auto ctrl) {
    static_for<0, P>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      // a lane with no source lane reads 0, which leaves its maximum as it is
      v[c] = max(v[c], (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v[c], decltype(ctrl)::value, 0xF, 0xF, true));
    });
  };
  step(std::integral_constant<int, 0xB1>{});  // quad_perm [1, 0, 3, 2]
  step(std::integral_constant<int, 0x4E>{});  // quad_perm [2, 3, 0, 1]
  if constexpr (G == 8) step(std::integral_constant<int, 0x114>{});  // row_shr:4
  // every lane computes the last step (one DPP max) rather than only the
  // storing lane (a DPP move, then a max in its branch)
#pragma unroll
  for (int c = 0; c < P; ++c) asm volatile("" : "+v"(v[c]));
}

// A bin's power and the half-bin power after it, as one store.
template <int PDT> struct PowerPair;
template <> struct PowerPair<FDAS_F32> {
  typedef float2 type;
  __device__ __forceinline__ static type pack(float p, float h) { return make_float2(p, h); }
};
template <> struct PowerPair<FDAS_BF16> {
  typedef uint32_t type;
  __device__ __forceinline__ static type pack(float p, float h) { return Store<FDAS_BF16>::pack(c32{p, h}); }
};
template <> struct PowerPair<FDAS_F16> {
  typedef uint32_t type;
  __device__ __forceinline__ static type pack(float p, float h) { return Store<FDAS_F16>::pack(c32{p, h}); }
};

// The 1024-point inverse FFTs of a 16-bit plane (one wavefront per tile,
// radix 16, bins or half bins) run their two DFT-16 stages in FP16 on the
// matrix cores (fft_mfma.hpp).  The operands are scaled per tile by a power
// of two: with |F| <= f and |T_j| <= tbound, every product is at most 2^10
// and every stage-1 result at most 2^14 in magnitude, inside FP16's range,
// and the power is scaled back exactly.
template <int L, int R, int PDT, bool IB>
constexpr bool use_mfma() {
  return L == 1024 && R == 16 && Store<PDT>::RBYTES == 2;
}

struct MfCtx {
  const uint32_t* tw2;
  const c32* tw3;
  mf::Weights W;
};

template <class FS, int SDT, int PDT, bool BLOCK, bool IB, bool MF = false>
__device__ __forceinline__ void conv_tile(const ConvArgs& a, int64_t tile, c32* xb, const c32* tw, int tid,
                                          c32* edge, const MfCtx* mc = nullptr) {
  using SS = Store<SDT>;
  using PS = Store<PDT>;
  using CT = typename SS::cplx_t;
  using RT = typename PS::real_t;
  constexpr int P = FS::P, NT = FS::NT, L = FS::L;
  const int s = find_series(a.desc, a.n_series, tile);
  const SeriesDesc d = a.desc[s];
  const int64_t local = tile - d.tile_begin;
  const int seg = (int)(local / a.G), grp = (int)(local % a.G);
  const int t0 = (int)(((int64_t)grp * a.Z) / a.G), t1 = (int)(((int64_t)(grp + 1) * a.Z) / a.G);
  const int r0 = seg * a.U - a.seg_margin;  // bin of FFT index 0 (segment start, may be negative)
  const CT* sp = reinterpret_cast<const CT*>(a.spec) + d.spec_off;

  // Segment load: indices outside [0, nbins) read a clamped address and are zeroed.
  c32 F[P];
  static_for<0, P>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    const int idx = r0 + tid + NT * c;
    const int ci = min(max(idx, 0), d.nbins - 1);
    const c32 val = SS::unpack(sp[ci]);
    const bool in = (idx >= 0) && (idx < d.nbins);
    F[c] = {in ? val.re : 0.f, in ? val.im : 0.f};
  });
  fft_run<FS, -1, BLOCK>(F, xb, tw, tid);
  float pscale = 1.f;  // FP16 path: factor that undoes the tile's scaling on the power
  uint32_t Fh[MF ? P : 1];  // FP16 path: the scaled segment spectrum as FP16 pairs
  if constexpr (MF) {
    float fm = 0.f;
    static_for<0, P>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      fm = fmaxf(fm, fmaxf(fabsf(F[c].re), fabsf(F[c].im)));
    });
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) fm = fmaxf(fm, __shfl_xor(fm, o, 64));
    // the FP16 templates are T_j 2^10: every product |F T_j 2^10| < 2^e
    int e;
    frexpf(fm * 1.41421356f * ldexpf(a.tbound, kTspec16Shift), &e);
    e = min(max(e, -60), 60);
    const float sc = ldexpf(1.f, 10 - e);
    static_for<0, P>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      Fh[c] = mf::pack_h2(F[c].re * sc, F[c].im * sc);
    });
    pscale = ldexpf(1.f, 2 * (e - 10 - kTspec16Shift));
  }

  const CT* T = reinterpret_cast<const CT*>(a.tspec);
  RT* out = reinterpret_cast<RT*>(a.plane) + d.plane_off;
  RT* mx = reinterpret_cast<RT*>(a.maxima) + d.plane_off / kPlaneMaxCols;
  // Output index i maps to bin r0 + i; valid for i in [lo, hi).  r0, lo and
  // hi are multiples of the bins per column maximum (G8 = 8, or 4 on a
  // half-bin plane), so the G8 outputs of an aligned group of lanes are all
  // valid or all not, and make one maximum.
  const int lo = a.seg_margin, hi = min(a.seg_margin + a.U, d.nbins - r0);
  constexpr int G8 = IB ? kPlaneMaxCols / 2 : kPlaneMaxCols;
  const int grp0 = tid & ~(G8 - 1);           // first lane of this lane's group
  const bool lead = (tid & (G8 - 1)) == G8 / 2;  // the lane that stores the group's maximum
  // template spectra: the stored bank, or its FP16 copy (times 2^10) on the FP16 path
  using TT = std::conditional_t<MF, uint32_t, CT>;
  const TT* TB = reinterpret_cast<const TT*>(MF ? a.tspec16 : a.tspec);
  const uint32_t toff = (uint32_t)tid * sizeof(TT);
  TT tc[P];
  static_for<0, P>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    tc[c] = ld_off<TT>(TB + (size_t)t0 * L, toff + c * NT * sizeof(TT));
  });
  for (int t = t0; t < t1; ++t) {
    // prefetch the next template while this one is transformed
    const TT* Tn = TB + (size_t)min(t + 1, t1 - 1) * L;
    TT tn[P];
    static_for<0, P>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      tn[c] = ld_off<TT>(Tn, toff + c * NT * sizeof(TT));
    });
    if constexpr (MF) {
      uint32_t h[P];
      static_for<0, P>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        h[c] = mf::cmul_h2(Fh[c], tc[c]);
      });
      // output y[e][kb] of lane (q, n) is FFT index n + 64 q + 16 e + 256 kb
      c32 y[4][4];
      mf::ifft1024(h, y, mc->tw2, mc->tw3, mc->W, tid);
      const int q = tid >> 4, n = tid & 15;
      RT* mdst = mx + (size_t)t * (uint32_t)(d.nbins / G8) + (r0 + (n & ~(G8 - 1)) + 64 * q) / G8;
      uint32_t m[16];
      if constexpr (IB) {
        // successor y[k + 1] of output k: the next lane of the row (DPP
        // row_shl:1); for the row's last lane, lane 0 of the row in the next
        // register (row_shr:15, the other lanes keeping theirs), or for the
        // last register (e = 3) lane 0 of the next row (a shuffle; lane 63
        // takes lane 0's register of the next kb)
        auto shl1 = [](float v) {
          return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x101, 0xF, 0xF, true));
        };
        auto from_row0 = [](float old, float v) {
          return __int_as_float(
              __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x11F, 0xF, 0xF, false));
        };
        c32 nx[4][4];
        static_for<0, 4>([&](auto kc) {
          constexpr int kb = decltype(kc)::value;
          static_for<0, 3>([&](auto ec) {
            constexpr int e = decltype(ec)::value;
            nx[e][kb] = {from_row0(shl1(y[e][kb].re), y[e + 1][kb].re), from_row0(shl1(y[e][kb].im), y[e + 1][kb].im)};
          });
          c32 o = y[0][kb];
          if constexpr (kb < 3) {
            if (tid == 0) o = y[0][kb + 1];
          } else {
            if (tid == 0) o = {0.f, 0.f};
          }
          const int src = (tid + 1) & 63;
          const c32 w = {__shfl(o.re, src, 64), __shfl(o.im, src, 64)};
          const c32 sl = {shl1(y[3][kb].re), shl1(y[3][kb].im)};
          nx[3][kb] = n == 15 ? w : sl;
        });
        using PP = PowerPair<PDT>;
        typename PP::type* dst =
            reinterpret_cast<typename PP::type*>(out + (size_t)t * (2u * (uint32_t)d.nbins)) + (r0 + n + 64 * q);
        float p[16], hh[16];
        static_for<0, 16>([&](auto ic) {
          constexpr int i = decltype(ic)::value, e = i / 4, kb = i % 4;
          const c32 dv = {y[e][kb].re - nx[e][kb].re, y[e][kb].im - nx[e][kb].im};
          p[i] = cnorm(y[e][kb]) * pscale;
          hh[i] = 0.5f * cnorm(dv) * pscale;
          m[i] = max(capped_bits<PDT>(PS::pack_real(p[i])), capped_bits<PDT>(PS::pack_real(hh[i])));
        });
        group_max<G8>(m);
        static_for<0, 16>([&](auto ic) {
          constexpr int i = decltype(ic)::value, off = 16 * (i / 4) + 256 * (i % 4);
          const int k = n + 64 * q + off;
          if (k >= lo && k < hi) {
            dst[off] = PP::pack(p[i], hh[i]);
            if (lead) mdst[off / G8] = from_bits<PDT>(m[i]);
          }
        });
      } else {
        RT* dst = out + (size_t)t * (uint32_t)d.nbins + (r0 + n + 64 * q);
        RT p[16];
        static_for<0, 16>([&](auto ic) {
          constexpr int i = decltype(ic)::value;
          p[i] = PS::pack_real(cnorm(y[i / 4][i % 4]) * pscale);
          m[i] = capped_bits<PDT>(p[i]);
        });
        group_max<G8>(m);
        static_for<0, 16>([&](auto ic) {
          constexpr int i = decltype(ic)::value, off = 16 * (i / 4) + 256 * (i % 4);
          const int k = n + 64 * q + off;
          if (k >= lo && k < hi) {
            dst[off] = p[i];
            if (lead) mdst[off / G8] = from_bits<PDT>(m[i]);
          }
        });
      }
    } else {
    c32 v[P];
    static_for<0, P>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      v[c] = cmul(F[c], SS::unpack(tc[c]));
    });
    fft_run<FS, 1, BLOCK>(v, xb, tw, tid);
    if constexpr (IB) {
      c32 nx[P];
      next_outputs<FS, BLOCK>(v, nx, edge, tid);
      using PP = PowerPair<PDT>;
      typename PP::type* dst =
          reinterpret_cast<typename PP::type*>(out + (size_t)t * (2u * (uint32_t)d.nbins)) + (r0 + tid);
      // maxima of row t: 2 nbins / 8 per row; group g of register c (the
      // lanes from grp0) at column (r0 + grp0 + NT c) / 4
      RT* mdst = mx + (size_t)t * (uint32_t)(d.nbins / G8) + (r0 + grp0) / G8;
      float p[P], h[P];
      uint32_t m[P];
      static_for<0, P>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        const c32 dv = {v[c].re - nx[c].re, v[c].im - nx[c].im};
        p[c] = cnorm(v[c]);
        h[c] = 0.5f * cnorm(dv);
        m[c] = max(capped_bits<PDT>(PS::pack_real(p[c])), capped_bits<PDT>(PS::pack_real(h[c])));
      });
      group_max<G8>(m);
      static_for<0, P>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if (NT * c + NT - 1 < lo || NT * c >= hi) return;
        const int i = tid + NT * c;
        if (i >= lo && i < hi) {
          dst[NT * c] = PP::pack(p[c], h[c]);
          if (lead) mdst[NT / G8 * c] = from_bits<PDT>(m[c]);
        }
      });
    } else {
      // this thread's output i = tid + NT c lands at bin r0 + i of row t: one
      // 64-bit pointer per template, the register index as an immediate offset
      RT* dst = out + (size_t)t * (uint32_t)d.nbins + (r0 + tid);
      RT* mdst = mx + (size_t)t * (uint32_t)(d.nbins / G8) + (r0 + grp0) / G8;
      RT p[P];
      uint32_t m[P];
      static_for<0, P>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        p[c] = PS::pack_real(cnorm(v[c]));
        m[c] = capped_bits<PDT>(p[c]);
      });
      group_max<G8>(m);
      static_for<0, P>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        // the register is out of range for every thread: skip (uniform branch)
        if (NT * c + NT - 1 < lo || NT * c >= hi) return;
        const int i = tid + NT * c;
        if (i >= lo && i < hi) {
          dst[NT * c] = p[c];
          if (lead) mdst[NT / G8 * c] = from_bits<PDT>(m[c]);
        }
      });
    }
    }
    static_for<0, P>([&](auto cc) { tc[decltype(cc)::value] = tn[decltype(cc)::value]; });
  }
}

constexpr int kConvWaves = 4;  // wavefronts per block of the one-wavefront-per-FFT kernel

// Convolution FFT shapes: 16 points per thread and passes of radix R (16 by
// default; the 1024-point one-wavefront FFT is also built with R = 8, passes
// 8 8 8 2, and R = 4, five passes of 4, for the autotuner).  The twiddle
// table depends only on the radix sequence (conv_twiddle_size / _fill in
// k_fft.hip).
template <int L, int R = 16>
using ConvShape = FftShape<L, 16, R>;

// Wavefronts per SIMD: two for the FP32 inverse FFTs (with the template
// prefetch in registers a third measured no faster); three for the FP16
// matrix-core inverse FFT with 16-bit storage (168 VGPRs, 52 KB of LDS per
// block), whose chain of dependent steps per template (register transpose,
// MFMA, twiddles, MFMA) needs the extra wavefront to hide its latency (-5 %).
template <int L, int R, int SDT, int PDT, bool IB>
constexpr int conv_wave_occupancy() { return use_mfma<L, R, PDT, IB>() && Store<SDT>::RBYTES == 2 ? 3 : 2; }

template <int L, int SDT, int PDT, bool IB, int R>
__global__ __launch_bounds__(64 * kConvWaves) __attribute__((amdgpu_waves_per_eu(conv_wave_occupancy<L, R, SDT, PDT, IB>())))
void k_conv_wave(ConvArgs a) {
  using FS = ConvShape<L, R>;
  static_assert(FS::NT == 64, "one wavefront per FFT");
  constexpr bool MF = use_mfma<L, R, PDT, IB>();
  __shared__ c32 tw[FS::TW_SIZE];
  __shared__ c32 xb[kConvWaves][FS::XBUF];
  __shared__ __align__(16) uint32_t tw2[MF ? mf::kTw2Size : 1];
  __shared__ c32 tw3[MF ? mf::kTw3Size : 1];
  stage_table(tw, a.tw, FS::TW_SIZE);
  if constexpr (MF) mf::fill_tables(tw2, tw3, threadIdx.x, blockDim.x);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * kConvWaves;
  MfCtx mc;
  if constexpr (MF) mc = {tw2, tw3, mf::make_weights(lane)};
  for (int64_t tile = (int64_t)blockIdx.x * kConvWaves + wave; tile < a.n_tiles; tile += nw)
    conv_tile<FS, SDT, PDT, false, IB, MF>(a, tile, xb[wave], tw, lane, nullptr, &mc);
}

template <int L, int SDT, int PDT, bool IB>
__global__ __launch_bounds__(ConvShape<L>::NT) __attribute__((amdgpu_waves_per_eu(2))) void k_conv_block(ConvArgs a) {
  using FS = ConvShape<L>;
  __shared__ c32 tw[FS::TW_SIZE];
  __shared__ c32 xb[FS::XBUF];
  __shared__ c32 edge[IB ? FS::NT / 64 * FS::P : 1];  // first lane's outputs of each wavefront
  stage_table(tw, a.tw, FS::TW_SIZE);
  __syncthreads();
  for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x)
    conv_tile<FS, SDT, PDT, true, IB>(a, tile, xb, tw, threadIdx.x, edge);
}

bool conv_uses_mfma(int L, int R, int pdt, bool) {
  return L == 1024 && R == 16 && (pdt == FDAS_BF16 || pdt == FDAS_F16);
}
static_assert(use_mfma<1024, 16, FDAS_BF16, false>() && use_mfma<1024, 16, FDAS_F16, false>() &&
                  use_mfma<1024, 16, FDAS_BF16, true>() && !use_mfma<1024, 16, FDAS_F32, false>() &&
                  !use_mfma<1024, 8, FDAS_BF16, false>() && !use_mfma<2048, 16, FDAS_BF16, false>(),
              "conv_uses_mfma matches use_mfma");

int conv_waves_per_block(int L) { return L == 1024 ? kConvWaves : L / 16 / 64; }

bool conv_radix_supported(int L, int R) { return R == 16 || (L == 1024 && (R == 8 || R == 4)); }

template <int L, int SDT, int PDT, bool IB, int R>
static void conv_launch(const ConvArgs& a, int grid, hipStream_t st) {
  if constexpr (ConvShape<L, R>::NT == 64)
    hipLaunchKernelGGL((k_conv_wave<L, SDT, PDT, IB, R>), dim3(grid), dim3(64 * kConvWaves), 0, st, a);
  else
    hipLaunchKernelGGL((k_conv_block<L, SDT, PDT, IB>), dim3(grid), dim3(ConvShape<L>::NT), 0, st, a);
}

template <int L, int SDT, int PDT, bool IB, int R>
static int occ() {
  int n = 0;
  hipError_t e;
  if constexpr (ConvShape<L, R>::NT == 64)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_conv_wave<L, SDT, PDT, IB, R>, 64 * kConvWaves, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_conv_block<L, SDT, PDT, IB>, ConvShape<L>::NT, 0);
  if (e != hipSuccess) n = 1;
  return n;
}

// Calls f(integral_constant<int, dt>) for a storage type known at run time.
template <class F>
static auto with_dtype(int dt, F&& f) {
  switch (dt) {
    case FDAS_F32: return f(std::integral_constant<int, FDAS_F32>{});
    case FDAS_BF16: return f(std::integral_constant<int, FDAS_BF16>{});
    default: return f(std::integral_constant<int, FDAS_F16>{});
  }
}

// Calls f(integral_constant<int, R>) for the radices built at length L.
template <int L, class F>
static auto with_radix(int r, F&& f) {
  if constexpr (L == 1024) {
    if (r == 8) return f(std::integral_constant<int, 8>{});
    if (r == 4) return f(std::integral_constant<int, 4>{});
  }
  return f(std::integral_constant<int, 16>{});
}

template <int L>
static int occ_l(int r, int sdt, int pdt, bool ib) {
  return with_radix<L>(r, [&](auto rc) {
    constexpr int R = decltype(rc)::value;
    return with_dtype(sdt, [&](auto sd) {
      return with_dtype(pdt, [&](auto pd) {
        constexpr int S = decltype(sd)::value, Q = decltype(pd)::value;
        return ib ? occ<L, S, Q, true, R>() : occ<L, S, Q, false, R>();
      });
    });
  });
}

int conv_blocks_per_cu(int L, int R, int sdt, int pdt, bool interbin) {
  switch (L) {
    case 1024: return occ_l<1024>(R, sdt, pdt, interbin);
    case 2048: return occ_l<2048>(R, sdt, pdt, interbin);
    case 4096: return occ_l<4096>(R, sdt, pdt, interbin);
    case 8192: return occ_l<8192>(R, sdt, pdt, interbin);
    default: return 1;
  }
}

template <int L>
static hipError_t conv_l(int r, int sdt, int pdt, bool ib, const ConvArgs& a, int grid, hipStream_t st) {
  if (sdt < FDAS_F32 || sdt > FDAS_F16 || pdt < FDAS_F32 || pdt > FDAS_F16) return hipErrorInvalidValue;
  if (!conv_radix_supported(L, r)) return hipErrorInvalidValue;
  with_radix<L>(r, [&](auto rc) {
    constexpr int R = decltype(rc)::value;
    with_dtype(sdt, [&](auto sd) {
      with_dtype(pdt, [&](auto pd) {
        constexpr int S = decltype(sd)::value, Q = decltype(pd)::value;
        if (ib)
          conv_launch<L, S, Q, true, R>(a, grid, st);
        else
          conv_launch<L, S, Q, false, R>(a, grid, st);
        return 0;
      });
      return 0;
    });
    return 0;
  });
  return hipGetLastError();
}

hipError_t launch_conv(int L, int R, int sdt, int pdt, bool interbin, const ConvArgs& a, int grid, hipStream_t st) {
  switch (L) {
    case 1024: return conv_l<1024>(R, sdt, pdt, interbin, a, grid, st);
    case 2048: return conv_l<2048>(R, sdt, pdt, interbin, a, grid, st);
    case 4096: return conv_l<4096>(R, sdt, pdt, interbin, a, grid, st);
    case 8192: return conv_l<8192>(R, sdt, pdt, interbin, a, grid, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fdas
