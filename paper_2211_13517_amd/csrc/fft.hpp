// Register + LDS FFT engine for gfx950 (wave64).
//
// An FFT of length L is computed by NT = L/P threads that each hold P complex
// values in registers.  Both input and output are in natural order in the
// "thread-strided" layout: register c of thread tid holds element tid + NT*c.
// The transform is a Stockham autosort sequence of radix passes (radix P for
// every full pass, then one smaller radix for the remainder).  A pass reads
// its R inputs at stride L/R, multiplies by twiddles exp(-+2 pi i (j mod Ns) t
// / (Ns R)), runs an in-register DFT_R and writes to index
// (j/Ns) Ns R + (j mod Ns) + t Ns.  Consecutive passes exchange data through
// a padded LDS buffer (one pad element per P) so that the stride-P writes of
// the first pass hit distinct banks.  Twiddles come from a per-size table
// (forward sign; the inverse uses its conjugate) staged in LDS.
//
// DFTs up to length 32 are unrolled at compile time (radix-4/radix-2
// decimation in time) with constant twiddles folded into the instruction
// stream; multiplications by +-1, +-i are free and odd multiples of pi/4 cost
// two additions and two multiplications.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace fdas {

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

namespace ct {
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double reduce(long k, long n) {
  long kk = ((k % n) + n) % n;
  double t = 2.0 * kPi * (double)kk / (double)n;
  return t > kPi ? t - 2.0 * kPi : t;
}
// Taylor series on [-pi, pi], evaluated by the compiler only.
constexpr double sin_t(double x) {
  double x2 = x * x, term = x, s = x;
  for (int i = 1; i < 30; ++i) {
    term *= -x2 / ((2.0 * i) * (2.0 * i + 1.0));
    s += term;
  }
  return s;
}
constexpr double cos_t(double x) {
  double x2 = x * x, term = 1.0, s = 1.0;
  for (int i = 1; i < 30; ++i) {
    term *= -x2 / ((2.0 * i - 1.0) * (2.0 * i));
    s += term;
  }
  return s;
}
constexpr double cos2pi(long k, long n) { return cos_t(reduce(k, n)); }
constexpr double sin2pi(long k, long n) { return sin_t(reduce(k, n)); }
constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }
}  // namespace ct

// x * exp(DIR * 2 pi i K / N) with K, N known at compile time.
template <long K, long N, int DIR>
__device__ __forceinline__ c32 twc(c32 x) {
  constexpr long k = ((K % N) + N) % N;
  if constexpr (k == 0) {
    return x;
  } else if constexpr (2 * k == N) {
    return {-x.re, -x.im};
  } else if constexpr (4 * k == N) {  // DIR * i
    if constexpr (DIR > 0) return {-x.im, x.re};
    else return {x.im, -x.re};
  } else if constexpr (4 * k == 3 * N) {  // -DIR * i
    if constexpr (DIR > 0) return {x.im, -x.re};
    else return {-x.im, x.re};
  } else if constexpr ((8 * k) % N == 0) {  // odd multiple of pi/4: |cos| = |sin| = 1/sqrt(2)
    constexpr float h = 0.70710678118654752440f;
    constexpr bool cpos = ct::cos2pi(k, N) > 0;
    constexpr bool spos = (DIR * ct::sin2pi(k, N)) > 0;
    const float a = (cpos ? x.re : -x.re) - (spos ? x.im : -x.im);
    const float b = (spos ? x.re : -x.re) + (cpos ? x.im : -x.im);
    return {h * a, h * b};
  } else {
    constexpr float c = (float)ct::cos2pi(k, N);
    constexpr float s = (float)(DIR * ct::sin2pi(k, N));
    return {__builtin_fmaf(x.re, c, -x.im * s), __builtin_fmaf(x.re, s, x.im * c)};
  }
}

template <int N, int DIR>
struct Dft;

template <int DIR>
struct Dft<1, DIR> {
  __device__ __forceinline__ static void run(c32*) {}
};

template <int DIR>
struct Dft<2, DIR> {
  __device__ __forceinline__ static void run(c32* v) {
    const c32 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int DIR>
struct Dft<4, DIR> {
  __device__ __forceinline__ static void run(c32* v) {
    const c32 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    const c32 c = cadd(v[1], v[3]), d = twc<1, 4, DIR>(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  }
};

// Decimation in time: R0 interleaved sub-sequences, DFT_{N/R0} each, twiddle
// by exp(DIR 2 pi i r k / N), DFT_R0 across them.
template <int N, int DIR>
struct Dft {
  __device__ __forceinline__ static void run(c32* v) {
    constexpr int R0 = (N % 4 == 0 && N != 8) ? 4 : 2;
    constexpr int M = N / R0;
    c32 s[R0][M];
    static_for<0, R0>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      static_for<0, M>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        s[r][i] = v[R0 * i + r];
      });
      Dft<M, DIR>::run(s[r]);
    });
    static_for<0, M>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      c32 t[R0];
      static_for<0, R0>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        t[r] = twc<(long)r * k, N, DIR>(s[r][k]);
      });
      Dft<R0, DIR>::run(t);
      static_for<0, R0>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        v[k + M * p] = t[p];
      });
    });
  }
};

// Static description of one FFT size: L points, P per thread, radix R for
// every full pass (R divides P; a thread runs P/R butterflies per pass) and
// one last pass with the remaining radix.
template <int L_, int P_, int R_ = P_>
struct FftShape {
  static constexpr int L = L_, P = P_, R = R_, NT = L / P, PADSHIFT = ilog2(R);
  static constexpr int count_full() {
    int n = 0, rem = L;
    while (rem >= R && rem % R == 0) {
      rem /= R;
      ++n;
    }
    return n;
  }
  static constexpr int NFULL = count_full();
  static constexpr int RLAST = L / ct::ipow(R, NFULL);
  static constexpr int NPASS = NFULL + (RLAST > 1 ? 1 : 0);
  static constexpr int radix(int p) { return p < NFULL ? R : RLAST; }
  static constexpr int ns(int p) {
    int n = 1;
    for (int i = 0; i < p; ++i) n *= radix(i);
    return n;
  }
  static constexpr int tw_off(int p) {
    int o = 0;
    for (int i = 1; i < p; ++i) o += ns(i) * (radix(i) - 1);
    return o;
  }
  static constexpr int TW_SIZE = tw_off(NPASS);    // complex entries of the twiddle table
  static constexpr int XBUF = L + (L >> PADSHIFT);  // complex entries of the exchange buffer
  static_assert(P % R == 0 && P % RLAST == 0, "radices must divide P");
  static_assert(NT % 64 == 0, "whole wavefronts");
  __device__ __forceinline__ static int pad(int e) { return e + (e >> PADSHIFT); }
};

// Register order of the butterflies of a pass with radix R: v[m R + t] is
// element t of butterfly m; the thread-strided order has it at m + t (P/R).
template <int P, int R>
__device__ __forceinline__ void to_butterfly_order(c32 (&v)[P]) {
  constexpr int G = P / R;
  if constexpr (G > 1) {
    c32 tmp[P];
    static_for<0, P>([&](auto ic) { tmp[decltype(ic)::value] = v[decltype(ic)::value]; });
    static_for<0, G>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      static_for<0, R>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        v[m * R + t] = tmp[m + t * G];
      });
    });
  }
}

template <int P, int R>
__device__ __forceinline__ void from_butterfly_order(c32 (&v)[P]) {
  constexpr int G = P / R;
  if constexpr (G > 1) {
    c32 tmp[P];
    static_for<0, P>([&](auto ic) { tmp[decltype(ic)::value] = v[decltype(ic)::value]; });
    static_for<0, G>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      static_for<0, R>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        v[m + t * G] = tmp[m * R + t];
      });
    });
  }
}

template <bool BLOCK>
__device__ __forceinline__ void xsync() {
  if constexpr (BLOCK) __syncthreads();
  else wave_lds_fence();
}

// In-place FFT of v (thread-strided natural order in and out).  DIR = -1
// forward, +1 inverse (unnormalised).  xbuf: this FFT's LDS exchange buffer
// (FS::XBUF entries); tw: the size's twiddle table in LDS.  BLOCK selects
// workgroup barriers (FFT spread over several wavefronts) or wavefront-local
// ordering (FFT owned by one wavefront).
// Offsets of the padded exchange buffer.  pad() is linear over the strides the
// passes use (multiples of 2^PADSHIFT, or sub-block steps inside a
// 2^PADSHIFT-aligned group), so every access is one base register plus a
// compile-time immediate.
template <class FS>
constexpr int padded(int e) {
  return e + (e >> FS::PADSHIFT);
}

template <class FS, int DIR, bool BLOCK>
__device__ __forceinline__ void fft_run(c32 (&v)[FS::P], c32* xbuf, const c32* tw, int tid) {
  {
    constexpr int R = FS::radix(0), G = FS::P / R;
    to_butterfly_order<FS::P, R>(v);
    static_for<0, G>([&](auto mc) { Dft<R, DIR>::run(&v[decltype(mc)::value * R]); });
  }
  const int rbase = FS::pad(tid);
  static_for<1, FS::NPASS>([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    constexpr int Rp = FS::radix(p - 1), NSp = FS::ns(p - 1), Gp = FS::P / Rp;
    constexpr int R = FS::radix(p), NS = FS::ns(p), G = FS::P / R, STRIDE = FS::L / R;
    static_assert(FS::NT % NSp == 0, "write pattern must be linear in the butterfly index");
    {
      const int idx0 = (tid / NSp) * NSp * Rp + (tid & (NSp - 1));
      c32* wb = xbuf + FS::pad(idx0);
      static_for<0, Gp>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        static_for<0, Rp>([&](auto tc) {
          constexpr int t = decltype(tc)::value;
          wb[padded<FS>(m * FS::NT * Rp + t * NSp)] = v[m * Rp + t];
        });
      });
    }
    xsync<BLOCK>();
    {
      const c32* rb = xbuf + rbase;
      static_for<0, G>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        static_for<0, R>([&](auto tc) {
          constexpr int t = decltype(tc)::value;
          v[m * R + t] = rb[padded<FS>(m * FS::NT + t * STRIDE)];
        });
      });
    }
    xsync<BLOCK>();
    static_for<0, G>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      const c32* twp = tw + FS::tw_off(p) + ((tid + m * FS::NT) & (NS - 1));
      static_for<1, R>([&](auto tc) {
        constexpr int t = decltype(tc)::value;
        const c32 w = twp[(t - 1) * NS];
        v[m * R + t] = DIR > 0 ? cmulc(v[m * R + t], w) : cmul(v[m * R + t], w);
      });
      Dft<R, DIR>::run(&v[m * R]);
    });
  });
  from_butterfly_order<FS::P, FS::radix(FS::NPASS - 1)>(v);
}

// Copies a twiddle table from global memory into LDS (all threads of the block).
__device__ __forceinline__ void stage_table(c32* dst, const c32* src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

}  // namespace fdas
