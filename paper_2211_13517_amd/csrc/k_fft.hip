// Twiddle tables of the FFT engine and a batched complex-FFT self-test kernel.
#include <cmath>

#include "fft.hpp"
#include "launch.hpp"

namespace fdas {

int fft_points_per_thread(int L) {
  switch (L) {
    case 256: return ShapeOf<256>::type::P;
    case 512: return ShapeOf<512>::type::P;
    case 1024: return ShapeOf<1024>::type::P;
    case 2048: return ShapeOf<2048>::type::P;
    case 4096: return ShapeOf<4096>::type::P;
    case 8192: return ShapeOf<8192>::type::P;
    default: return 0;
  }
}

template <class FS>
static void fill_table(c32* dst) {
  for (int p = 1; p < FS::NPASS; ++p) {
    const int R = FS::radix(p), NS = FS::ns(p);
    for (int t = 1; t < R; ++t)
      for (int jm = 0; jm < NS; ++jm) {
        const long k = (long)jm * t, n = (long)NS * R;
        const double a = -2.0 * M_PI * (double)k / (double)n;
        dst[FS::tw_off(p) + (t - 1) * NS + jm] = {(float)std::cos(a), (float)std::sin(a)};
      }
  }
}

int twiddle_table_size(int L) {
  switch (L) {
    case 256: return ShapeOf<256>::type::TW_SIZE;
    case 512: return ShapeOf<512>::type::TW_SIZE;
    case 1024: return ShapeOf<1024>::type::TW_SIZE;
    case 2048: return ShapeOf<2048>::type::TW_SIZE;
    case 4096: return ShapeOf<4096>::type::TW_SIZE;
    case 8192: return ShapeOf<8192>::type::TW_SIZE;
    default: return 0;
  }
}

void twiddle_table_fill(int L, c32* dst) {
  switch (L) {
    case 256: fill_table<ShapeOf<256>::type>(dst); break;
    case 512: fill_table<ShapeOf<512>::type>(dst); break;
    case 1024: fill_table<ShapeOf<1024>::type>(dst); break;
    case 2048: fill_table<ShapeOf<2048>::type>(dst); break;
    case 4096: fill_table<ShapeOf<4096>::type>(dst); break;
    case 8192: fill_table<ShapeOf<8192>::type>(dst); break;
    default: break;
  }
}

// Tables of the convolution's FFT shapes: 16 points per thread, passes of
// radix R (the radix-16 ones are the tables above).
int conv_twiddle_size(int L, int R) {
  if (R == 16) return twiddle_table_size(L);
  if (L == 1024 && R == 8) return FftShape<1024, 16, 8>::TW_SIZE;
  if (L == 1024 && R == 4) return FftShape<1024, 16, 4>::TW_SIZE;
  return 0;
}

void conv_twiddle_fill(int L, int R, c32* dst) {
  if (R == 16) twiddle_table_fill(L, dst);
  else if (L == 1024 && R == 8) fill_table<FftShape<1024, 16, 8>>(dst);
  else if (L == 1024 && R == 4) fill_table<FftShape<1024, 16, 4>>(dst);
}

// One FFT per group of NT threads; blocks hold whole groups.
template <int L, int DIR>
__global__ __launch_bounds__(512) void k_test_fft(const c32* __restrict__ in, c32* __restrict__ out, int64_t batch,
                                                  const c32* __restrict__ twg) {
  using FS = typename ShapeOf<L>::type;
  constexpr int P = FS::P;
  constexpr int GROUPS = (256 / FS::NT) > 0 ? (256 / FS::NT) : 1;  // NT <= 256: blocks of 256 threads
  constexpr bool BLOCK = FS::NT > 64;
  __shared__ c32 tw[FS::TW_SIZE];
  __shared__ c32 xb[GROUPS][FS::XBUF];
  stage_table(tw, twg, FS::TW_SIZE);
  __syncthreads();
  const int grp = threadIdx.x / FS::NT, tid = threadIdx.x % FS::NT;
  const int64_t f = (int64_t)blockIdx.x * GROUPS + grp;
  if (BLOCK) {
    // whole block is one FFT; all threads stay for the barriers
    c32 v[P];
    static_for<0, P>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      v[c] = f < batch ? in[f * L + tid + FS::NT * c] : c32{0.f, 0.f};
    });
    fft_run<FS, DIR, true>(v, xb[grp], tw, tid);
    if (f < batch)
      static_for<0, P>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        out[f * L + tid + FS::NT * c] = v[c];
      });
  } else {
    if (f >= batch) return;
    c32 v[P];
    static_for<0, P>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      v[c] = in[f * L + tid + FS::NT * c];
    });
    fft_run<FS, DIR, false>(v, xb[grp], tw, tid);
    static_for<0, P>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      out[f * L + tid + FS::NT * c] = v[c];
    });
  }
}

template <int L>
static hipError_t run_test(int dir, const c32* in, c32* out, int64_t batch, const c32* tw, hipStream_t st) {
  using FS = typename ShapeOf<L>::type;
  constexpr int threads = FS::NT > 256 ? FS::NT : 256;
  constexpr int groups = FS::NT > 256 ? 1 : 256 / FS::NT;
  const int64_t blocks = (batch + groups - 1) / groups;
  if (dir < 0)
    hipLaunchKernelGGL((k_test_fft<L, -1>), dim3((unsigned)blocks), dim3(threads), 0, st, in, out, batch, tw);
  else
    hipLaunchKernelGGL((k_test_fft<L, 1>), dim3((unsigned)blocks), dim3(threads), 0, st, in, out, batch, tw);
  return hipGetLastError();
}

hipError_t launch_test_fft(int L, int dir, const c32* in, c32* out, int64_t batch, const c32* tw, hipStream_t st) {
  switch (L) {
    case 256: return run_test<256>(dir, in, out, batch, tw, st);
    case 512: return run_test<512>(dir, in, out, batch, tw, st);
    case 1024: return run_test<1024>(dir, in, out, batch, tw, st);
    case 2048: return run_test<2048>(dir, in, out, batch, tw, st);
    case 4096: return run_test<4096>(dir, in, out, batch, tw, st);
    case 8192: return run_test<8192>(dir, in, out, batch, tw, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fdas
