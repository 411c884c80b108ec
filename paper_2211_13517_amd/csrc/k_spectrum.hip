// Real FFT of each series and spectrum normalisation.
//
// A real series x of N samples is read as M = N/2 complex values
// z[n] = x[2n] + i x[2n+1] and transformed with a four-step FFT, M = M1 * M2:
//   columns: for each n2, FFT_M1 over z[n1 M2 + n2], times exp(-2 pi i n2 k1 / M),
//            stored at Y[k1 M2 + n2];
//   rows:    for each k1, FFT_M2 over Y[k1 M2 + n2], giving Z[k1 + M1 k2].
// The last kernel splits Z into the spectra of the even and odd samples,
//   E_k = (Z_k + conj Z_{M-k})/2,  O_k = (Z_k - conj Z_{M-k})/(2i),
//   A_k = E_k + exp(-2 pi i k / N) O_k,   k < N/2,
// zeroes A_0, normalises each block of B bins (by the lower median of |A|^2,
// or by a constant) and stores the spectrum in the storage dtype.
#include "fft.hpp"
#include "launch.hpp"

namespace fdas {

constexpr int kWaves = 8;  // FFTs (one per wavefront) per 512-thread block

// Both passes move data between HBM and the wavefronts' thread-strided FFT
// layout (lane l holds points l + 64 c) through 64-row x 8-column chunks in
// LDS: the block's 8 columns (or rows) are 8 consecutive complex values in
// memory, so every global access of a chunk is a run of 64 bytes instead of
// one 8-byte value per lane at a 16 KB stride.  The chunks borrow the FFT
// exchange buffers, which are idle before and after the transform.
struct Chunk {
  static constexpr int PITCH = 9;                // floats per row: 8 columns + pad (no bank conflicts)
  static constexpr int FLOATS = 2 * 64 * PITCH;  // re and im planes of one chunk
};

// every thread: chunk element (row t / 8, column t % 8) <-> this lane's (l, column w)
__device__ __forceinline__ void chunk_put(float* buf, int row, int col, c32 v) {
  buf[row * Chunk::PITCH + col] = v.re;
  buf[64 * Chunk::PITCH + row * Chunk::PITCH + col] = v.im;
}
__device__ __forceinline__ c32 chunk_get(const float* buf, int row, int col) {
  return {buf[row * Chunk::PITCH + col], buf[64 * Chunk::PITCH + row * Chunk::PITCH + col]};
}

template <int M1>
__global__ __launch_bounds__(512) void k_rfft_cols(const float* __restrict__ x, const SeriesDesc* __restrict__ desc,
                                                   const int32_t* __restrict__ list, int M2, c32* __restrict__ Y,
                                                   const c32* __restrict__ twg) {
  using FS = typename ShapeOf<M1>::type;
  constexpr int P = FS::P;
  static_assert(kWaves * FS::XBUF * 2 >= 2 * Chunk::FLOATS, "chunks fit in the exchange buffers");
  __shared__ c32 tw[FS::TW_SIZE];
  __shared__ c32 xb[kWaves][FS::XBUF];
  stage_table(tw, twg, FS::TW_SIZE);
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int n2_0 = blockIdx.x * kWaves;  // M2 is a multiple of kWaves
  const SeriesDesc d = desc[list[blockIdx.y]];
  const uint32_t M = (uint32_t)M1 * (uint32_t)M2;
  const float2* z = reinterpret_cast<const float2*>(x + d.in_off);
  float* cbuf = reinterpret_cast<float*>(&xb[0][0]);
  // every load of the column group in flight at once
  float2 g[P];
  static_for<0, P>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    g[c] = z[(size_t)(64 * c + (t >> 3)) * M2 + n2_0 + (t & 7)];
  });
  c32 v[P];
  static_for<0, P>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    float* buf = cbuf + (c & 1) * Chunk::FLOATS;
    chunk_put(buf, t >> 3, t & 7, c32{g[c].x, g[c].y});
    __syncthreads();
    v[c] = chunk_get(buf, lane, wave);
  });
  __syncthreads();  // the chunks' LDS becomes the FFT exchange buffers
  fft_run<FS, -1, false>(v, xb[wave], tw, lane);
  const int n2 = n2_0 + wave;
  const float inv = 1.0f / (float)M;
  static_for<0, P>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    const uint32_t k1 = lane + 64 * c;
    const uint32_t idx = ((uint32_t)n2 * k1) & (M - 1);
    float s, co;
    sincospif(-2.0f * (float)idx * inv, &s, &co);
    v[c] = cmul(v[c], c32{co, s});
  });
  __syncthreads();  // and back to chunks
  c32* y = Y + d.spec_off;
  static_for<0, P>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    float* buf = cbuf + (c & 1) * Chunk::FLOATS;
    chunk_put(buf, lane, wave, v[c]);
    __syncthreads();
    const c32 o = chunk_get(buf, t >> 3, t & 7);
    y[(size_t)(64 * c + (t >> 3)) * M2 + n2_0 + (t & 7)] = o;
  });
}

template <int M2>
__global__ __launch_bounds__(512) void k_rfft_rows(const SeriesDesc* __restrict__ desc,
                                                   const int32_t* __restrict__ list, int M1,
                                                   const c32* __restrict__ Y, c32* __restrict__ Zb,
                                                   const c32* __restrict__ twg) {
  using FS = typename ShapeOf<M2>::type;
  constexpr int P = FS::P;
  static_assert(kWaves * FS::XBUF * 2 >= 2 * Chunk::FLOATS, "chunks fit in the exchange buffers");
  __shared__ c32 tw[FS::TW_SIZE];
  __shared__ c32 xb[kWaves][FS::XBUF];
  stage_table(tw, twg, FS::TW_SIZE);
  __syncthreads();
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int k1_0 = blockIdx.x * kWaves;  // M1 is a multiple of kWaves
  const SeriesDesc d = desc[list[blockIdx.y]];
  const c32* y = Y + d.spec_off + (size_t)(k1_0 + wave) * M2;
  c32 v[P];
  static_for<0, P>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    v[c] = y[lane + 64 * c];
  });
  fft_run<FS, -1, false>(v, xb[wave], tw, lane);
  __syncthreads();  // the exchange buffers become chunks
  float* cbuf = reinterpret_cast<float*>(&xb[0][0]);
  c32* zo = Zb + d.spec_off;
  static_for<0, P>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    float* buf = cbuf + (c & 1) * Chunk::FLOATS;
    chunk_put(buf, lane, wave, v[c]);
    __syncthreads();
    // Z[k1 + M1 k2]: the block's 8 rows k1 are 8 consecutive outputs
    zo[(size_t)k1_0 + (t & 7) + (size_t)M1 * (64 * c + (t >> 3))] = chunk_get(buf, t >> 3, t & 7);
  });
}

// ---------------------------------------------------------------- median

// Inclusive prefix sum over a 256-thread block.
__device__ __forceinline__ int block_scan256(int v, int* wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  if (lane == 63) wsum[wave] = v;
  __syncthreads();
  int add = 0;
  for (int w = 0; w < wave; ++w) add += wsum[w];
  __syncthreads();
  return v + add;
}

// Exact k-th smallest of n non-negative floats given as their bit patterns
// (which order like the values), by an MSB-first 8-bit radix selection.
__device__ uint32_t block_select(const uint32_t* keys, int n, int k, int* hist, int* wsum, int* shared_sel) {
  uint32_t prefix = 0, mask = 0;
  for (int shift = 24; shift >= 0; shift -= 8) {
    hist[threadIdx.x] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 256) {
      const uint32_t key = keys[i];
      if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255], 1);
    }
    __syncthreads();
    const int h = hist[threadIdx.x];
    const int incl = block_scan256(h, wsum);
    const int excl = incl - h;
    if (excl <= k && k < incl) {
      shared_sel[0] = threadIdx.x;
      shared_sel[1] = excl;
    }
    __syncthreads();
    prefix |= (uint32_t)shared_sel[0] << shift;
    mask |= 255u << shift;
    k -= shared_sel[1];
    __syncthreads();
  }
  return prefix;
}

// Sub-block width of the rednoise normalisation in block b of B bins: the
// largest power of two <= b B / 8, kept within [32, B].
__device__ __forceinline__ int rednoise_width(int b, int B) {
  const int s8 = (b * B) >> 3;
  const int w = s8 > 0 ? 1 << (31 - __clz(s8)) : 1;
  return min(max(w, 32), B);
}

template <int SDT>
__global__ __launch_bounds__(256) void k_unpack_norm(const SeriesDesc* __restrict__ desc,
                                                     const int32_t* __restrict__ list, int M, int B, int mode,
                                                     float var_scale, const c32* __restrict__ Zb, void* spec,
                                                     int32_t* status) {
  using SS = Store<SDT>;
  extern __shared__ unsigned char smem[];
  c32* a = reinterpret_cast<c32*>(smem);
  uint32_t* keys = reinterpret_cast<uint32_t*>(a + B);
  __shared__ int hist[256];
  __shared__ int wsum[4];
  __shared__ int sel[2];
  __shared__ float subscale[128];  // rednoise: one scale per sub-block (B / 32 <= 128)
  const SeriesDesc d = desc[list[blockIdx.y]];
  const c32* zb = Zb + d.spec_off;
  const int N = 2 * M;
  const float invN = 2.0f / (float)N;
  int mybad = 0;
  for (int i = threadIdx.x; i < B; i += 256) {
    const int k = blockIdx.x * B + i;
    const c32 zk = zb[k], zm = zb[(M - k) & (M - 1)];
    const c32 e = {0.5f * (zk.re + zm.re), 0.5f * (zk.im - zm.im)};
    const c32 o = {0.5f * (zk.im + zm.im), -0.5f * (zk.re - zm.re)};
    float s, c;
    sincospif(-(float)k * invN, &s, &c);
    c32 v = cadd(e, cmul(o, c32{c, s}));
    if (k == 0) v = {0.f, 0.f};
    a[i] = v;
    const float p = cnorm(v);
    if (!(p <= 3.4e38f)) mybad = 1;
    keys[i] = __float_as_uint(p);
  }
  const int bad = __syncthreads_or(mybad);
  constexpr float kLn2 = 0.69314718055994530942f;
  float scale = var_scale;
  const int w = mode == FDAS_NORM_REDNOISE ? rednoise_width(blockIdx.x, B) : B;
  if (mode == FDAS_NORM_MEDIAN || (mode == FDAS_NORM_REDNOISE && w == B)) {
    const uint32_t m = block_select(keys, B, (B - 1) / 2, hist, wsum, sel);
    const float med = __uint_as_float(m);
    scale = med > 0.f ? sqrtf(kLn2 / med) : 0.f;
  } else if (mode == FDAS_NORM_REDNOISE) {
    if (w <= 256) {
      // small sub-blocks: each element's rank within its sub-block by direct
      // count (ties ordered by position); rank (w-1)/2 is the lower median
      for (int i = threadIdx.x; i < B; i += 256) {
        const int base = i & ~(w - 1);
        const uint32_t ki = keys[i];
        int rank = 0;
        for (int l = 0; l < w; ++l) {
          const uint32_t kl = keys[base + l];
          rank += (kl < ki) || (kl == ki && base + l < i);
        }
        if (rank == (w - 1) / 2) {
          const float med = __uint_as_float(ki);
          subscale[i / w] = med > 0.f ? sqrtf(kLn2 / med) : 0.f;
        }
      }
    } else {
      for (int j = 0; j < B / w; ++j) {
        const float med = __uint_as_float(block_select(keys + j * w, w, (w - 1) / 2, hist, wsum, sel));
        if (threadIdx.x == 0) subscale[j] = med > 0.f ? sqrtf(kLn2 / med) : 0.f;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && bad) atomicOr(status, 1);
  typename SS::cplx_t* out = reinterpret_cast<typename SS::cplx_t*>(spec) + d.spec_off + (size_t)blockIdx.x * B;
  const bool sub = mode == FDAS_NORM_REDNOISE && w < B;
  for (int i = threadIdx.x; i < B; i += 256) {
    const c32 v = a[i];
    const float sc = sub ? subscale[i / w] : scale;
    out[i] = SS::pack(c32{v.re * sc, v.im * sc});
  }
}

// ---------------------------------------------------------------- launchers

template <int M1>
static void cols(int M2, dim3 g, const float* x, const SeriesDesc* desc, const int32_t* list, c32* Y, const c32* tw,
                 hipStream_t st) {
  hipLaunchKernelGGL((k_rfft_cols<M1>), g, dim3(512), 0, st, x, desc, list, M2, Y, tw);
}

hipError_t launch_rfft_columns(int M1, int M2, const float* x, const SeriesDesc* desc, const int32_t* list,
                               int nlist, c32* Y, const c32* tw, hipStream_t st) {
  const dim3 g((M2 + kWaves - 1) / kWaves, nlist);
  switch (M1) {
    case 256: cols<256>(M2, g, x, desc, list, Y, tw, st); break;
    case 512: cols<512>(M2, g, x, desc, list, Y, tw, st); break;
    case 1024: cols<1024>(M2, g, x, desc, list, Y, tw, st); break;
    case 2048: cols<2048>(M2, g, x, desc, list, Y, tw, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int M2>
static void rows(int M1, dim3 g, const SeriesDesc* desc, const int32_t* list, const c32* Y, c32* Zb, const c32* tw,
                 hipStream_t st) {
  hipLaunchKernelGGL((k_rfft_rows<M2>), g, dim3(512), 0, st, desc, list, M1, Y, Zb, tw);
}

hipError_t launch_rfft_rows(int M1, int M2, const SeriesDesc* desc, const int32_t* list, int nlist, const c32* Y,
                            c32* Zb, const c32* tw, hipStream_t st) {
  const dim3 g((M1 + kWaves - 1) / kWaves, nlist);
  switch (M2) {
    case 256: rows<256>(M1, g, desc, list, Y, Zb, tw, st); break;
    case 512: rows<512>(M1, g, desc, list, Y, Zb, tw, st); break;
    case 1024: rows<1024>(M1, g, desc, list, Y, Zb, tw, st); break;
    case 2048: rows<2048>(M1, g, desc, list, Y, Zb, tw, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_unpack_normalise(int sdt, int M, int B, int mode, double var_scale, const SeriesDesc* desc,
                                   const int32_t* list, int nlist, const c32* Zb, void* spec, int32_t* status,
                                   hipStream_t st) {
  const dim3 g(M / B, nlist);
  const size_t shm = (size_t)B * (sizeof(c32) + sizeof(uint32_t));
  const float vs = (float)var_scale;
  switch (sdt) {
    case FDAS_F32:
      hipLaunchKernelGGL((k_unpack_norm<FDAS_F32>), g, dim3(256), shm, st, desc, list, M, B, mode, vs, Zb, spec, status);
      break;
    case FDAS_BF16:
      hipLaunchKernelGGL((k_unpack_norm<FDAS_BF16>), g, dim3(256), shm, st, desc, list, M, B, mode, vs, Zb, spec, status);
      break;
    case FDAS_F16:
      hipLaunchKernelGGL((k_unpack_norm<FDAS_F16>), g, dim3(256), shm, st, desc, list, M, B, mode, vs, Zb, spec, status);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fdas
