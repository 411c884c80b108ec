// Shared device helpers for the FDAS kernels: complex arithmetic, storage-dtype
// packing (float32 / bfloat16 / float16 pairs) and wavefront-local LDS ordering.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fdas.h"

namespace fdas {

struct c32 {
  float re, im;
};

__device__ __forceinline__ c32 cadd(c32 a, c32 b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ c32 csub(c32 a, c32 b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ c32 cmul(c32 a, c32 b) {
  return {__builtin_fmaf(a.re, b.re, -a.im * b.im), __builtin_fmaf(a.re, b.im, a.im * b.re)};
}
// a * conj(b)
__device__ __forceinline__ c32 cmulc(c32 a, c32 b) {
  return {__builtin_fmaf(a.re, b.re, a.im * b.im), __builtin_fmaf(a.im, b.re, -a.re * b.im)};
}
__device__ __forceinline__ float cnorm(c32 a) { return __builtin_fmaf(a.re, a.re, a.im * a.im); }

// ---------------------------------------------------------------- storage types
// Complex values are stored as an (re, im) pair of the storage type:
//   FDAS_F32  -> 8 bytes (two floats)
//   FDAS_BF16 -> 4 bytes (two bfloat16, re in the low half)
//   FDAS_F16  -> 4 bytes (two IEEE binary16, re in the low half)
// Conversions to the 16-bit types round to nearest even.

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

template <int DT> struct Store;

template <> struct Store<FDAS_F32> {
  typedef float2 cplx_t;
  typedef float real_t;
  static constexpr int CBYTES = 8, RBYTES = 4;
  __device__ __forceinline__ static c32 unpack(cplx_t v) { return {v.x, v.y}; }
  __device__ __forceinline__ static cplx_t pack(c32 v) { return make_float2(v.re, v.im); }
  __device__ __forceinline__ static real_t pack_real(float v) { return v; }
  __device__ __forceinline__ static float unpack_real(real_t v) { return v; }
};

template <> struct Store<FDAS_BF16> {
  typedef uint32_t cplx_t;
  typedef uint16_t real_t;
  static constexpr int CBYTES = 4, RBYTES = 2;
  __device__ __forceinline__ static c32 unpack(cplx_t v) {
    return {__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u)};
  }
  __device__ __forceinline__ static cplx_t pack(c32 v) {
    bf16x2 p;
    p.x = (__bf16)v.re;
    p.y = (__bf16)v.im;
    return __builtin_bit_cast(uint32_t, p);
  }
  __device__ __forceinline__ static real_t pack_real(float v) {
    return __builtin_bit_cast(uint16_t, (__bf16)v);
  }
  __device__ __forceinline__ static float unpack_real(real_t v) { return __uint_as_float(((uint32_t)v) << 16); }
};

template <> struct Store<FDAS_F16> {
  typedef uint32_t cplx_t;
  typedef uint16_t real_t;
  static constexpr int CBYTES = 4, RBYTES = 2;
  __device__ __forceinline__ static c32 unpack(cplx_t v) {
    f16x2 p = __builtin_bit_cast(f16x2, v);
    return {(float)p.x, (float)p.y};
  }
  __device__ __forceinline__ static cplx_t pack(c32 v) {
    f16x2 p;
    p.x = (_Float16)v.re;
    p.y = (_Float16)v.im;
    return __builtin_bit_cast(uint32_t, p);
  }
  __device__ __forceinline__ static real_t pack_real(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
  __device__ __forceinline__ static float unpack_real(real_t v) { return (float)__builtin_bit_cast(_Float16, v); }
};

// Column maxima of a plane are taken on bit patterns: for a non-negative
// value (+inf included) the pattern read as an unsigned integer orders like
// the value, and every other pattern (a NaN, or a sign bit) is capped at
// +inf's, so that it counts as +inf; a maximum is then an upper bound of
// every value of its run, whatever the values are.
template <int PDT>
__device__ __forceinline__ uint32_t capped_bits(typename Store<PDT>::real_t x) {
  if constexpr (PDT == FDAS_F32)
    return min(__float_as_uint(x), 0x7f800000u);
  else
    return min((uint32_t)x, PDT == FDAS_BF16 ? 0x7f80u : 0x7c00u);
}
template <int PDT>
__device__ __forceinline__ typename Store<PDT>::real_t from_bits(uint32_t b) {
  if constexpr (PDT == FDAS_F32)
    return __uint_as_float(b);
  else
    return (typename Store<PDT>::real_t)b;
}

// Orders LDS traffic of one wavefront: LDS operations of a wavefront complete
// in issue order, so a compiler-level barrier is all a wave-private exchange
// buffer needs between its writes and the reads of other lanes.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  asm volatile("" ::: "memory");
}

// Direct global-to-LDS load of 16 bytes per lane (gfx950): lane i's bytes go
// to lds_wave_base + 16 i, lds_wave_base being wave-uniform; inactive lanes
// write nothing.  The data is visible to the block after a barrier (the
// compiler waits for the loads there).  The builtin exists only in the
// device pass, so the host pass sees an empty body.
__device__ __forceinline__ void load_lds16(const void* src, void* lds_wave_base) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds_wave_base, 16, 0, 0);
#endif
}

// Loads and stores at a uniform base plus a 32-bit byte offset, so that the
// compiler can address with one offset register and immediates.
template <typename T>
__device__ __forceinline__ T ld_off(const void* base, uint32_t off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
template <typename T>
__device__ __forceinline__ void st_off(void* base, uint32_t off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off) = v;
}

__device__ __forceinline__ int wave_lane() { return (int)(threadIdx.x & 63); }

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

}  // namespace fdas
