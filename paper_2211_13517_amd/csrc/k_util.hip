// Small device helpers: an int64 fill (a kernel, so it is safe inside
// captured graphs) and a deterministic complex-noise spectrum used by the
// autotuner to time the convolution without any host data.
#include "launch.hpp"

namespace fdas {

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// SplitMix64 (Steele, Lea & Flood 2014) mapped to a value in [-1, 1).
__device__ inline float u11(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (float)((double)(x >> 11) * (1.0 / 4503599627370496.0) - 1.0);
}

template <int SDT>
__global__ void k_fill_noise(void* spec, int64_t n, uint64_t seed) {
  using SS = Store<SDT>;
  auto* o = reinterpret_cast<typename SS::cplx_t*>(spec);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    o[i] = SS::pack(c32{u11(seed ^ (2 * (uint64_t)i)), u11(seed ^ (2 * (uint64_t)i + 1))});
}

hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t value, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, st, p, n, value);
  return hipGetLastError();
}

hipError_t launch_fill_noise(void* spec, int sdt, int64_t nbins, uint64_t seed, hipStream_t st) {
  const dim3 g(1024), b(256);
  switch (sdt) {
    case FDAS_F32: hipLaunchKernelGGL((k_fill_noise<FDAS_F32>), g, b, 0, st, spec, nbins, seed); break;
    case FDAS_BF16: hipLaunchKernelGGL((k_fill_noise<FDAS_BF16>), g, b, 0, st, spec, nbins, seed); break;
    case FDAS_F16: hipLaunchKernelGGL((k_fill_noise<FDAS_F16>), g, b, 0, st, spec, nbins, seed); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fdas
