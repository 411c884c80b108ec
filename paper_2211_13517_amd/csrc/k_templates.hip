// The FP64 template bank.
//
// For acceleration trial z_j = z_min + j dz the matched filter has taps
//   t_q = conj(rho(q, z_j)) / sqrt(E_j),  |q| <= h_j = ceil(|z_j|/2) + m,
//   E_j = sum_{|q| <= h_j} |rho(q, z_j)|^2,
// zero for h_j < |q| <= h_max.  Placing tap q at index (L - q) mod L turns the
// correlation sum_q A_{r+q} t_q into a cyclic convolution, whose kernel
// spectrum (with the inverse FFT's 1/L folded in) is
//   T_j[k] = (1/L) sum_q t_q exp(+2 pi i k q / L),
// evaluated here as a direct FP64 sum over the at most 2 h_max + 1 taps with
// exactly reduced phases (k q mod L) from an FP64 table, then rounded once to
// the storage type.
#include "fft.hpp"
#include "launch.hpp"

namespace fdas {

__global__ void k_exp_table(c64* tab, int L) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < L) tab[m] = cispi64(2.0 * (double)m / (double)L);
}

__global__ __launch_bounds__(256) void k_template_taps(double z_min, double z_step, int margin, int hmax,
                                                       c64* __restrict__ taps) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  const double z = z_min + z_step * (double)j;
  const int h = (int)ceil(fabs(z) / 2.0) + margin;
  const int K = 2 * hmax + 1;
  c64* row = taps + (size_t)j * K;
  double e = 0.0;
  for (int i = threadIdx.x; i < K; i += 256) {
    const int q = i - hmax;
    c64 r = {0.0, 0.0};
    if (q >= -h && q <= h) {
      r = response64((double)q, z);
      e += r.re * r.re + r.im * r.im;
    }
    row[i] = r;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double inv = 1.0 / sqrt(red[0]);
  for (int i = threadIdx.x; i < K; i += 256) row[i] = c64scale(c64conj(row[i]), inv);
}

template <int SDT>
__global__ __launch_bounds__(256) void k_template_spectra(const c64* __restrict__ taps, const c64* __restrict__ tab,
                                                          int hmax, int L, void* out, int shift) {
  using SS = Store<SDT>;
  const int j = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= L) return;
  const int K = 2 * hmax + 1;
  const c64* row = taps + (size_t)j * K;
  c64 acc = {0.0, 0.0};
  for (int i = 0; i < K; ++i) {
    const c64 t = row[i];
    if (t.re == 0.0 && t.im == 0.0) continue;
    const int q = i - hmax;
    const int idx = (int)(((int64_t)k * q) & (int64_t)(L - 1));  // L is a power of two
    acc = c64add(acc, c64mul(t, tab[idx]));
  }
  const double s = ldexp(1.0, shift) / (double)L;
  typename SS::cplx_t* o = reinterpret_cast<typename SS::cplx_t*>(out) + (size_t)j * L;
  o[k] = SS::pack(c32{(float)(acc.re * s), (float)(acc.im * s)});
}

hipError_t launch_exp_table(int L, c64* tab, hipStream_t st) {
  hipLaunchKernelGGL(k_exp_table, dim3((L + 255) / 256), dim3(256), 0, st, tab, L);
  return hipGetLastError();
}

hipError_t launch_template_taps(double z_min, double z_step, int Z, int margin, int hmax, c64* taps,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_template_taps, dim3(Z), dim3(256), 0, st, z_min, z_step, margin, hmax, taps);
  return hipGetLastError();
}

hipError_t launch_template_spectra(int sdt, const c64* taps, const c64* tab, int Z, int hmax, int L, void* out,
                                   hipStream_t st, int shift) {
  const dim3 g((L + 255) / 256, Z);
  switch (sdt) {
    case FDAS_F32: hipLaunchKernelGGL((k_template_spectra<FDAS_F32>), g, dim3(256), 0, st, taps, tab, hmax, L, out, shift); break;
    case FDAS_BF16: hipLaunchKernelGGL((k_template_spectra<FDAS_BF16>), g, dim3(256), 0, st, taps, tab, hmax, L, out, shift); break;
    case FDAS_F16: hipLaunchKernelGGL((k_template_spectra<FDAS_F16>), g, dim3(256), 0, st, taps, tab, hmax, L, out, shift); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fdas
