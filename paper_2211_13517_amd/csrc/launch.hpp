// Host-side launchers of the FDAS kernels (one definition per kernel file).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "fresnel.hpp"

namespace fdas {

// One series of a batch, as the kernels see it.
struct SeriesDesc {
  int64_t in_off;      // first float32 sample in the input
  int64_t spec_off;    // first complex bin in the packed spectrum (and FFT scratch)
  int64_t plane_off;   // first element of the series' power plane (= Z * spec_off)
  int64_t tile_begin;  // first convolution tile of the series
  int32_t nbins;       // N/2
  int32_t nseg;        // overlap-save segments ceil(nbins / U)
};

// Twiddle tables of the FFT sizes the library builds, concatenated; offsets
// are in complex entries.
struct TwiddleSet {
  int off[14];  // indexed by log2(L)
};
int twiddle_table_size(int L);             // entries, 0 if the size is not built
void twiddle_table_fill(int L, c32* dst);  // forward-sign twiddles of FftShape<L, P(L)>
int fft_points_per_thread(int L);

}  // namespace fdas
#include "fft.hpp"
namespace fdas {
// FFT shapes the library builds: L points, P per thread, pass radix R.
template <int L> struct ShapeOf;
template <> struct ShapeOf<256> { using type = FftShape<256, 4, 4>; };
template <> struct ShapeOf<512> { using type = FftShape<512, 8, 8>; };
template <> struct ShapeOf<1024> { using type = FftShape<1024, 16, 16>; };
template <> struct ShapeOf<2048> { using type = FftShape<2048, 32, 16>; };
template <> struct ShapeOf<4096> { using type = FftShape<4096, 16, 16>; };
template <> struct ShapeOf<8192> { using type = FftShape<8192, 16, 16>; };

// spectrum
hipError_t launch_rfft_columns(int M1, int M2, const float* x, const SeriesDesc* desc, const int32_t* list,
                               int nlist, c32* Y, const c32* tw, hipStream_t st);
hipError_t launch_rfft_rows(int M1, int M2, const SeriesDesc* desc, const int32_t* list, int nlist,
                            const c32* Y, c32* Zb, const c32* tw, hipStream_t st);
hipError_t launch_unpack_normalise(int sdt, int M, int B, int mode, double var_scale, const SeriesDesc* desc,
                                   const int32_t* list, int nlist, const c32* Zb, void* spec, int32_t* status,
                                   hipStream_t st);

// templates
hipError_t launch_exp_table(int L, c64* tab, hipStream_t st);
hipError_t launch_template_taps(double z_min, double z_step, int Z, int margin, int hmax, c64* taps,
                                hipStream_t st);
// out[j][k] = T_j[k] 2^shift in dtype sdt (shift = 0 for the stored bank)
hipError_t launch_template_spectra(int sdt, const c64* taps, const c64* tab, int Z, int hmax, int L, void* out,
                                   hipStream_t st, int shift = 0);

// Column maxima: a plane buffer holds the batch's plane values, then for
// every row of every series the maximum of each run of kPlaneMaxCols columns
// (series i's maxima from element plane_off / kPlaneMaxCols of that section).
constexpr int kPlaneMaxCols = 8;

// convolution
struct ConvArgs {
  const void* spec;        // packed normalised spectrum, store dtype
  const void* tspec;       // template spectra [Z][L], store dtype
  const void* tspec16;     // FP16 matrix-core path: the spectra times 2^10 as FP16 pairs
  void* plane;             // packed planes, plane dtype
  void* maxima;            // their column maxima, plane dtype
  const SeriesDesc* desc;  // per series
  const c32* tw;           // twiddle table of size L
  int64_t n_tiles;         // sum over series of nseg * G
  // seg_margin: FFT index of a segment's first output (>= h_max; it and U
  // are multiples of the bins per column maximum)
  int32_t n_series, Z, G, U, seg_margin;
  // bound on |T_j[k]| of the template spectra, sqrt(2 h_max + 1) / L (unit-energy
  // taps, the inverse FFT's 1/L folded in): sets the FP16 inverse FFT's scaling
  float tbound;
};
// interbin: also write the half-bin power between each output and the next
// R: radix of the convolution FFT's passes (16; 8 or 4 at L = 1024)
hipError_t launch_conv(int L, int R, int sdt, int pdt, bool interbin, const ConvArgs& a, int grid, hipStream_t st);
int conv_waves_per_block(int L);
// whether the convolution's inverse FFTs run in FP16 on the matrix cores
bool conv_uses_mfma(int L, int R, int pdt, bool interbin);
constexpr int kTspec16Shift = 10;  // FP16 template spectra are stored times 2^10
int conv_blocks_per_cu(int L, int R, int sdt, int pdt, bool interbin);  // resident blocks per CU (occupancy query)
bool conv_radix_supported(int L, int R);
int conv_twiddle_size(int L, int R);           // entries of the convolution FFT's twiddle table
void conv_twiddle_fill(int L, int R, c32* dst);

hipError_t launch_plane_maxima(int pdt, const void* plane, void* maxima, const SeriesDesc* desc, int n_series, int Z,
                               int res_shift, int64_t max_bins, int cus, hipStream_t st);

// harmonic sums
struct HarmArgs {
  const void* plane;
  const void* maxima;  // column maxima of the plane
  const SeriesDesc* desc;
  fdas_candidate* cands;
  unsigned long long* count;
  int64_t capacity;
  float tau[5];
  double z_min, z_step;
  // plane columns: a series of nbins bins has nbins << res_shift columns
  // (res_shift 1 on a half-bin plane); r_lo, hmax and max_bins are given in
  // columns
  int32_t n_series, Z, j0, n_harm, r_lo, hmax;
  int32_t res_shift;
  int32_t max_bins;     // longest series in the batch (sets the tile grid)
  int32_t series_base;  // added to the batch index in the records' series field
};
hipError_t launch_harmonic_sum(int pdt, const HarmArgs& a, hipStream_t st);

// off-grid power and refinement
hipError_t launch_rz_power(int sdt, const void* spec, int64_t nb, const double* r, const double* z, int64_t n, int margin,
                           double* p, c64* y, hipStream_t st);
// acc: 2 nb fixed-point words; max_bits, scale: one word each (set here)
hipError_t launch_rz_grad(int sdt, const void* spec, int64_t nb, const double* r, const double* z, const c64* y,
                          const double* gp, int64_t n, int margin, double* gr, double* gz, float* gspec,
                          unsigned long long* acc, unsigned long long* max_bits, double* scale, int32_t* status,
                          hipStream_t st);
hipError_t launch_refine(int sdt, const void* spec, int64_t nb, double* r, double* z, int64_t n, int iters, int margin,
                         double* p_final, hipStream_t st);
hipError_t launch_refine_harmonics(int sdt, const void* spec, int64_t nb, double* r, double* z, const int32_t* harm,
                                   int64_t n, int iters, int margin, double* p_final, hipStream_t st);

// candidate clustering
constexpr int64_t kClusterStaticMaxRecords = int64_t(1) << 20;  // capacity of the static-scratch variant
int64_t cluster_scratch_bytes(int64_t capacity);
// device address of the static clustering scratch on `device` (looked up once per device)
hipError_t cluster_static_scratch(int device, void** ptr);
hipError_t launch_cluster(const fdas_candidate* c, const unsigned long long* count, int64_t capacity, int rr, int rj,
                          void* table, uint8_t* keep, int cus, hipStream_t st);

// small helpers (fill kernels are graph-capture safe, unlike memset nodes)
hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t value, hipStream_t st);
hipError_t launch_fill_noise(void* spec, int sdt, int64_t nbins, uint64_t seed, hipStream_t st);

// self-test hook: batched complex FFT of size L
hipError_t launch_test_fft(int L, int dir, const c32* in, c32* out, int64_t batch, const c32* tw, hipStream_t st);

}  // namespace fdas
