// C ABI of the FDAS library: plan validation, thresholds, workspace layout,
// batch descriptors and kernel launches.  No device memory is allocated here:
// the caller binds one workspace and passes every data buffer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "launch.hpp"

using namespace fdas;

namespace {

constexpr int kFftSizes[] = {256, 512, 1024, 2048, 4096, 8192};
constexpr int kNumFftSizes = 6;

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }
bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
int log2i(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}
int cbytes(int dt) { return dt == FDAS_F32 ? 8 : 4; }
int rbytes(int dt) { return dt == FDAS_F32 ? 4 : 2; }

thread_local std::string g_plan_error;

// ln P(Gamma(h,1) > x) for integer h (closed form of the upper incomplete gamma)
double log_tail_gamma_host(double x, int h) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < h; ++k) {
    term *= x / k;
    sum += term;
  }
  return -x + std::log(sum);
}

// tau with P(Gamma(h,1) > tau) = P(N(0,1) > sigma), by bisection in log space.
double threshold_for(int h, double sigma) {
  const double target = std::log(0.5 * std::erfc(sigma / std::sqrt(2.0)));
  double lo = 0.0, hi = 10.0;
  while (log_tail_gamma_host(hi, h) > target) hi *= 2.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (log_tail_gamma_host(mid, h) > target) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

struct LengthClass {
  int64_t nsamp;
  int M1, M2;
  int list_off, count;
};

}  // namespace

struct fdas_plan_s {
  fdas_params p{};
  int device = 0;
  hipStream_t stream = nullptr;
  int Z = 0, j0 = 0, hmax = 0, K = 0, L = 0, U = 0, seg_margin = 0, nstages = 0;
  int res = 1;  // plane columns per bin: 2 on a half-bin plane
  double tau[5] = {0, 0, 0, 0, 0};
  int64_t max_batch = 0;
  int max_series = 0;
  int cu_count = 0;
  // workspace layout (byte offsets)
  char* ws = nullptr;
  int64_t ws_bytes = 0;
  int64_t off_status = 0, off_tw[kNumFftSizes] = {}, off_exptab = 0, off_taps = 0, off_tspec = 0, off_desc = 0,
          off_lists = 0, off_Y = 0, off_Zb = 0, off_spec = 0, off_tw_conv = 0, off_tspec16 = 0, total = 0;
  bool mfma = false;  // inverse FFTs in FP16 on the matrix cores (FP16 template copy in the workspace)
  bool templates_ready = false;
  std::string err;
  // current batch
  std::vector<SeriesDesc> desc;
  std::vector<int32_t> lists;
  std::vector<LengthClass> classes;
  std::vector<int64_t> key_offsets, key_lengths;
  int64_t total_bins = 0, n_tiles = 0, max_bins = 0;
  int G = 1;
  bool batch_valid = false;
  SeriesDesc* h_desc_pinned = nullptr;
  int32_t* h_lists_pinned = nullptr;
  // captured search graph and the arguments it was captured for
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<uintptr_t> graph_key;
  hipError_t static_table_status = hipSuccess;  // look-up of the static clustering table at plan time
  // plane buffers whose column maxima this plan wrote (convolution or
  // fdas_plane_maxima), with the batch they were written for: the harmonic
  // sum reads the maxima where its own batch puts them, so it refuses a
  // buffer and batch that no maxima were written for
  struct MaximaWrite {
    uintptr_t plane = 0;
    uint64_t batch = 0;
  };
  MaximaWrite maxima_writes[8];
  int maxima_next = 0;

  fdas_status fail(fdas_status s, const std::string& m) {
    err = m;
    return s;
  }
  const c32* tw(int L_) const {
    for (int i = 0; i < kNumFftSizes; ++i)
      if (kFftSizes[i] == L_) return reinterpret_cast<const c32*>(ws + off_tw[i]);
    return nullptr;
  }
};

// Release calls on cleanup paths ((void) below) drop their status on purpose:
// a failed release leaves nothing for the caller to undo.
static fdas_status hip_fail(fdas_plan_t pl, hipError_t e, const char* what) {
  return pl->fail(FDAS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

extern "C" {

fdas_status fdas_default_params(fdas_params* p) {
  if (!p) return FDAS_ERR_ARG;
  std::memset(p, 0, sizeof(*p));
  p->n_samples = int64_t(1) << 23;
  p->tsamp = 64e-6;
  p->z_min = -96.0;
  p->z_max = 96.0;
  p->z_step = 1.0;
  p->n_harmonics = 16;
  p->kernel_margin = 16;
  p->segment_len = 0;
  p->store_dtype = FDAS_F32;
  p->plane_dtype = FDAS_F32;
  p->norm = FDAS_NORM_MEDIAN;
  p->norm_block = 2048;
  p->noise_var = 1.0;
  p->sigma_threshold = 6.0;
  return FDAS_OK;
}

fdas_status fdas_plan(const fdas_params* params, int device, void* hip_stream, fdas_plan_t* out) {
  if (out) *out = nullptr;
  auto bad = [](const std::string& m) {
    g_plan_error = m;
    return FDAS_ERR_ARG;
  };
  if (!params || !out) return bad("params and out must be non-NULL");
  const fdas_params& p = *params;
  if (!is_pow2(p.n_samples) || p.n_samples < (1 << 17) || p.n_samples > (1 << 23))
    return bad("n_samples must be a power of two in [2^17, 2^23]");
  const int64_t mb = p.max_batch_samples ? p.max_batch_samples : p.n_samples;
  if (mb < p.n_samples) return bad("max_batch_samples must be 0 or >= n_samples");
  if (!(p.z_step > 0) || !(p.z_max >= 0) || std::fabs(p.z_min + p.z_max) > 1e-9 * std::max(1.0, p.z_max))
    return bad("z grid must be symmetric (z_min = -z_max) with z_step > 0");
  const double zn = (p.z_max - p.z_min) / p.z_step;
  if (std::fabs(zn - std::round(zn)) > 1e-9 || std::fabs(p.z_max / p.z_step - std::round(p.z_max / p.z_step)) > 1e-9)
    return bad("z_max / z_step must be an integer");
  const int Z = (int)std::llround(zn) + 1;
  if (Z > 4096) return bad("at most 4096 acceleration trials");
  if (!(p.n_harmonics == 1 || p.n_harmonics == 2 || p.n_harmonics == 4 || p.n_harmonics == 8 || p.n_harmonics == 16))
    return bad("n_harmonics must be 1, 2, 4, 8 or 16");
  const int margin = p.kernel_margin ? p.kernel_margin : 16;
  if (margin < 1 || margin > 256) return bad("kernel_margin must be in [1, 256]");
  const int hmax = (int)std::ceil(p.z_max / 2.0) + margin;
  const int L = p.segment_len ? p.segment_len : 1024;
  if (!(L == 1024 || L == 2048 || L == 4096 || L == 8192)) return bad("segment_len must be 0, 1024, 2048, 4096 or 8192");
  if (4 * hmax > L) return bad("segment_len must be at least 4 * h_max (h_max = ceil(z_max/2) + margin)");
  for (int dt : {p.store_dtype, p.plane_dtype})
    if (dt < FDAS_F32 || dt > FDAS_F16) return bad("store_dtype / plane_dtype must be FDAS_F32, FDAS_BF16 or FDAS_F16");
  if (p.norm < FDAS_NORM_NONE || p.norm > FDAS_NORM_REDNOISE) return bad("unknown norm");
  const int B = p.norm_block ? p.norm_block : 2048;
  if (!is_pow2(B) || B < 256 || B > 4096) return bad("norm_block must be a power of two in [256, 4096]");
  if (p.norm == FDAS_NORM_VARIANCE && !(p.noise_var > 0)) return bad("noise_var must be > 0");
  const double sig = p.sigma_threshold ? p.sigma_threshold : 6.0;
  if (!(sig > 0 && sig < 30)) return bad("sigma_threshold must be in (0, 30)");
  if (p.r_lo < 0) return bad("r_lo must be >= 0");
  if (p.templates_per_tile < 0) return bad("templates_per_tile must be >= 0");
  if (p.interbin != 0 && p.interbin != 1) return bad("interbin must be 0 or 1");
  const int radix = p.fft_radix ? p.fft_radix : 16;
  if (!conv_radix_supported(L, radix)) return bad("fft_radix must be 0 or 16 (8 and 4 also at segment_len 1024)");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return bad("invalid device");

  fdas_plan_s* pl = new (std::nothrow) fdas_plan_s();
  if (!pl) return bad("out of host memory");
  pl->p = p;
  pl->p.max_batch_samples = mb;
  pl->p.kernel_margin = margin;
  pl->p.segment_len = L;
  pl->p.fft_radix = radix;
  pl->p.norm_block = B;
  pl->p.sigma_threshold = sig;
  pl->device = device;
  pl->stream = (hipStream_t)hip_stream;
  pl->Z = Z;
  pl->j0 = (int)std::llround(-p.z_min / p.z_step);
  pl->hmax = hmax;
  pl->K = 2 * hmax + 1;
  pl->L = L;
  // a half-bin plane needs y one past the last output of each segment
  pl->res = p.interbin ? 2 : 1;
  // Segments put their first output seg_margin >= h_max points into the
  // FFT and keep U outputs, both multiples of the bins per column maximum,
  // so every run of 8 plane columns lies in one segment and the convolution
  // writes its maximum (a half-bin plane needs y one past each segment's
  // last output as well).
  const int run = kPlaneMaxCols / pl->res;
  pl->seg_margin = (hmax + run - 1) / run * run;
  pl->U = (L - 2 * pl->seg_margin - (p.interbin ? 1 : 0)) / run * run;
  pl->nstages = log2i(p.n_harmonics) + 1;
  if (pl->p.r_lo == 0) pl->p.r_lo = hmax;
  for (int i = 0; i < pl->nstages; ++i) pl->tau[i] = threshold_for(1 << i, sig);
  pl->max_batch = mb;
  pl->max_series = (int)(mb / (p.n_samples / 4));
  if (hipDeviceGetAttribute(&pl->cu_count, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      pl->cu_count <= 0) {
    delete pl;
    return bad("could not query the device's compute-unit count");
  }
  // set-up of the allocation-free clustering: the static table's address on
  // this device (looked up once per device; a failure is reported by that
  // entry point, the others do not need it)
  void* unused_table = nullptr;
  pl->static_table_status = cluster_static_scratch(device, &unused_table);

  // workspace layout
  int64_t o = 0;
  pl->off_status = o;
  o += 256;
  for (int i = 0; i < kNumFftSizes; ++i) {
    pl->off_tw[i] = o;
    o = align256(o + (int64_t)twiddle_table_size(kFftSizes[i]) * (int64_t)sizeof(c32));
  }
  pl->off_tw_conv = o;  // the convolution FFT's table when its radix is not 16
  o = align256(o + (radix == 16 ? 0 : (int64_t)conv_twiddle_size(L, radix)) * (int64_t)sizeof(c32));
  pl->off_exptab = o;
  o = align256(o + (int64_t)L * 16);
  pl->off_taps = o;
  o = align256(o + (int64_t)Z * pl->K * 16);
  pl->off_tspec = o;
  o = align256(o + (int64_t)Z * L * cbytes(p.store_dtype));
  pl->mfma = conv_uses_mfma(L, radix, p.plane_dtype, p.interbin != 0);
  pl->off_tspec16 = o;
  o = align256(o + (pl->mfma ? (int64_t)Z * L * 4 : 0));
  pl->off_desc = o;
  o = align256(o + (int64_t)pl->max_series * (int64_t)sizeof(SeriesDesc));
  pl->off_lists = o;
  o = align256(o + (int64_t)pl->max_series * 4);
  pl->off_Y = o;
  o = align256(o + mb / 2 * 8);
  pl->off_Zb = o;
  o = align256(o + mb / 2 * 8);
  pl->off_spec = o;
  o = align256(o + mb / 2 * cbytes(p.store_dtype));
  pl->total = o;

  if (hipHostMalloc((void**)&pl->h_desc_pinned, sizeof(SeriesDesc) * pl->max_series) != hipSuccess ||
      hipHostMalloc((void**)&pl->h_lists_pinned, sizeof(int32_t) * pl->max_series) != hipSuccess) {
    if (pl->h_desc_pinned) (void)hipHostFree(pl->h_desc_pinned);
    delete pl;
    return bad("could not allocate pinned host staging");
  }
  *out = pl;
  return FDAS_OK;
}

fdas_status fdas_query(fdas_plan_t pl, int64_t* ws, int32_t* L, int32_t* hmax, int32_t* Z) {
  if (!pl) return FDAS_ERR_ARG;
  if (ws) *ws = pl->total;
  if (L) *L = pl->L;
  if (hmax) *hmax = pl->hmax;
  if (Z) *Z = pl->Z;
  return FDAS_OK;
}

fdas_status fdas_set_workspace(fdas_plan_t pl, void* dev_ptr, int64_t bytes) {
  if (!pl) return FDAS_ERR_ARG;
  if (!dev_ptr || bytes < pl->total) return pl->fail(FDAS_ERR_NOMEM, "workspace missing or smaller than fdas_query's size");
  if (((uintptr_t)dev_ptr) & 255) return pl->fail(FDAS_ERR_ARG, "workspace must be 256-byte aligned");
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  // a captured search graph reads descriptors, templates and the status word
  // of the old workspace: it is dropped with the binding
  if (pl->graph_exec) (void)hipGraphExecDestroy(pl->graph_exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  pl->graph_exec = nullptr;
  pl->graph = nullptr;
  pl->graph_key.clear();
  pl->ws = (char*)dev_ptr;
  pl->ws_bytes = bytes;
  pl->templates_ready = false;
  pl->batch_valid = false;
  std::vector<c32> tab;
  for (int i = 0; i < kNumFftSizes; ++i) {
    const int n = twiddle_table_size(kFftSizes[i]);
    tab.assign(n, c32{0.f, 0.f});
    twiddle_table_fill(kFftSizes[i], tab.data());
    e = hipMemcpyAsync(pl->ws + pl->off_tw[i], tab.data(), n * sizeof(c32), hipMemcpyHostToDevice, pl->stream);
    if (e != hipSuccess) return hip_fail(pl, e, "twiddle upload");
    e = hipStreamSynchronize(pl->stream);
    if (e != hipSuccess) return hip_fail(pl, e, "twiddle upload");
  }
  if (pl->p.fft_radix != 16) {
    const int n = conv_twiddle_size(pl->L, pl->p.fft_radix);
    tab.assign(n, c32{0.f, 0.f});
    conv_twiddle_fill(pl->L, pl->p.fft_radix, tab.data());
    e = hipMemcpyAsync(pl->ws + pl->off_tw_conv, tab.data(), n * sizeof(c32), hipMemcpyHostToDevice, pl->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
    if (e != hipSuccess) return hip_fail(pl, e, "twiddle upload");
  }
  e = hipMemsetAsync(pl->ws + pl->off_status, 0, 256, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "status clear");
  e = hipStreamSynchronize(pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "status clear");
  return FDAS_OK;
}

fdas_status fdas_make_templates(fdas_plan_t pl) {
  if (!pl) return FDAS_ERR_ARG;
  if (!pl->ws) return pl->fail(FDAS_ERR_STATE, "no workspace bound");
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  c64* tab = reinterpret_cast<c64*>(pl->ws + pl->off_exptab);
  c64* taps = reinterpret_cast<c64*>(pl->ws + pl->off_taps);
  if ((e = launch_exp_table(pl->L, tab, pl->stream)) != hipSuccess) return hip_fail(pl, e, "exp table");
  if ((e = launch_template_taps(pl->p.z_min, pl->p.z_step, pl->Z, pl->p.kernel_margin, pl->hmax, taps, pl->stream)) !=
      hipSuccess)
    return hip_fail(pl, e, "template taps");
  if ((e = launch_template_spectra(pl->p.store_dtype, taps, tab, pl->Z, pl->hmax, pl->L, pl->ws + pl->off_tspec,
                                   pl->stream)) != hipSuccess)
    return hip_fail(pl, e, "template spectra");
  if (pl->mfma && (e = launch_template_spectra(FDAS_F16, taps, tab, pl->Z, pl->hmax, pl->L, pl->ws + pl->off_tspec16,
                                               pl->stream, kTspec16Shift)) != hipSuccess)
    return hip_fail(pl, e, "template spectra (FP16)");
  pl->templates_ready = true;
  return FDAS_OK;
}

}  // extern "C"

// Validates a batch and uploads its descriptors when it differs from the last one.
static fdas_status set_batch(fdas_plan_t pl, const int64_t* offsets, const int64_t* lengths, int32_t n) {
  if (!lengths || n <= 0) return pl->fail(FDAS_ERR_ARG, "need n_series > 0 and a lengths array");
  if (n > pl->max_series) return pl->fail(FDAS_ERR_ARG, "more series than max_batch_samples allows");
  const int64_t N = pl->p.n_samples;
  int64_t tot = 0;
  for (int i = 0; i < n; ++i) {
    const int64_t len = lengths[i];
    if (!(len == N || len == N / 2 || len == N / 4) || len < (1 << 17))
      return pl->fail(FDAS_ERR_ARG, "series lengths must be n_samples, n_samples/2 or n_samples/4 (and >= 2^17)");
    if (offsets && (offsets[i] < 0 || (offsets[i] & 1)))
      return pl->fail(FDAS_ERR_ARG, "series offsets must be even and non-negative");
    tot += len;
  }
  if (tot > pl->max_batch) return pl->fail(FDAS_ERR_ARG, "sum of lengths exceeds max_batch_samples");
  std::vector<int64_t> ko(offsets ? offsets : lengths, (offsets ? offsets : lengths) + n), kl(lengths, lengths + n);
  if (!offsets) std::fill(ko.begin(), ko.end(), -1);
  if (pl->batch_valid && ko == pl->key_offsets && kl == pl->key_lengths) return FDAS_OK;

  // segments and template groups
  int64_t nseg_total = 0;
  for (int i = 0; i < n; ++i) nseg_total += (lengths[i] / 2 + pl->U - 1) / pl->U;
  int G;
  if (pl->p.templates_per_tile > 0) {
    G = (pl->Z + pl->p.templates_per_tile - 1) / pl->p.templates_per_tile;
  } else {
    // A tile costs Z/G inverse FFTs plus its segment's forward FFT.  The
    // T = nseg * G tiles are dealt evenly over the CUs, and the tile owners
    // resident on one CU (waves, or blocks for the multi-wave FFTs) share its
    // throughput, so a CU with T_cu tiles and S owners takes about
    // max(1, T_cu / S) tile times: choose the G that minimises that.  (A
    // model by rounds of the slowest owner over-weights a partial last round
    // and picked groups of ~28 templates, 5 % slower at N = 2^23 than the
    // 65-193 this one picks.)
    const int per_cu = std::max(1, conv_blocks_per_cu(pl->L, pl->p.fft_radix, pl->p.store_dtype, pl->p.plane_dtype,
                                                      pl->p.interbin != 0));
    const double S = (double)per_cu * (pl->L == 1024 ? conv_waves_per_block(pl->L) : 1);
    double best = 1e300;
    G = 1;
    for (int g = 1; g <= pl->Z; ++g) {
      const double t_cu = std::ceil((double)nseg_total * g / (double)pl->cu_count);
      const double t = std::max(1.0, t_cu / S) * ((double)pl->Z / g + 1.0);
      if (t < best - 1e-9) {
        best = t;
        G = g;
      }
    }
  }
  pl->G = G;
  pl->desc.resize(n);
  int64_t spec = 0, tiles = 0, maxb = 0;
  for (int i = 0; i < n; ++i) {
    SeriesDesc& d = pl->desc[i];
    d.in_off = offsets ? offsets[i] : 0;
    d.spec_off = spec;
    d.plane_off = spec * pl->Z * pl->res;
    d.nbins = (int32_t)(lengths[i] / 2);
    d.nseg = (int32_t)((d.nbins + pl->U - 1) / pl->U);
    d.tile_begin = tiles;
    tiles += (int64_t)d.nseg * G;
    spec += d.nbins;
    maxb = std::max<int64_t>(maxb, d.nbins);
  }
  pl->total_bins = spec;
  pl->n_tiles = tiles;
  pl->max_bins = maxb;
  // group series by length for the FFT launches
  pl->classes.clear();
  pl->lists.clear();
  for (int64_t len : {N, N / 2, N / 4}) {
    LengthClass c;
    c.nsamp = len;
    const int lm = log2i(len / 2);
    c.M1 = 1 << ((lm + 1) / 2);
    c.M2 = 1 << (lm / 2);
    c.list_off = (int)pl->lists.size();
    for (int i = 0; i < n; ++i)
      if (lengths[i] == len) pl->lists.push_back(i);
    c.count = (int)pl->lists.size() - c.list_off;
    if (c.count) pl->classes.push_back(c);
  }
  hipError_t e = hipStreamSynchronize(pl->stream);  // staging buffers may still feed a copy
  if (e != hipSuccess) return hip_fail(pl, e, "stream sync");
  std::memcpy(pl->h_desc_pinned, pl->desc.data(), n * sizeof(SeriesDesc));
  std::memcpy(pl->h_lists_pinned, pl->lists.data(), pl->lists.size() * sizeof(int32_t));
  e = hipMemcpyAsync(pl->ws + pl->off_desc, pl->h_desc_pinned, n * sizeof(SeriesDesc), hipMemcpyHostToDevice, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "descriptor upload");
  e = hipMemcpyAsync(pl->ws + pl->off_lists, pl->h_lists_pinned, pl->lists.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "descriptor upload");
  pl->key_offsets = ko;
  pl->key_lengths = kl;
  pl->batch_valid = true;
  return FDAS_OK;
}

// Batches that only need the per-series lengths (plane and spectrum layout)
// reuse the current descriptors when the lengths match.
static fdas_status ensure_lengths(fdas_plan_t pl, const int64_t* lengths, int32_t n) {
  if (lengths && n > 0 && pl->batch_valid && pl->key_lengths.size() == (size_t)n &&
      std::equal(pl->key_lengths.begin(), pl->key_lengths.end(), lengths))
    return FDAS_OK;
  return set_batch(pl, nullptr, lengths, n);
}

static fdas_status run_spectrum(fdas_plan_t pl, const float* series, void* spec_out) {
  const SeriesDesc* desc = reinterpret_cast<const SeriesDesc*>(pl->ws + pl->off_desc);
  const int32_t* lists = reinterpret_cast<const int32_t*>(pl->ws + pl->off_lists);
  c32* Y = reinterpret_cast<c32*>(pl->ws + pl->off_Y);
  c32* Zb = reinterpret_cast<c32*>(pl->ws + pl->off_Zb);
  int32_t* status = reinterpret_cast<int32_t*>(pl->ws + pl->off_status);
  hipError_t e;
  for (const LengthClass& c : pl->classes) {
    const int32_t* l = lists + c.list_off;
    if ((e = launch_rfft_columns(c.M1, c.M2, series, desc, l, c.count, Y, pl->tw(c.M1), pl->stream)) != hipSuccess)
      return hip_fail(pl, e, "rfft columns");
    if ((e = launch_rfft_rows(c.M1, c.M2, desc, l, c.count, Y, Zb, pl->tw(c.M2), pl->stream)) != hipSuccess)
      return hip_fail(pl, e, "rfft rows");
    const int M = (int)(c.nsamp / 2);
    double vs = 1.0;
    if (pl->p.norm == FDAS_NORM_VARIANCE) vs = 1.0 / std::sqrt((double)c.nsamp * pl->p.noise_var);
    if ((e = launch_unpack_normalise(pl->p.store_dtype, M, pl->p.norm_block, pl->p.norm, vs, desc, l, c.count, Zb,
                                     spec_out, status, pl->stream)) != hipSuccess)
      return hip_fail(pl, e, "unpack/normalise");
  }
  return FDAS_OK;
}

// The harmonic sum copies plane strips with 16-byte loads from the plane's
// base: a plane that is only element-aligned is refused before any launch.
static fdas_status check_harm_plane(fdas_plan_t pl, const void* plane) {
  if (((uintptr_t)plane) & 15) return pl->fail(FDAS_ERR_ARG, "plane must be 16-byte aligned for the harmonic sum");
  return FDAS_OK;
}

// Bytes of the packed plane values of `bins` bins in all, and of a plane
// buffer for them: the values, then their column maxima.
static int64_t plane_data_bytes(fdas_plan_t pl, int64_t bins) {
  return bins * pl->Z * pl->res * rbytes(pl->p.plane_dtype);
}
static int64_t plane_buffer_bytes(fdas_plan_t pl, int64_t bins) {
  return plane_data_bytes(pl, bins) + plane_data_bytes(pl, bins) / kPlaneMaxCols;
}
static int64_t plane_need(fdas_plan_t pl) { return plane_buffer_bytes(pl, pl->total_bins); }

// FNV-1a over the current batch's lengths (the plane layout they give).
static uint64_t batch_key(fdas_plan_t pl) {
  uint64_t h = 1469598103934665603ull;
  for (int64_t v : pl->key_lengths)
    for (int b = 0; b < 8; ++b) {
      h ^= (uint64_t)((v >> (8 * b)) & 0xff);
      h *= 1099511628211ull;
    }
  return h ^ (uint64_t)pl->key_lengths.size();
}
static void note_maxima_written(fdas_plan_t pl, const void* plane) {
  const uint64_t k = batch_key(pl);
  for (auto& w : pl->maxima_writes)
    if (w.plane == (uintptr_t)plane && w.batch == k) return;
  pl->maxima_writes[pl->maxima_next] = {(uintptr_t)plane, k};
  pl->maxima_next = (pl->maxima_next + 1) % 8;
}
static bool maxima_written(fdas_plan_t pl, const void* plane) {
  const uint64_t k = batch_key(pl);
  for (const auto& w : pl->maxima_writes)
    if (w.plane == (uintptr_t)plane && w.batch == k) return true;
  return false;
}
static void* plane_maxima(fdas_plan_t pl, const void* plane) {
  return const_cast<char*>(reinterpret_cast<const char*>(plane)) + plane_data_bytes(pl, pl->total_bins);
}

// Harmonic-sum arguments for the current batch; on a half-bin plane the bin
// limits are given in half bins.
static HarmArgs harm_args(fdas_plan_t pl, const void* plane, fdas_candidate* cands, int64_t capacity,
                          int64_t* d_count) {
  HarmArgs a;
  a.plane = plane;
  a.maxima = plane_maxima(pl, plane);
  a.desc = reinterpret_cast<const SeriesDesc*>(pl->ws + pl->off_desc);
  a.cands = cands;
  a.count = reinterpret_cast<unsigned long long*>(d_count);
  a.capacity = capacity;
  for (int i = 0; i < 5; ++i) a.tau[i] = i < pl->nstages ? (float)pl->tau[i] : 0.f;
  a.z_min = pl->p.z_min;
  a.z_step = pl->p.z_step;
  a.n_series = (int)pl->desc.size();
  a.Z = pl->Z;
  a.j0 = pl->j0;
  a.n_harm = pl->p.n_harmonics;
  a.r_lo = pl->p.r_lo * pl->res;
  a.hmax = pl->hmax * pl->res;
  a.res_shift = pl->res == 2 ? 1 : 0;
  a.max_bins = (int32_t)(pl->max_bins * pl->res);
  a.series_base = 0;
  return a;
}

static fdas_status run_conv(fdas_plan_t pl, const void* spec, void* plane, int64_t plane_bytes) {
  if (!pl->templates_ready) return pl->fail(FDAS_ERR_STATE, "fdas_make_templates has not run");
  const int64_t need = plane_need(pl);
  if (!plane || plane_bytes < need) return pl->fail(FDAS_ERR_NOMEM, "plane buffer missing or too small");
  // (bin, half-bin) pairs are written as one store, the maxima read in 16-byte pieces
  if (((uintptr_t)plane) & 15) return pl->fail(FDAS_ERR_ARG, "plane buffers must be 16-byte aligned");
  ConvArgs a;
  a.spec = spec;
  a.tspec = pl->ws + pl->off_tspec;
  a.tspec16 = pl->ws + pl->off_tspec16;
  a.plane = plane;
  a.maxima = plane_maxima(pl, plane);
  a.desc = reinterpret_cast<const SeriesDesc*>(pl->ws + pl->off_desc);
  a.tw = pl->p.fft_radix == 16 ? pl->tw(pl->L) : reinterpret_cast<const c32*>(pl->ws + pl->off_tw_conv);
  a.n_tiles = pl->n_tiles;
  a.n_series = (int)pl->desc.size();
  a.Z = pl->Z;
  a.G = pl->G;
  a.U = pl->U;
  a.seg_margin = pl->seg_margin;
  a.tbound = (float)(std::sqrt(2.0 * pl->hmax + 1.0) / pl->L);
  // The grid is exactly what is resident at once: tiles are dealt
  // round-robin, so a block that had to wait for a slot would finish last.
  const int per_block = conv_waves_per_block(pl->L);
  const int per_cu = std::max(1, conv_blocks_per_cu(pl->L, pl->p.fft_radix, pl->p.store_dtype, pl->p.plane_dtype,
                                                    pl->p.interbin != 0));
  const int64_t blocks_needed = pl->L == 1024 ? (pl->n_tiles + per_block - 1) / per_block : pl->n_tiles;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(blocks_needed, (int64_t)pl->cu_count * per_cu));
  hipError_t e =
      launch_conv(pl->L, pl->p.fft_radix, pl->p.store_dtype, pl->p.plane_dtype, pl->p.interbin != 0, a, grid, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "convolve");
  note_maxima_written(pl, plane);
  return FDAS_OK;
}

extern "C" {

fdas_status fdas_spectrum(fdas_plan_t pl, const float* series, const int64_t* offsets, const int64_t* lengths,
                          int32_t n, void* spec_out) {
  if (!pl) return FDAS_ERR_ARG;
  if (!pl->ws) return pl->fail(FDAS_ERR_STATE, "no workspace bound");
  if (!series || !offsets || !spec_out) return pl->fail(FDAS_ERR_ARG, "series, offsets and spectrum_out are required");
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  fdas_status s = set_batch(pl, offsets, lengths, n);
  if (s != FDAS_OK) return s;
  return run_spectrum(pl, series, spec_out);
}

fdas_status fdas_convolve_spectrum(fdas_plan_t pl, const void* spectrum, const int64_t* lengths, int32_t n,
                                   void* plane, int64_t plane_bytes) {
  if (!pl) return FDAS_ERR_ARG;
  if (!pl->ws) return pl->fail(FDAS_ERR_STATE, "no workspace bound");
  if (!spectrum) return pl->fail(FDAS_ERR_ARG, "spectrum is required");
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  fdas_status s = ensure_lengths(pl, lengths, n);
  if (s != FDAS_OK) return s;
  return run_conv(pl, spectrum, plane, plane_bytes);
}

fdas_status fdas_convolve(fdas_plan_t pl, const float* series, const int64_t* offsets, const int64_t* lengths,
                          int32_t n, void* spec_out, void* plane, int64_t plane_bytes) {
  if (!pl) return FDAS_ERR_ARG;
  if (!pl->ws) return pl->fail(FDAS_ERR_STATE, "no workspace bound");
  if (!series || !offsets) return pl->fail(FDAS_ERR_ARG, "series and offsets are required");
  if (!pl->templates_ready) return pl->fail(FDAS_ERR_STATE, "fdas_make_templates has not run");
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  fdas_status s = set_batch(pl, offsets, lengths, n);
  if (s != FDAS_OK) return s;
  if (!plane || plane_bytes < plane_need(pl)) return pl->fail(FDAS_ERR_NOMEM, "plane buffer missing or too small");
  void* spec = spec_out ? spec_out : (void*)(pl->ws + pl->off_spec);
  if ((s = run_spectrum(pl, series, spec)) != FDAS_OK) return s;
  return run_conv(pl, spec, plane, plane_bytes);
}

fdas_status fdas_plane_maxima(fdas_plan_t pl, void* plane, const int64_t* lengths, int32_t n, int64_t plane_bytes) {
  if (!pl) return FDAS_ERR_ARG;
  if (!pl->ws) return pl->fail(FDAS_ERR_STATE, "no workspace bound");
  if (!plane) return pl->fail(FDAS_ERR_ARG, "plane is required");
  if (((uintptr_t)plane) & 15) return pl->fail(FDAS_ERR_ARG, "plane must be 16-byte aligned");
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  fdas_status s = ensure_lengths(pl, lengths, n);
  if (s != FDAS_OK) return s;
  if (plane_bytes < plane_need(pl)) return pl->fail(FDAS_ERR_NOMEM, "plane buffer too small for the values and their maxima");
  e = launch_plane_maxima(pl->p.plane_dtype, plane, plane_maxima(pl, plane),
                          reinterpret_cast<const SeriesDesc*>(pl->ws + pl->off_desc), (int)pl->desc.size(), pl->Z,
                          pl->res == 2 ? 1 : 0, pl->max_bins, pl->cu_count, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "column maxima");
  note_maxima_written(pl, plane);
  return FDAS_OK;
}

fdas_status fdas_harmonic_sum(fdas_plan_t pl, const void* plane, const int64_t* lengths, int32_t n,
                              fdas_candidate* cands, int64_t capacity, int64_t* d_count) {
  if (!pl) return FDAS_ERR_ARG;
  if (!pl->ws) return pl->fail(FDAS_ERR_STATE, "no workspace bound");
  if (!plane || !d_count || capacity < 0 || (capacity > 0 && !cands))
    return pl->fail(FDAS_ERR_ARG, "plane and d_count are required; cands when capacity > 0");
  fdas_status s = check_harm_plane(pl, plane);
  if (s != FDAS_OK) return s;
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  s = ensure_lengths(pl, lengths, n);
  if (s != FDAS_OK) return s;
  if (!maxima_written(pl, plane))
    return pl->fail(FDAS_ERR_STATE,
                    "no column maxima were written for this plane buffer and batch (run the convolution or "
                    "fdas_plane_maxima on it with this plan first)");
  const HarmArgs a = harm_args(pl, plane, cands, capacity, d_count);
  if ((e = launch_harmonic_sum(pl->p.plane_dtype, a, pl->stream)) != hipSuccess)
    return hip_fail(pl, e, "harmonic sum");
  return FDAS_OK;
}

}  // extern "C"

// Enqueues the whole search for the current batch (descriptors already uploaded).
static fdas_status enqueue_search(fdas_plan_t pl, const float* series, void* spec, void* plane, int64_t plane_bytes,
                                  fdas_candidate* cands, int64_t capacity, int64_t* d_count) {
  hipError_t e = launch_fill_i64(d_count, 1, 0, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "count reset");
  fdas_status s = run_spectrum(pl, series, spec);
  if (s != FDAS_OK) return s;
  if ((s = run_conv(pl, spec, plane, plane_bytes)) != FDAS_OK) return s;
  const HarmArgs a = harm_args(pl, plane, cands, capacity, d_count);
  if ((e = launch_harmonic_sum(pl->p.plane_dtype, a, pl->stream)) != hipSuccess)
    return hip_fail(pl, e, "harmonic sum");
  return FDAS_OK;
}

extern "C" {

fdas_status fdas_search(fdas_plan_t pl, const float* series, const int64_t* offsets, const int64_t* lengths, int32_t n,
                        void* spec_out, void* plane, int64_t plane_bytes, fdas_candidate* cands, int64_t capacity,
                        int64_t* d_count, int32_t use_graph) {
  if (!pl) return FDAS_ERR_ARG;
  if (!pl->ws) return pl->fail(FDAS_ERR_STATE, "no workspace bound");
  if (!pl->templates_ready) return pl->fail(FDAS_ERR_STATE, "fdas_make_templates has not run");
  if (!series || !offsets || !d_count || capacity < 0 || (capacity > 0 && !cands))
    return pl->fail(FDAS_ERR_ARG, "series, offsets and d_count are required; cands when capacity > 0");
  if (use_graph && pl->stream == nullptr)
    return pl->fail(FDAS_ERR_STATE, "graph mode needs a non-default stream");
  fdas_status s = check_harm_plane(pl, plane);
  if (s != FDAS_OK) return s;
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  s = set_batch(pl, offsets, lengths, n);  // uploads descriptors outside any capture
  if (s != FDAS_OK) return s;
  if (!plane || plane_bytes < plane_need(pl)) return pl->fail(FDAS_ERR_NOMEM, "plane buffer missing or too small");
  void* spec = spec_out ? spec_out : (void*)(pl->ws + pl->off_spec);
  if (!use_graph) return enqueue_search(pl, series, spec, plane, plane_bytes, cands, capacity, d_count);

  std::vector<uintptr_t> key = {(uintptr_t)pl->ws, (uintptr_t)series, (uintptr_t)spec, (uintptr_t)plane,
                                (uintptr_t)plane_bytes, (uintptr_t)cands, (uintptr_t)capacity, (uintptr_t)d_count};
  for (int i = 0; i < n; ++i) {
    key.push_back((uintptr_t)offsets[i]);
    key.push_back((uintptr_t)lengths[i]);
  }
  if (!pl->graph_exec || key != pl->graph_key) {
    if (pl->graph_exec) (void)hipGraphExecDestroy(pl->graph_exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    pl->graph_exec = nullptr;
    pl->graph = nullptr;
    if ((e = hipStreamBeginCapture(pl->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(pl, e, "begin capture");
    s = enqueue_search(pl, series, spec, plane, plane_bytes, cands, capacity, d_count);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(pl->stream, &g);
    if (s != FDAS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return hip_fail(pl, e, "end capture");
    if ((e = hipGraphInstantiate(&pl->graph_exec, g, nullptr, nullptr, 0)) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(pl, e, "graph instantiate");
    }
    pl->graph = g;
    pl->graph_key = key;
  }
  if ((e = hipGraphLaunch(pl->graph_exec, pl->stream)) != hipSuccess) return hip_fail(pl, e, "graph launch");
  return FDAS_OK;
}

fdas_status fdas_search_chunked(fdas_plan_t pl, const float* series, const int64_t* offsets, const int64_t* lengths,
                                int32_t n, void* plane, int64_t plane_bytes, fdas_candidate* cands, int64_t capacity,
                                int64_t* d_count, int32_t* n_chunks) {
  if (n_chunks) *n_chunks = 0;
  if (!pl) return FDAS_ERR_ARG;
  if (!pl->ws) return pl->fail(FDAS_ERR_STATE, "no workspace bound");
  if (!pl->templates_ready) return pl->fail(FDAS_ERR_STATE, "fdas_make_templates has not run");
  if (!series || !offsets || !lengths || n <= 0 || !d_count || capacity < 0 || (capacity > 0 && !cands))
    return pl->fail(FDAS_ERR_ARG, "series, offsets, lengths (n > 0) and d_count are required; cands when capacity > 0");
  fdas_status s = check_harm_plane(pl, plane);
  if (s != FDAS_OK) return s;
  if (!plane) return pl->fail(FDAS_ERR_ARG, "plane is required");
  // the chunks: longest runs of consecutive series whose samples fit
  // max_batch_samples (and the per-call series limit) and whose plane fits
  // plane_bytes; a series that fits neither alone is an error before any work
  const int64_t N = pl->p.n_samples;
  std::vector<std::pair<int32_t, int32_t>> chunks;
  for (int32_t i = 0; i < n;) {
    int64_t samples = 0, bins = 0;
    int32_t j = i;
    while (j < n) {
      const int64_t len = lengths[j];
      if (!(len == N || len == N / 2 || len == N / 4) || len < (1 << 17))
        return pl->fail(FDAS_ERR_ARG, "series lengths must be n_samples, n_samples/2 or n_samples/4 (and >= 2^17)");
      if (offsets[j] < 0 || (offsets[j] & 1)) return pl->fail(FDAS_ERR_ARG, "series offsets must be even and non-negative");
      // the chunk's plane buffer: its values and their column maxima
      if (samples + len > pl->max_batch || plane_buffer_bytes(pl, bins + len / 2) > plane_bytes ||
          j - i >= pl->max_series)
        break;
      samples += len;
      bins += len / 2;
      ++j;
    }
    if (j == i)
      return pl->fail(FDAS_ERR_NOMEM, "plane_bytes is smaller than the plane of series " + std::to_string(i));
    chunks.emplace_back(i, j - i);
    i = j;
  }
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  if ((e = launch_fill_i64(d_count, 1, 0, pl->stream)) != hipSuccess) return hip_fail(pl, e, "count reset");
  void* spec = pl->ws + pl->off_spec;
  for (const auto& c : chunks) {
    // set_batch waits for the stream before it reuses its staging buffers
    if ((s = set_batch(pl, offsets + c.first, lengths + c.first, c.second)) != FDAS_OK) return s;
    if ((s = run_spectrum(pl, series, spec)) != FDAS_OK) return s;
    if ((s = run_conv(pl, spec, plane, plane_bytes)) != FDAS_OK) return s;
    HarmArgs a = harm_args(pl, plane, cands, capacity, d_count);
    a.series_base = c.first;
    if ((e = launch_harmonic_sum(pl->p.plane_dtype, a, pl->stream)) != hipSuccess) return hip_fail(pl, e, "harmonic sum");
  }
  if (n_chunks) *n_chunks = (int32_t)chunks.size();
  return FDAS_OK;
}

fdas_status fdas_autotune(const fdas_params* base, int device, void* hip_stream, void* scratch, int64_t scratch_bytes,
                          fdas_params* best, double* best_ms) {
  if (!base || !best || !scratch) {
    g_plan_error = "base, best and scratch are required";
    return FDAS_ERR_ARG;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const int Ls[] = {1024, 2048, 4096, 8192};
  const int tpts[] = {0, 12, 24, 48, 96};
  const int radices[] = {16, 8, 4};
  double best_t = 1e300;
  fdas_params winner = *base;
  bool any = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    g_plan_error = "hipEventCreate failed";
    return FDAS_ERR_HIP;
  }
  fdas_status result = FDAS_OK;
  struct Cfg {
    int L, tpt, radix;
  };
  std::vector<Cfg> cfgs;
  for (int L : Ls)
    for (int tpt : tpts)
      for (int radix : radices)
        if (conv_radix_supported(L, radix)) cfgs.push_back({L, tpt, radix});
  for (const Cfg& c : cfgs) {
    fdas_params p = *base;
    p.segment_len = c.L;
    p.templates_per_tile = c.tpt;
    p.fft_radix = c.radix;
    p.max_batch_samples = p.n_samples;
    fdas_plan_t pl = nullptr;
    if (fdas_plan(&p, device, hip_stream, &pl) != FDAS_OK) continue;  // e.g. L < 4 h_max
    if (c.tpt > pl->Z) {
      fdas_plan_destroy(pl);
      continue;
    }
    const int64_t nb = p.n_samples / 2;
    const int64_t spec_bytes = align256(nb * cbytes(p.store_dtype));
    const int64_t plane_bytes = align256(plane_buffer_bytes(pl, nb));
    const int64_t need = pl->total + spec_bytes + plane_bytes;
    if (need > scratch_bytes) {
      g_plan_error = "autotune scratch too small: need " + std::to_string(need) + " bytes";
      fdas_plan_destroy(pl);
      result = FDAS_ERR_NOMEM;
      break;
    }
    char* base_ptr = (char*)scratch;
    fdas_status s = fdas_set_workspace(pl, base_ptr, pl->total);
    if (s == FDAS_OK) s = fdas_make_templates(pl);
    void* spec = base_ptr + pl->total;
    void* plane = base_ptr + pl->total + spec_bytes;
    if (s == FDAS_OK && launch_fill_noise(spec, p.store_dtype, nb, 12345u, st) != hipSuccess) s = FDAS_ERR_HIP;
    const int64_t len = p.n_samples;
    float best_one = 1e30f;
    for (int rep = 0; rep < 4 && s == FDAS_OK; ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess) {
        s = FDAS_ERR_HIP;
        break;
      }
      s = fdas_convolve_spectrum(pl, spec, &len, 1, plane, plane_bytes);
      float ms = 0.f;
      if (s == FDAS_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        s = FDAS_ERR_HIP;
      if (s == FDAS_OK && rep > 0) best_one = std::min(best_one, ms);  // first run warms up
    }
    if (s != FDAS_OK) g_plan_error = "autotune: " + (pl->err.empty() ? std::string("a HIP event call failed") : pl->err);
    fdas_plan_destroy(pl);
    if (s != FDAS_OK) {
      result = s;
      break;
    }
    if (best_one < best_t) {
      best_t = best_one;
      winner = p;
      any = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (result != FDAS_OK) return result;
  if (!any) {
    g_plan_error = "no candidate configuration was valid";
    return FDAS_ERR_ARG;
  }
  winner.max_batch_samples = base->max_batch_samples;
  *best = winner;
  if (best_ms) *best_ms = best_t;
  return FDAS_OK;
}

fdas_status fdas_check(fdas_plan_t pl, const int64_t* d_count, int64_t capacity) {
  if (!pl) return FDAS_ERR_ARG;
  if (!pl->ws) return pl->fail(FDAS_ERR_STATE, "no workspace bound");
  hipError_t e = hipSetDevice(pl->device);
  if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "stream sync");
  int32_t st = 0;
  e = hipMemcpy(&st, pl->ws + pl->off_status, sizeof(st), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(pl, e, "status read");
  int64_t cnt = 0;
  if (d_count) {
    e = hipMemcpy(&cnt, d_count, sizeof(cnt), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(pl, e, "count read");
  }
  if (st) {
    int32_t zero = 0;
    e = hipMemcpy(pl->ws + pl->off_status, &zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(pl, e, "status clear");
  }
  if (st & 1) return pl->fail(FDAS_ERR_NONFINITE, "a spectrum contained NaN or Inf");
  if (st & 2)
    return pl->fail(FDAS_ERR_NONFINITE, "a spectrum-gradient term was not finite (skipped): non-finite grad_p or y");
  if (d_count && cnt > capacity)
    return pl->fail(FDAS_ERR_OVERFLOW, "candidate buffer overflow: " + std::to_string(cnt) + " passing cells, capacity " +
                                           std::to_string(capacity));
  return FDAS_OK;
}

fdas_status fdas_copy_templates(fdas_plan_t pl, void* taps_out, void* spectra_out) {
  if (!pl) return FDAS_ERR_ARG;
  if (!pl->templates_ready) return pl->fail(FDAS_ERR_STATE, "fdas_make_templates has not run");
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  if (taps_out &&
      (e = hipMemcpyAsync(taps_out, pl->ws + pl->off_taps, (size_t)pl->Z * pl->K * 16, hipMemcpyDeviceToDevice,
                          pl->stream)) != hipSuccess)
    return hip_fail(pl, e, "copy taps");
  if (spectra_out &&
      (e = hipMemcpyAsync(spectra_out, pl->ws + pl->off_tspec, (size_t)pl->Z * pl->L * cbytes(pl->p.store_dtype),
                          hipMemcpyDeviceToDevice, pl->stream)) != hipSuccess)
    return hip_fail(pl, e, "copy spectra");
  return FDAS_OK;
}

int64_t fdas_cluster_scratch_bytes(int64_t capacity) {
  return capacity < 0 || capacity > (int64_t(1) << 30) ? -1 : cluster_scratch_bytes(capacity);
}

fdas_status fdas_cluster(fdas_plan_t pl, const fdas_candidate* cands, const int64_t* d_count, int64_t capacity,
                         int32_t radius_r, int32_t radius_j, void* scratch, int64_t scratch_bytes, uint8_t* keep) {
  if (!pl) return FDAS_ERR_ARG;
  if (!d_count || capacity < 0 || (capacity > 0 && (!cands || !keep)))
    return pl->fail(FDAS_ERR_ARG, "d_count is required; cands and keep when capacity > 0");
  if (radius_r < 0 || radius_r > 64 || radius_j < 0 || radius_j > 64)
    return pl->fail(FDAS_ERR_ARG, "radius_r and radius_j must be in [0, 64]");
  if (capacity > (int64_t(1) << 30)) return pl->fail(FDAS_ERR_ARG, "capacity must be at most 2^30 records");
  if (capacity == 0) return FDAS_OK;
  if (!scratch || scratch_bytes < cluster_scratch_bytes(capacity) || (((uintptr_t)scratch) & 7))
    return pl->fail(FDAS_ERR_NOMEM, "scratch missing, misaligned or smaller than fdas_cluster_scratch_bytes(capacity)");
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  e = launch_cluster(cands, reinterpret_cast<const unsigned long long*>(d_count), capacity, radius_r, radius_j,
                     scratch, keep, pl->cu_count, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "cluster");
  return FDAS_OK;
}

fdas_status fdas_cluster_noalloc(fdas_plan_t pl, const fdas_candidate* cands, const int64_t* d_count, int64_t capacity,
                                 int32_t radius_r, int32_t radius_j, uint8_t* keep) {
  if (!pl) return FDAS_ERR_ARG;
  if (!d_count || capacity < 0 || (capacity > 0 && (!cands || !keep)))
    return pl->fail(FDAS_ERR_ARG, "d_count is required; cands and keep when capacity > 0");
  if (radius_r < 0 || radius_r > 64 || radius_j < 0 || radius_j > 64)
    return pl->fail(FDAS_ERR_ARG, "radius_r and radius_j must be in [0, 64]");
  if (capacity > kClusterStaticMaxRecords)
    return pl->fail(FDAS_ERR_ARG, "fdas_cluster_noalloc takes at most " + std::to_string(kClusterStaticMaxRecords) +
                                      " records (capacity " + std::to_string(capacity) + "); use fdas_cluster");
  if (capacity == 0) return FDAS_OK;
  if (pl->static_table_status != hipSuccess) return hip_fail(pl, pl->static_table_status, "static table look-up");
  void* table = nullptr;
  hipError_t e = cluster_static_scratch(pl->device, &table);  // the address found at plan time
  if (e != hipSuccess) return hip_fail(pl, e, "static table look-up");
  if ((e = hipSetDevice(pl->device)) != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  e = launch_cluster(cands, reinterpret_cast<const unsigned long long*>(d_count), capacity, radius_r, radius_j, table,
                     keep, pl->cu_count, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "cluster");
  return FDAS_OK;
}

fdas_status fdas_copy_thresholds(fdas_plan_t pl, double* tau) {
  if (!pl || !tau) return FDAS_ERR_ARG;
  for (int i = 0; i < pl->nstages; ++i) tau[i] = pl->tau[i];
  return FDAS_OK;
}

static fdas_status rz_check(fdas_plan_t pl, const void* spec, int64_t nb, int64_t n) {
  if (!pl->ws) return pl->fail(FDAS_ERR_STATE, "no workspace bound");
  if (!spec || nb <= 0 || n < 0) return pl->fail(FDAS_ERR_ARG, "spectrum, n_bins > 0 and n >= 0 are required");
  if (nb > pl->max_batch / 2) return pl->fail(FDAS_ERR_ARG, "n_bins exceeds max_batch_samples / 2");
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  return FDAS_OK;
}

fdas_status fdas_rz_power(fdas_plan_t pl, const void* spec, int64_t nb, const double* r, const double* z, int64_t n,
                          double* p, void* y_out) {
  if (!pl) return FDAS_ERR_ARG;
  fdas_status s = rz_check(pl, spec, nb, n);
  if (s != FDAS_OK) return s;
  if (n == 0) return FDAS_OK;
  if (!r || !z || !p) return pl->fail(FDAS_ERR_ARG, "r, z and p are required");
  hipError_t e = launch_rz_power(pl->p.store_dtype, spec, nb, r, z, n, pl->p.kernel_margin, p, (c64*)y_out, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "rz power");
  return FDAS_OK;
}

fdas_status fdas_rz_power_grad(fdas_plan_t pl, const void* spec, int64_t nb, const double* r, const double* z,
                               const void* y, const double* grad_p, int64_t n, double* grad_r, double* grad_z,
                               void* grad_spectrum) {
  if (!pl) return FDAS_ERR_ARG;
  fdas_status s = rz_check(pl, spec, nb, n);
  if (s != FDAS_OK) return s;
  if (n == 0) return FDAS_OK;
  if (!r || !z || !grad_p || !grad_r || !grad_z) return pl->fail(FDAS_ERR_ARG, "r, z, grad_p, grad_r, grad_z are required");
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(pl->ws + pl->off_Y);
  // status word at byte 0 of the status block, the gradient bound at 8 and the
  // fixed-point unit at 16
  int32_t* status = reinterpret_cast<int32_t*>(pl->ws + pl->off_status);
  unsigned long long* max_bits = reinterpret_cast<unsigned long long*>(pl->ws + pl->off_status + 8);
  double* scale = reinterpret_cast<double*>(pl->ws + pl->off_status + 16);
  hipError_t e = launch_rz_grad(pl->p.store_dtype, spec, nb, r, z, (const c64*)y, grad_p, n, pl->p.kernel_margin, grad_r,
                                grad_z, (float*)grad_spectrum, acc, max_bits, scale, status, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "rz power grad");
  return FDAS_OK;
}

fdas_status fdas_refine(fdas_plan_t pl, const void* spec, int64_t nb, double* r, double* z, int64_t n, int32_t n_iter,
                        double* p_final) {
  if (!pl) return FDAS_ERR_ARG;
  fdas_status s = rz_check(pl, spec, nb, n);
  if (s != FDAS_OK) return s;
  if (n == 0) return FDAS_OK;
  if (!r || !z || !p_final || n_iter < 0 || n_iter > 1000)
    return pl->fail(FDAS_ERR_ARG, "r, z, p_final are required and 0 <= n_iter <= 1000");
  hipError_t e = launch_refine(pl->p.store_dtype, spec, nb, r, z, n, n_iter, pl->p.kernel_margin, p_final, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "refine");
  return FDAS_OK;
}

fdas_status fdas_refine_harmonics(fdas_plan_t pl, const void* spec, int64_t nb, double* r, double* z,
                                  const int32_t* n_harm, int64_t n, int32_t n_iter, double* p_final) {
  if (!pl) return FDAS_ERR_ARG;
  fdas_status s = rz_check(pl, spec, nb, n);
  if (s != FDAS_OK) return s;
  if (n == 0) return FDAS_OK;
  if (!r || !z || !n_harm || !p_final || n_iter < 0 || n_iter > 1000)
    return pl->fail(FDAS_ERR_ARG, "r, z, n_harm, p_final are required and 0 <= n_iter <= 1000");
  hipError_t e = launch_refine_harmonics(pl->p.store_dtype, spec, nb, r, z, n_harm, n, n_iter, pl->p.kernel_margin,
                                         p_final, pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "refine harmonics");
  return FDAS_OK;
}

fdas_status fdas_test_fft(fdas_plan_t pl, int32_t L, int32_t direction, const void* in, void* out, int64_t batch) {
  if (!pl) return FDAS_ERR_ARG;
  if (!pl->ws) return pl->fail(FDAS_ERR_STATE, "no workspace bound");
  if (!in || !out || batch <= 0 || !(direction == -1 || direction == 1))
    return pl->fail(FDAS_ERR_ARG, "in/out required, batch > 0, direction -1 or +1");
  if (!pl->tw(L)) return pl->fail(FDAS_ERR_UNSUPPORTED, "FFT length not built");
  hipError_t e = hipSetDevice(pl->device);
  if (e != hipSuccess) return hip_fail(pl, e, "hipSetDevice");
  e = launch_test_fft(L, direction, (const c32*)in, (c32*)out, batch, pl->tw(L), pl->stream);
  if (e != hipSuccess) return hip_fail(pl, e, "test fft");
  return FDAS_OK;
}

fdas_status fdas_plan_destroy(fdas_plan_t pl) {
  if (!pl) return FDAS_OK;
  if (pl->graph_exec) (void)hipGraphExecDestroy(pl->graph_exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->h_desc_pinned || pl->h_lists_pinned) {
    (void)hipSetDevice(pl->device);
    (void)hipStreamSynchronize(pl->stream);
    if (pl->h_desc_pinned) (void)hipHostFree(pl->h_desc_pinned);
    if (pl->h_lists_pinned) (void)hipHostFree(pl->h_lists_pinned);
  }
  delete pl;
  return FDAS_OK;
}

const char* fdas_last_error(fdas_plan_t pl) {
  if (!pl) return g_plan_error.c_str();
  return pl->err.c_str();
}

}  // extern "C"
