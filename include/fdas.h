/*
 * fdas.h - C ABI of the MI355X (gfx950) Fourier Domain Acceleration Search hot path.
 *
 * The method: the paper's section 2.1 ("FDAS") describes a matched filter that
 * correlates the spectrum of each dedispersed time series with templates of
 * constant acceleration, so the cost grows linearly with the number of
 * acceleration trials; section 2.2 ("Mixed-Precision") performs that
 * correlation in the frequency domain with FFTs and converts this
 * convolution stage to bfloat16 (here: its data stored in 16 bits, its
 * arithmetic FP32 apart from the FP16 matrix-core stages described at
 * fdas_convolve_spectrum); section 3
 * ("Results") sets the SKA-like workload (600 s at 64 us, 5925 DM trials of
 * which 3050 at full time resolution, 193 acceleration trials).  The
 * harmonic-summing stage that follows the correlation is cited in the
 * introduction.  Formulas that the paper leaves implicit are stated at each
 * entry point below.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Ownership: every data pointer is caller-owned DEVICE memory on the plan's
 *    device unless stated otherwise; the library allocates no device memory.
 *    Its scratch space is one caller-allocated workspace (fdas_query, then
 *    fdas_set_workspace).  Host arrays (offsets, lengths, outputs named
 *    *_host) are read or written before the call returns.
 *  - Asynchrony: work is enqueued on the plan's HIP stream and the call returns
 *    without waiting, except where stated (fdas_check, fdas_copy_thresholds).
 *  - Errors: arguments are checked before anything is enqueued; a failed check
 *    returns a non-zero fdas_status, enqueues nothing and sets the plan's
 *    message (fdas_last_error).  A HIP launch error returns FDAS_ERR_HIP.
 *    Conditions detected on the device (non-finite spectrum, candidate buffer
 *    overflow) are latched in the workspace and reported by fdas_check.
 *    No C++ exception crosses this interface and nothing aborts.
 *  - Threading: a plan is used by one host thread at a time; plans are
 *    independent of each other.
 *  - Complex values are (re, im) pairs of the storage type: FDAS_F32 8 bytes,
 *    FDAS_BF16 and FDAS_F16 4 bytes (re in the low half), rounded to nearest
 *    even on conversion.  FDAS_F16 holds magnitudes up to 65504: a spectrum
 *    component or a power above that is stored as +inf (a power plane of
 *    median-normalised noise has mean 1; a signal saturates an FP16 plane
 *    only above ~65000 times the noise power, where FDAS_BF16 does not).
 *  - Batches: series are float32, given by device pointer `series` plus host
 *    arrays offsets[i] (first sample of series i in `series`) and lengths[i]
 *    (its length N_i: n_samples, n_samples/2 or n_samples/4, i.e. full
 *    resolution or 2x/4x decimated DM trials).  Spectra are packed in series
 *    order, series i starting at complex element S_i = sum_{k<i} N_k/2.  Power
 *    planes are packed the same way, series i starting at element Z*S_i and
 *    laid out z-major: plane_i[j][r], j < Z acceleration trials, r < N_i/2.
 *  - Plane buffers: the packed plane values (C = sum_i N_i/2 columns per
 *    trial, twice that on a half-bin plane; Z*C elements of plane_dtype) are
 *    followed by their column maxima, Z*C/8 elements of plane_dtype: series
 *    i's from element Z*S_i/8 of that section (Z*S_i/4 on a half-bin plane),
 *    row j holding M_i[j][c] = max_{q<8} plane_i[j][8c + q], a NaN or
 *    negative value (sign bit set) counting as +inf, so that M bounds every
 *    value of its run whatever they are.  A plane buffer therefore holds
 *    9*Z*C/8 elements.  The convolution writes both parts; the harmonic sum
 *    reads both (it bounds the upper half of the harmonics by the maxima and
 *    sums exactly only where a bound passes, see fdas_harmonic_sum).  A
 *    caller that writes plane values itself calls fdas_plane_maxima before
 *    the harmonic sum.
 */
#ifndef FDAS_H
#define FDAS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdas_plan_s *fdas_plan_t; /* opaque, owned by the library */

typedef enum {
  FDAS_OK = 0,
  FDAS_ERR_ARG = 1,         /* invalid argument or size */
  FDAS_ERR_NOMEM = 2,       /* workspace or output buffer too small */
  FDAS_ERR_HIP = 3,         /* HIP runtime error */
  FDAS_ERR_UNSUPPORTED = 4, /* valid but not built (e.g. a segment length) */
  FDAS_ERR_OVERFLOW = 5,    /* more candidates than the buffer holds */
  FDAS_ERR_NONFINITE = 6,   /* NaN or Inf in a spectrum */
  FDAS_ERR_STATE = 7        /* call out of order (no workspace, no templates) */
} fdas_status;

typedef enum { FDAS_F32 = 0, FDAS_BF16 = 1, FDAS_F16 = 2 } fdas_dtype;

typedef enum { FDAS_NORM_NONE = 0, FDAS_NORM_VARIANCE = 1, FDAS_NORM_MEDIAN = 2, FDAS_NORM_REDNOISE = 3 } fdas_norm;

typedef struct {
  int64_t n_samples;         /* N of the longest series: a power of two, 2^17 .. 2^23 */
  int64_t max_batch_samples; /* largest sum of lengths per call; 0 means n_samples */
  double tsamp;              /* sampling time in s (metadata: f = r/T, fdot = z/T^2, T = N tsamp) */
  double z_min, z_max, z_step; /* acceleration trials z_j = z_min + j z_step in bins, z_min = -z_max */
  int32_t n_harmonics;       /* highest harmonic summed: 1, 2, 4, 8 or 16 */
  int32_t kernel_margin;     /* m: template half-width h(z) = ceil(|z|/2) + m bins (default 16) */
  int32_t segment_len;       /* overlap-save FFT length L: 1024, 2048, 4096 or 8192; 0 = 1024 */
  int32_t store_dtype;       /* fdas_dtype of spectra and template spectra */
  int32_t plane_dtype;       /* fdas_dtype of the power plane */
  int32_t norm;              /* fdas_norm */
  int32_t norm_block;        /* bins per median block B (power of two, divides N/2; default 2048) */
  double noise_var;          /* sigma^2 for FDAS_NORM_VARIANCE */
  double sigma_threshold;    /* Gaussian-equivalent detection threshold (default 6) */
  int32_t r_lo;              /* lowest fundamental bin searched; 0 means h_max */
  int32_t templates_per_tile; /* templates one wavefront runs per loaded segment; 0 = automatic */
  int32_t interbin;          /* 0: plane at bin resolution; 1: half-bin plane (below) */
  int32_t fft_radix;         /* radix of the convolution FFT's passes: 0 or 16 (default), 8 or 4 at
                                segment_len 1024 (passes 8 8 8 2, or five of 4); fdas_autotune picks it */
} fdas_params;

/* Half-bin plane (interbin = 1; the paper works at whole bins, this sub-bin
 * step is an addition).  After the matched filter a signal at mean frequency
 * rbar leaves y(r) proportional to exp(-i pi d) sinc(d), d = r - rbar, at every
 * z (the template autocorrelation, by Parseval), so a signal midway between
 * bins keeps only sinc(1/2)^2 = 0.405 of its power in either.  The half-bin
 * value |y_r - y_{r+1}|^2 / 2 keeps 8/pi^2 = 0.81 of it, and has unit-mean
 * noise like the bins (neighbouring outputs are uncorrelated).  With it on:
 *  - the plane of series i has 2 N_i/2 = N_i columns per trial and starts at
 *    element 2 Z S_i; column 2r holds P[j][r], column 2r+1 the half-bin power
 *    between r and r+1 (y(N_i/2) from the zero-extended spectrum);
 *  - U <= L - 2 h' - 1 (fdas_plan), so every segment holds y at its last
 *    output + 1;
 *  - fdas_harmonic_sum works on half-bin columns: R counts half bins, a cell
 *    is searched at stage H' if R >= 2 H' r_lo and R < 2 (N/2 - h_max), and
 *    the record's r = R / (2H) bins;
 *  - fdas_cluster's radius_r counts half bins;
 *  - plane buffers are 16-byte aligned (as every plane buffer). */

/* One detection: 32 bytes. harm is the number of harmonics summed (H), R and j
 * the cell of the H-th harmonic (bin, or half bin on a half-bin plane;
 * acceleration-trial index), r = R/H bins (R/(2H) on a half-bin plane) and
 * z = z_j/H the fundamental, power the harmonic sum S_H, sigma its
 * Gaussian-equivalent significance. */
typedef struct {
  int32_t series, harm, R, j;
  float r, z, power, sigma;
} fdas_candidate;

/* Fills *p with defaults (margin 16, L 1024, FP32 storage and plane, median
 * normalisation with B = 2048, 6 sigma, 16 harmonics, z in [-96, 96] step 1,
 * N = 2^23, tsamp 64 us).  Never fails for a non-NULL p. */
fdas_status fdas_default_params(fdas_params *p);

/* Plan (section 2.1: the search is set by the series length and sampling,
 * the acceleration trials z = fdot T^2 and the harmonics summed; section 3:
 * the SKA-like workload, 2^23 samples at 64 us, the longest series a plan
 * takes, searched over 193 acceleration trials).
 * Validates *params and creates a plan bound to `device` and the HIP stream
 * `hip_stream` (NULL = default stream).  Derived sizes: Z = (z_max - z_min)/z_step + 1,
 * h_max = ceil(z_max/2) + m; segments keep U outputs from FFT index h',
 * h' = h_max rounded up to a multiple of 8 (of 4 on a half-bin plane) and U
 * the largest such multiple <= L - 2 h' (<= L - 2 h' - 1 on a half-bin
 * plane), so that every run of 8 plane columns lies in one segment.  Thresholds
 * tau_H solve P(Gamma(H,1) > tau_H) = P(N(0,1) > sigma_threshold) in FP64: a
 * noise harmonic sum of H unit-mean exponential powers is Gamma(H,1).
 * On failure *out is NULL and the message is available from fdas_last_error(NULL). */
fdas_status fdas_plan(const fdas_params *params, int device, void *hip_stream, fdas_plan_t *out);

/* Workspace bytes the plan needs (templates, FFT scratch for max_batch_samples,
 * twiddle tables, device status), and the derived L, h_max and Z.  Any output
 * pointer may be NULL. */
fdas_status fdas_query(fdas_plan_t plan, int64_t *workspace_bytes, int32_t *L, int32_t *h_max, int32_t *Z);

/* Binds caller-allocated device memory (256-byte aligned, at least the queried
 * size) as the plan's workspace.  The plan keeps the pointer, never frees it;
 * binding a new workspace discards templates made in the old one. */
fdas_status fdas_set_workspace(fdas_plan_t plan, void *dev_ptr, int64_t bytes);

/* Builds the template bank on the device in FP64 (section 2.1's matched-filter
 * templates, one per acceleration trial):
 *   rho(q, z) = int_0^1 exp(-2 pi i q u + i pi z (u - 1/2)^2) du  (Fresnel integrals),
 *   t_q(z_j) = conj(rho(q, z_j)) / sqrt(E_j) for |q| <= h(z_j), E_j = sum |rho|^2,
 * and their length-L spectra T_j[k] = (1/L) sum_q t_q exp(+2 pi i k q / L)
 * (the 1/L of the inverse FFT folded in), stored in store_dtype.
 * Needs a workspace.  Must run before fdas_convolve*. */
fdas_status fdas_make_templates(fdas_plan_t plan);

/* Spectrum: real FFT of every series, A_r = sum_n x_n exp(-2 pi i r n/N) for
 * r < N/2 (Nyquist dropped, A_0 set to 0), then normalisation: NONE; VARIANCE
 * A/sqrt(N sigma^2); MEDIAN A sqrt(ln2/m_b) with m_b the lower median of |A|^2
 * (rank (B-1)/2) in each block of B bins (a zero median scales the block by 0);
 * REDNOISE (an addition for red-noise continua, which the paper leaves
 * implicit) as MEDIAN, but block b (bins b B ... (b+1) B - 1) is cut into equal
 * sub-blocks of width w_b = clamp(largest power of two <= b B / 8, 32, B), each
 * scaled by its own lower median (whitening of a steep low-frequency
 * continuum: a block is at most an eighth of its frequency wide).
 * spectrum_out: store_dtype complex, packed as described above. */
fdas_status fdas_spectrum(fdas_plan_t plan, const float *series, const int64_t *offsets_host,
                          const int64_t *lengths_host, int32_t n_series, void *spectrum_out);

/* Convolution (section 2.2: the correlation with every template runs in the
 * frequency domain through FFTs, this stage's data stored in store_dtype;
 * section 2.1: one output row per acceleration trial).  Arithmetic is FP32,
 * except with a 16-bit plane_dtype at L = 1024 (fft_radix 16; bins or half bins):
 * there the two 16-point DFT stages of each 1024-point inverse FFT are FP16
 * matrix-core products with FP32 sums, the products with the templates are
 * FP16 (templates rounded once from FP64 to FP16, times 2^10), and every
 * segment's operands are scaled by a power of two that keeps them inside
 * FP16's range (undone exactly on the power; the scale covers segments whose
 * largest spectrum component lies between about 2^-44 and 2^56 in
 * magnitude, normalised spectra being of order 1, and a segment below that
 * range yields powers of 0); the error this adds to an output is about
 * 2^-11 of the segment's rms amplitude.
 * From a normalised spectrum (store_dtype, packed): overlap-save
 * segments of L bins starting at s U - h' (zero outside [0, N/2); h' and U
 * as at fdas_plan), one forward FFT per segment, then for every template j:
 * product with T_j, inverse FFT, and P[j][s U + i] = |y[h' + i]|^2 for
 * i < U, i.e.
 *   P[j][r] = | sum_{q=-h_max}^{h_max} A'_{r+q} t_q(z_j) |^2,
 * written to plane_out (plane_dtype, packed z-major; with interbin the
 * half-bin plane described at fdas_params), together with the column
 * maxima of the plane-buffer convention.  plane_bytes is the size of
 * plane_out and must cover the whole batch (9*Z*C/8 elements). */
fdas_status fdas_convolve_spectrum(fdas_plan_t plan, const void *spectrum, const int64_t *lengths_host,
                                   int32_t n_series, void *plane_out, int64_t plane_bytes);

/* Spectrum and convolution in one call (sections 2.1 and 2.2, as the two
 * entry points it chains): fdas_spectrum then fdas_convolve_spectrum.
 * spectrum_out may be NULL, in which case the spectrum lives in the workspace. */
fdas_status fdas_convolve(fdas_plan_t plan, const float *series, const int64_t *offsets_host,
                          const int64_t *lengths_host, int32_t n_series, void *spectrum_out,
                          void *plane_out, int64_t plane_bytes);

/* Column maxima of a plane buffer whose values the caller wrote (an
 * addition: the harmonic sum's bound, see the plane-buffer convention above;
 * the convolution entry points write them with the plane).  plane: device,
 * 16-byte aligned; plane_bytes: its size, at least 9*Z*C/8 elements of
 * plane_dtype for the batch given by lengths_host (FDAS_ERR_NOMEM otherwise).
 * Reads the values, writes the maxima section. */
fdas_status fdas_plane_maxima(fdas_plan_t plan, void *plane, const int64_t *lengths_host, int32_t n_series,
                              int64_t plane_bytes);

/* Harmonic sums (the introduction's harmonic-summing stage, which follows the
 * correlation; the paper names it without formulas, so the index rule below
 * is this library's reading): nested harmonic sums and thresholding over a
 * plane buffer (values and column maxima, as fdas_convolve* or
 * fdas_plane_maxima left it).  plane: device, 16-byte aligned (FDAS_ERR_ARG
 * otherwise).  For cell (R, j) with m = j - j0 (j0 the z = 0 trial) and H the top stage,
 *   S_H(R, j) = sum_{k=1}^{H} P[j0 + sgn(m) floor((2k|m| + H)/(2H))][floor((2kR + H)/(2H))],
 * and the lower stages H' use the terms k = H/H', 2H/H', ..., H.  A cell is
 * searched at stage H' if R >= H' r_lo and R < N/2 - h_max, passes if
 * S_{H'} >= tau_{H'}, and emits one record for its most significant passing
 * stage.  Records are appended at atomically reserved indices of `cands`
 * (device, `capacity` records, order not deterministic); *d_count (device
 * int64, zeroed by the caller before the first call of a search) counts every
 * passing cell, also those that did not fit.  On a half-bin plane the same
 * sums run over half-bin columns (see fdas_params).  The sums are first
 * bounded with each term k > H/2 replaced by the column maximum over its
 * run of 8 columns; only cells with a bound at or above a threshold read
 * those terms from the plane and sum exactly, in the same order, so the
 * records are those of the exact sums (stale maxima would lose detections).
 * The maxima are read where this call's batch puts them, so the plan must
 * have written them for this plane buffer and batch (its convolution entry
 * points, fdas_search or fdas_plane_maxima, among its last 8 such writes):
 * otherwise FDAS_ERR_STATE and nothing is enqueued.  Plane values changed
 * after that need fdas_plane_maxima again. */
fdas_status fdas_harmonic_sum(fdas_plan_t plan, const void *plane, const int64_t *lengths_host,
                              int32_t n_series, fdas_candidate *cands, int64_t capacity,
                              int64_t *d_count);

/* Off-grid power, forward (an addition: the paper stops at grid candidates;
 * this is section 2.1's matched filter evaluated between grid points, the
 * differentiable form used for refinement): Fourier-interpolated
 * matched-filter power at off-grid candidates:
 *   y(r, z) = sum_{k = k0-w+1}^{k0+w} A_k conj(rho(k - r, z)),  k0 = floor(r),
 *   w = kernel_margin + ceil(|z|/2) (32 bins at z = 0), A_k = 0 outside [0, n_bins),
 *   P = |y|^2, evaluated in FP64.
 * spectrum: store_dtype complex [n_bins] (one series, e.g. from fdas_spectrum);
 * r, z, p: double [n] device arrays (positions need FP64: bins reach 2^22);
 * a position that is not finite, has |z| > 2^17 or |r| >= 2^52 gives NaN (in
 * every output of these calls, and fdas_refine* leave it where it is);
 * y_out (optional, complex128 [n]) keeps y for the adjoint.
 * n_bins <= max_batch_samples / 2. */
fdas_status fdas_rz_power(fdas_plan_t plan, const void *spectrum, int64_t n_bins, const double *r, const double *z,
                          int64_t n, double *p, void *y_out);

/* Off-grid power, adjoint (an addition, like fdas_rz_power): given the
 * upstream gradient grad_p[i] of a real loss with
 * respect to p[i], writes grad_r[i] = grad_p 2 Re(conj(y) dy/dr),
 * grad_z[i] = grad_p 2 Re(conj(y) dy/dz) (dy/dr = -sum A_k conj(d rho/dq),
 * dy/dz = sum A_k conj(d rho/dz), FP64), and, if grad_spectrum is non-NULL,
 * overwrites it (complex64 [n_bins]) with sum_i grad_p[i] 2 y_i rho(k - r_i, z_i),
 * the gradient with respect to A_k as d/dRe + i d/dIm.  That sum is formed in
 * fixed point with integer atomics, so it is bitwise deterministic, at a unit
 * 2^-s chosen per call that no partial sum can overflow: |rho| <= 1, so every
 * term of candidate i is at most b_i = 2 |grad_p[i]| |y_i|, and s is the
 * largest integer <= 40 with n max_i b_i 2^s <= 2^61 (|dP/dA| of any size
 * keeps 2^-61 of n max_i b_i as its resolution).  A term that is not finite
 * (non-finite grad_p or y) is left out and reported by fdas_check as
 * FDAS_ERR_NONFINITE.
 * y: the forward's y_out, or NULL to recompute it.  Uses the workspace. */
fdas_status fdas_rz_power_grad(fdas_plan_t plan, const void *spectrum, int64_t n_bins, const double *r,
                               const double *z, const void *y, const double *grad_p, int64_t n, double *grad_r,
                               double *grad_z, void *grad_spectrum);

/* Refinement (an addition: the paper stops at grid candidates; this climbs
 * the off-grid power of fdas_rz_power from a candidate): n_iter steps of
 * preconditioned gradient ascent of
 * P(r, z) per candidate (step (dP/dr / (2 a P), dP/dz / (2 b P)) with
 * a = pi^2/3, b = pi^2/180, clamped to 0.25 bin and 2 z, halved until P
 * grows), r and z updated in place (double [n]), and the final power evaluated
 * in FP64 at the returned position into p_final (double [n]). */
fdas_status fdas_refine(fdas_plan_t plan, const void *spectrum, int64_t n_bins, double *r, double *z, int64_t n,
                        int32_t n_iter, double *p_final);

/* Harmonic refinement (an addition: the paper stops at candidates; this
 * refines a harmonic-sum candidate of the introduction's harmonic summing on
 * the sum it was found with): the same ascent on the incoherent harmonic
 * power of a fundamental (r, z), harmonic k of a signal drifting by z bins
 * lying at k r and drifting by k z:
 *   S(r, z) = sum_{k=1}^{H} P(k r, k z),  dS/dr = sum_k k dP/dr(k r, k z), likewise z,
 * step (dS/dr / (2 a W), dS/dz / (2 b W)) with W = sum_k k^2 P(k r, k z),
 * clamped to 0.25/H bin and 2/H z and halved until S grows; for H = 1 exactly
 * fdas_refine.  n_harm: device int32 [n], H per candidate in [1, 32] (any
 * other value leaves that candidate's r and z unchanged and sets its p_final
 * to NaN).  r, z (double [n], fundamentals) are updated in place; p_final
 * (double [n]) receives S in FP64 at the returned position.  n_iter = 0
 * evaluates S at the given positions. */
fdas_status fdas_refine_harmonics(fdas_plan_t plan, const void *spectrum, int64_t n_bins, double *r, double *z,
                                  const int32_t *n_harm, int64_t n, int32_t n_iter, double *p_final);

/* The whole search for one batch in one call: resets *d_count (with a kernel),
 * then spectrum, convolution and harmonic sums exactly as fdas_spectrum,
 * fdas_convolve_spectrum and fdas_harmonic_sum.  With use_graph != 0 the
 * launches are captured once into a HIP graph (the plan's stream must not be
 * the default stream) and replayed on later calls with the same pointers,
 * offsets and lengths; the batch descriptors are uploaded before capture.
 * The batch may mix full-length and decimated series; the
 * convolution tiles of all series go to one persistent launch. */
fdas_status fdas_search(fdas_plan_t plan, const float *series, const int64_t *offsets_host,
                        const int64_t *lengths_host, int32_t n_series, void *spectrum_out, void *plane_out,
                        int64_t plane_bytes, fdas_candidate *cands, int64_t capacity, int64_t *d_count,
                        int32_t use_graph);

/* The whole search for a batch of any size within a plane buffer of
 * plane_bytes (the HBM budget): the series are taken in consecutive chunks,
 * each the longest run whose samples fit max_batch_samples and whose plane
 * buffers (values and maxima) fit plane_bytes, and every chunk runs as
 * fdas_search (spectrum in the
 * workspace; no graph).  *d_count is reset once (with a kernel) and counts
 * the passing cells of every chunk; the records' series field is the index
 * in offsets/lengths.  The planes are overwritten chunk by chunk (the last
 * chunk's remain).  n_chunks (host, optional) receives the number of chunks.
 * Every argument is checked before any work: a series whose plane alone
 * exceeds plane_bytes is FDAS_ERR_NOMEM.  Waits for the plan's stream before
 * each chunk's descriptors are uploaded (the previous chunk's work). */
fdas_status fdas_search_chunked(fdas_plan_t plan, const float *series, const int64_t *offsets_host,
                                const int64_t *lengths_host, int32_t n_series, void *plane_out, int64_t plane_bytes,
                                fdas_candidate *cands, int64_t capacity, int64_t *d_count, int32_t *n_chunks_host);

/* Tuning: times the convolution of one full-length noise spectrum
 * for every segment length L in {1024, 2048, 4096, 8192} allowed by the z
 * range, templates_per_tile in {auto, 12, 24, 48, 96} and FFT radix plan
 * (fft_radix 16, and 8 and 4 at L = 1024) on `device`/`hip_stream`,
 * using `scratch` (device memory, at least workspace + spectrum + plane
 * buffer of one series; FDAS_ERR_NOMEM names the size), and writes the fastest parameters
 * to *best (and its time in ms to *best_ms).  Blocks until done. */
fdas_status fdas_autotune(const fdas_params *base, int device, void *hip_stream, void *scratch,
                          int64_t scratch_bytes, fdas_params *best, double *best_ms);

/* Waits for the plan's stream, then reports device-side conditions latched
 * since the last fdas_check: FDAS_ERR_NONFINITE if a spectrum held NaN/Inf,
 * FDAS_ERR_OVERFLOW if d_count (optional, device) exceeds capacity. Clears
 * the latch. */
fdas_status fdas_check(fdas_plan_t plan, const int64_t *d_count, int64_t capacity);

/* Copies the FP64 template taps (complex128 [Z][2 h_max + 1], column q + h_max)
 * and/or the template spectra (store_dtype complex [Z][L]) into device buffers;
 * either pointer may be NULL.  For inspection and tests. */
fdas_status fdas_copy_templates(fdas_plan_t plan, void *taps_out, void *spectra_out);

/* Writes the thresholds tau_H for H = 1, 2, 4, ... n_harmonics to the host
 * array tau_host (log2(n_harmonics)+1 values). */
fdas_status fdas_copy_thresholds(fdas_plan_t plan, double *tau_host);

/* Candidate clustering (local maxima; an addition: the paper stops at
 * candidates), the first step of sifting the records of fdas_harmonic_sum /
 * fdas_search: a strong signal leaves a patch of passing cells around its
 * peak.  Record i (i < min(*d_count, capacity)) gets
 * keep[i] = 1 when no record of the same series with |R' - R| <= radius_r and
 * |j' - j| <= radius_j has a larger sigma (equal sigma: the record with the
 * smaller (j, R) wins), else 0 (R in the records' units: half bins after a
 * half-bin search).  cands: the records (device, with sigma filled
 * as those calls leave them); d_count: device int64 record count; keep:
 * device uint8 [capacity]; scratch: caller-owned device memory of at least
 * fdas_cluster_scratch_bytes(capacity) bytes, 8-byte aligned, overwritten.
 * Radii in [0, 64], capacity at most 2^30.  Enqueued on the plan's stream;
 * allocates nothing.  fdas_cluster_scratch_bytes returns -1 for a capacity
 * outside [0, 2^30]. */
int64_t fdas_cluster_scratch_bytes(int64_t capacity);
fdas_status fdas_cluster(fdas_plan_t plan, const fdas_candidate *cands, const int64_t *d_count, int64_t capacity,
                         int32_t radius_r, int32_t radius_j, void *scratch, int64_t scratch_bytes, uint8_t *keep);

/* Candidate clustering without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): exactly fdas_cluster, with its hash table
 * in a static device array of the library (24 MiB on each GPU it runs on,
 * reserved when the library's code is loaded there and held until the process
 * ends) instead of caller scratch.  capacity at most 2^20 records
 * (FDAS_ERR_ARG above that: use fdas_cluster).  The table's device address is
 * looked up once per device when a plan is made there.  Every call on one GPU
 * shares that GPU's table and clears it (with a fill kernel) before use, so
 * calls that overlap on one GPU (two plans on different streams, or two host
 * threads) race and must be ordered by the caller.  Calls no hipMalloc or
 * hipFree. */
fdas_status fdas_cluster_noalloc(fdas_plan_t plan, const fdas_candidate *cands, const int64_t *d_count,
                                 int64_t capacity, int32_t radius_r, int32_t radius_j, uint8_t *keep);

/* Self-test hook of the FFT engine: `batch` independent complex FFTs of
 * length L (256 ... 8192) from `in` to `out` (device, complex64, contiguous),
 * direction -1: X_k = sum_n x_n exp(-2 pi i k n / L), +1: the unnormalised
 * inverse.  Uses the plan's stream and twiddle tables (needs a workspace). */
fdas_status fdas_test_fft(fdas_plan_t plan, int32_t L, int32_t direction, const void *in, void *out, int64_t batch);

/* Releases the plan (not the workspace, which the caller owns). NULL is allowed. */
fdas_status fdas_plan_destroy(fdas_plan_t plan);

/* Message of the last failed call on `plan`, or of the last failed
 * fdas_plan() when plan is NULL.  Valid until the next call on that plan. */
const char *fdas_last_error(fdas_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* FDAS_H */
