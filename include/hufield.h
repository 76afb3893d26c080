/*
 * hufield: generator of anisotropic hyperuniform continuous random fields on gfx950.
 *
 * The method is the single-shot spectral filter of Zhong & Mao (arXiv 2509.08675):
 *   white noise -> forward FFT -> multiply by A = sqrt(chi)            (Sec. II.B, Eq. (8))
 *   chi(k) = C exp[alpha ln K - (K - k0)^2 / (2 w^2)], K the superellipse norm
 *                                                                      (Eqs. (12)-(13); k0 = 0 is Eq. (13))
 *   -> inverse FFT to a real field                                     (Eq. (9))
 *   -> f <- sigma_f (f - <f>) / sqrt(Var f)                           (Eq. (15))
 *   -> sign map f -> +-1 and binned power spectra                      (Sec. II.B end, Sec. III figures)
 * plus the adjoint of the binned spectrum with respect to the filter parameters, the
 * hyperuniformity diagnostics of Sec. II.A (local variance over a spherical window, small-k
 * exponent, class of Eqs. (6)-(7)), a level cut for a target volume fraction with the two-point
 * function of the resulting phases, and the mask variants alpha = 0, alpha < 0 and an offset.
 *
 * Conventions used by every entry point
 * -------------------------------------
 * Grid: hu_dims.n[0] is the slowest axis and n[ndim-1] = n_x the fastest (row-major).  2D is
 *   (n_y, n_x), 3D is (n_z, n_y, n_x).  Each n must be 2^k (4..2048) or 3*2^k (6..768), and n_x/2
 *   must also be one of the supported lengths (so n_x >= 4).  A field holds fewer than 2^31
 *   voxels and its FP32 half spectrum (8 N/n_x (n_x/2+1) bytes) is smaller than 4 GiB (in-field
 *   offsets are 32-bit), so e.g. 1024^2 x 768 is accepted and 1024^3 is not.
 * Wavenumbers: kappa_i = 2 m~_i / n_i in units of the Nyquist wavenumber (m~ the signed index).
 * Noise: voxel i (row-major linear index within a field) takes normal z_{i mod 4} of the
 *   Philox4x32-10 block i // 4 with key (seed lo, seed hi) and counter (block lo, block hi, 0, 0);
 *   uniforms u = (2*(x >> 9) + 1) 2^-24 and Box-Muller on (u0,u1), (u2,u3).
 * Transforms: forward kernel exp(-i k.x), unnormalised.
 * Variance: population (ddof = 0).  Sign map: f >= 0 -> +1, else -1.
 * Spectrum: P(k) = |DFT(g)(k)|^2 / N.  Bins: radial r = floor(R |kappa|) (exact integer rule,
 *   edges go up), angular (2D only) A bins over [0, pi) after folding k -> -k; slot
 *   r * A + a, plus one last slot (index R * A) for the corner modes with |kappa| >= 1.  Each
 *   half-spectrum mode counts with multiplicity 2, or 1 where m_x is 0 or n_x/2.
 *
 * Memory: every array argument is DEVICE memory owned by the caller unless marked "host".
 *   The library keeps per-process read-only tables (twiddles, bin edges and bin tables) that
 *   it allocates on first use of a size and keeps until the process ends; hu_pipeline_batch
 *   also keeps a pinned upload buffer and its cached graphs, and hu_autotune allocates (and
 *   frees) its own test fields.  Apart from those it never allocates.  Workspace is
 *   caller-provided and its required size comes from hu_workspace_size(_batch), except for
 *   hu_pipeline_noalloc, whose workspace is a fixed 128 MiB device array of the library.
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  All work is enqueued
 *   asynchronously; outputs are valid once the stream has been synchronised.  The first call
 *   on a new size waits on the host until its tables are built; hu_pipeline_batch waits for
 *   its previous upload to have been read.  No call reads device memory back to the host.
 * Errors: every argument is validated on the host before any launch; on error nothing is
 *   enqueued and a negative HU_ERR_* code is returned (hu_strerror names it).  HIP launch
 *   errors are returned as HU_ERR_HIP; errors of earlier asynchronous work surface there too.
 *   A filter with no support on the lattice (max ln chi < -80) cannot be detected on the host
 *   without a pass over the lattice, so it is reported in the stats output (flag = 1) and the
 *   field is then all zeros.
 * Determinism: fields, sign maps, counts, the statistics (mean and variance come from a
 *   fixed-order reduction) and the binned spectra (tile partials combined in integer
 *   arithmetic, then summed in a fixed order) are bit-reproducible for a given plan (see
 *   hu_autotune), also across batch layouts and, under the default plans, across batch sizes.
 */
#ifndef HUFIELD_H
#define HUFIELD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HU_OK = 0,
  HU_ERR_ARG = -1,        /* null pointer, non-positive parameter, bad batch or bin count */
  HU_ERR_SIZE = -2,       /* grid size outside the supported set */
  HU_ERR_ALIGN = -3,      /* array not aligned to 16 bytes (workspace: 256 bytes) */
  HU_ERR_WORKSPACE = -4,  /* workspace smaller than hu_workspace_size */
  HU_ERR_DEGENERATE = -5, /* reserved: returned by host-side helpers for a filter with no lattice support */
  HU_ERR_HIP = -6,        /* a HIP runtime call failed */
  HU_ERR_UNSUPPORTED = -7, /* valid request that the library does not implement */
  HU_ERR_TABLES = -8      /* hu_pipeline_noalloc: the per-size tables of the grid / bins do not exist yet */
};

enum { HU_F32 = 0, HU_I8 = 1 };

/* Operations for hu_workspace_size. */
enum { HU_OP_GEN_FIELD = 0, HU_OP_PIPELINE = 1, HU_OP_POWER_SPECTRUM = 2, HU_OP_LOSS = 3, HU_OP_FILTER_SPECTRUM = 4,
       HU_OP_WINDOW_VARIANCE = 5, HU_OP_TWO_POINT = 6 };

/* Most window radii of one hu_window_variance call. */
#define HU_MAX_RADII 32

typedef struct hu_dims {
  int32_t ndim;   /* 2 or 3 */
  int32_t n[3];   /* n[0] slowest ... n[ndim-1] = n_x fastest */
} hu_dims;

/* Filter parameters (Eqs. (12)-(13) and Eq. (15)); all in Nyquist units. */
typedef struct hu_filter {
  double p;        /* superellipse exponent, > 0 (Eq. (12)) */
  double semi[3];  /* semi-axes a (x), b (y), c (z), > 0; c unused in 2D */
  double rot;      /* mask rotation, radians, counter-clockwise in (kappa_x, kappa_y); about z in 3D */
  double alpha;    /* small-k exponent, > -d (Eqs. (13)-(14)); 0 is the standard nonhyperuniform
                      class and -d < alpha < 0 the antihyperuniform one of Eq. (7) */
  double k0;       /* band centre, >= 0 (0 gives Eq. (13) exactly) */
  double width;    /* Gaussian band width w, > 0 (sigma of Eq. (13)) */
  double sigma_f;  /* target standard deviation of the field, > 0 (Eq. (15)) */
  double offset;   /* offset regularisation >= 0 added to the peak-normalised spectral density on
                      every mode but the DC (chi(k -> 0) = offset); 0 is the paper's mask;
                      HU_ERR_UNSUPPORTED together with alpha < 0 */
  /* Optional tabulated radial form (a radial profile beyond Eq. (13), the generalisation named in
   * Sec. IV): when prof_n > 0, ln chi at superellipse norm K is the linear interpolation of the
   * prof_n >= 2 samples prof[i] = ln chi(i * prof_dk) (device memory, FP32, caller-owned, 4-byte
   * aligned; held at the last sample beyond K = (prof_n - 1) prof_dk) in place of
   * alpha ln K - (K - k0)^2 / (2 w^2).  The samples are used as given (an added constant does not
   * change the normalised field, but their lattice maximum must be >= -80); alpha, k0 and width
   * are then unused, offset must be 0 (else HU_ERR_UNSUPPORTED), the DC mode keeps amplitude 0,
   * and hu_spectrum_grad returns HU_ERR_UNSUPPORTED.  prof_n = 0: Eq. (13). */
  const float* prof;
  int32_t prof_n;
  double prof_dk;  /* sample spacing in K, > 0 when prof_n > 0 */
} hu_filter;

typedef struct hu_bins {
  int32_t n_radial;   /* R >= 1 */
  int32_t n_angular;  /* A >= 1; A > 1 only for 2D grids */
} hu_bins;

/* Outputs of hu_pipeline; a NULL member skips that output (and the work only it needs). */
typedef struct hu_outputs {
  float* field;        /* [B][N] FP32 normalised field */
  int8_t* pm1;         /* [B][N] sign map, +1 / -1 */
  double* stats;       /* [B][4] mu_raw, var_raw, max ln chi over the lattice, degenerate flag (0/1) */
  uint64_t* counts;    /* [B][2] n_pos = #(+1), n_near = #(|f| < near_tol * sigma_f) */
  double* cont_sum;    /* [B][R*A+1] binned spectrum of the normalised continuous field */
  uint64_t* cont_cnt;  /* [B][R*A+1] modes per bin (with multiplicity) */
  double* pm1_sum;     /* [B][R*A+1] binned spectrum of the +-1 field */
  uint64_t* pm1_cnt;   /* [B][R*A+1] */
} hu_outputs;

/* Size in bytes of the workspace that `op` needs for `batch` fields of `dims` with `bins`
 * (bins may be NULL when the op uses none).  Returns HU_OK and writes *bytes (host). */
int hu_workspace_size(int op, hu_dims dims, int32_t batch, const hu_bins* bins, size_t* bytes);

/* Generate `batch` normalised fields on `dims` with one filter and per-field seeds
 * (Sec. II.B pipeline, Eqs. (8), (9), (12), (13), (15)).
 *   filt   host pointer to the filter parameters
 *   seeds  host array of `batch` 64-bit seeds
 *   field  [B][N] FP32 output; stats [B][4] as in hu_outputs (may be NULL)
 *   cont_bins  host pointer, or NULL to skip the continuous spectrum; cont_sum/cont_cnt then unused
 *   work   device workspace of at least hu_workspace_size(HU_OP_GEN_FIELD, ...) bytes */
int hu_gen_field(hu_dims dims, int32_t batch, const hu_filter* filt, const uint64_t* seeds,
                 float* field, double* stats, const hu_bins* cont_bins, double* cont_sum,
                 uint64_t* cont_cnt, void* work, size_t work_bytes, void* stream);

/* Sign map of `batch` FP32 fields (the +-1 two-phase medium of Sec. II.B, last paragraphs):
 * out = +1 where field >= 0 else -1; counts [B][2] = (n_pos, n_near) with
 * n_near = #(|field| < near_tol), or counts = NULL.  Needs no workspace. */
int hu_threshold(hu_dims dims, int32_t batch, const float* field, int8_t* out, uint64_t* counts,
                 float near_tol, void* stream);

/* Binned power spectrum P = |DFT(x)|^2 / N of `batch` real fields x (dtype HU_F32 or HU_I8),
 * the spectral densities shown in the figure rows of Sec. III.  sum [B][R*A+1] FP64,
 * cnt [B][R*A+1] (or NULL).  Workspace: hu_workspace_size(HU_OP_POWER_SPECTRUM, ...). */
int hu_power_spectrum(hu_dims dims, int32_t batch, const void* x, int32_t dtype, hu_bins bins,
                      double* sum, uint64_t* cnt, void* work, size_t work_bytes, void* stream);

/* The whole hot path in one call: field, sign map with counts, continuous and +-1 spectra,
 * fused so that normalisation, threshold and the first transform of the +-1 field share one
 * pass.  near_tol is relative to sigma_f (1e-5 is the parity convention).
 * Workspace: hu_workspace_size(HU_OP_PIPELINE, ...). */
int hu_pipeline(hu_dims dims, int32_t batch, const hu_filter* filt, const uint64_t* seeds,
                hu_bins bins, float near_tol, const hu_outputs* out, void* work, size_t work_bytes,
                void* stream);

/* hu_pipeline for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same work, kernels and outputs as
 * hu_pipeline(dims, batch, filt, seeds, bins, near_tol, out, work, bytes, stream), with the
 * workspace taken from a fixed device array inside the library instead of a caller buffer.
 *   Limit: the workspace hu_workspace_size(HU_OP_PIPELINE, dims, min(batch, 64), &bins) reports
 *   must be at most HU_NOALLOC_WORK_BYTES (128 MiB: e.g. one 256^3 field, seven 2048^2 fields,
 *   thirty-one 1024^2 fields with 64 radial bins per call); larger requests return
 *   HU_ERR_WORKSPACE and enqueue nothing.
 *   The array exists once per GPU (the library holds 128 MiB of device memory on every GPU it
 *   runs on until the process ends); its address is looked up once per device on the first call
 *   with that device current.
 *   The call allocates nothing: no hipMalloc / hipFree and no host staging.  The per-size tables
 *   (twiddles, bin tables) must already exist on the current device, i.e. some allocating call
 *   (hu_pipeline, hu_gen_field, hu_power_spectrum, ...) on the same grid and bins has been made
 *   earlier in the process; otherwise HU_ERR_TABLES is returned and nothing is enqueued.
 *   Every call on one GPU shares that GPU's array: calls that overlap in time on one GPU (two
 *   streams, two host threads) race on it and corrupt each other's results; order them on one
 *   stream.  The only words that must start at zero (the work counter of the persistent
 *   binning pass) are cleared by the first kernel of every call; everything else a pass reads was
 *   written by an earlier pass of the same call.
 *   Arguments, outputs and errors otherwise as hu_pipeline. */
#define HU_NOALLOC_WORK_BYTES ((size_t)128 << 20)
int hu_pipeline_noalloc(hu_dims dims, int32_t batch, const hu_filter* filt, const uint64_t* seeds, hu_bins bins,
                        float near_tol, const hu_outputs* out, void* stream);

/* Expected binned spectrum of a filter, with no noise: per mode E[P(k)] = sigma_f^2 N H_sym(k)^2 /
 * sum_k' w_k' H_sym(k')^2 (Eqs. (10)-(11) under the normalisation of Eq. (15)), summed per bin
 * with the half-spectrum multiplicities w exactly like the continuous spectrum of a field, so
 * that sum / cnt is the expected bin mean.  The target of a spectrum-matching loss (parameter
 * optimisation is the extension named in Sec. IV).  sum [R*A+1] FP64 and cnt [R*A+1] (or NULL),
 * device.  The bin sums are formed without floating-point atomics (runs combined in integer
 * arithmetic per chunk of modes, per-workgroup rows summed in a fixed order): bit-reproducible.
 * Workspace: hu_workspace_size(HU_OP_FILTER_SPECTRUM, dims, 1, &bins, ...) (bins required). */
int hu_filter_spectrum(hu_dims dims, const hu_filter* filt, hu_bins bins, double* sum, uint64_t* cnt,
                       void* work, size_t work_bytes, void* stream);

/* Hyperuniformity diagnostics (Sec. II.A).
 *
 * hu_window_variance: the local variance of Eq. (1) over a spherical window (a disk in 2D, a ball
 * in 3D) of radius R, for each of n_radii radii (lattice units, finite, >= 0), of `batch` real
 * periodic fields x (dtype HU_F32 or HU_I8, [B][N] device).  Averaging one Fourier mode of
 * wavevector k over the window multiplies it by W(|k| R), W = 2 J_1(u)/u (2D) or
 * 3 (sin u - u cos u)/u^3 (3D), so with X the unnormalised DFT and k_m = 2 pi m / n per axis
 *   out[b][j] = sum_{m != 0} |X(m)|^2 / N^2 * W(|k_m| R_j)^2,
 * the variance over all window positions of the window average of the field's trigonometric
 * interpolant (R = 0 gives the field's variance).  radii: host array of n_radii (1..HU_MAX_RADII)
 * values; out: device FP64 [B][n_radii].  W in FP32, sums in FP64, reduced in a fixed order
 * (bit-reproducible).  Workspace: hu_workspace_size(HU_OP_WINDOW_VARIANCE, dims, batch, NULL, ...).
 * HU_ERR_ARG for a bad radius count or value, HU_ERR_ALIGN for x or out not 16-byte aligned. */
int hu_window_variance(hu_dims dims, int32_t batch, const void* x, int32_t dtype, const double* radii,
                       int32_t n_radii, double* out, void* work, size_t work_bytes, void* stream);

/* General level cut (Sec. II.B, last paragraphs: the two phases may come from any functional map of
 * the field): out = +1 where field >= t_phi, else -1, with t_phi = sigma_f Phi^-1(1 - phi), the level
 * at which a Gaussian field of standard deviation sigma_f has expected volume fraction phi in the +1
 * phase (phi = 1/2 is the sign map).  counts [B][2] = (n_pos, n_near), n_near = #(|field - t_phi| <
 * near_tol), or NULL.  field, out, counts: device.  HU_ERR_ARG unless 0 < phi < 1, sigma_f > 0 and
 * near_tol >= 0 (all finite).  Needs no workspace. */
int hu_level_cut(hu_dims dims, int32_t batch, const float* field, double phi, double sigma_f, int8_t* out,
                 uint64_t* counts, float near_tol, void* stream);

/* t_phi = sigma_f Phi^-1(1 - phi) in FP64 on the host (Newton's method on the normal CDF from erfc,
 * bracketed by bisection; relative error ~1e-15).  HU_ERR_ARG outside 0 < phi < 1 or sigma_f <= 0. */
int hu_level_threshold(double phi, double sigma_f, double* t);

/* Two-point probability function of the +1 phase of `batch` +-1 maps (int8, [B][N] device):
 * s2[b][r] = (1/N) sum_x I(x) I(x + r), I = (1 + pm1) / 2, for every periodic lattice displacement r
 * (array layout of the field, index r mod n per axis), by the Wiener-Khinchin relation
 * (Eqs. (10)-(11)): S_2 = (1 + 2m + IDFT(|G|^2) / N^2) / 4 with G the DFT of pm1 and m its mean.
 * s2: device FP32 [B][N] (S_2(0) is the volume fraction, the mean over r its square).  Values other
 * than +-1 in pm1 are taken as given (the formula is the autocorrelation of (1 + x) / 2).
 * Workspace: hu_workspace_size(HU_OP_TWO_POINT, dims, batch, NULL, ...). */
int hu_two_point(hu_dims dims, int32_t batch, const int8_t* pm1, float* s2, void* work, size_t work_bytes,
                 void* stream);

/* Small-k exponent of a binned spectrum (the alpha of spectral density ~ |k|^alpha, Sec. II.A):
 * the least-squares slope of ln(sum_r / cnt_r) against ln((r + 1/2) / R) over radial bins
 * r = 1..nfit (bin 0 holds the DC mode), the angular bins of a radius pooled.  sum and cnt are
 * HOST arrays in the [R*A+1] layout of hu_power_spectrum.  Bins with cnt = 0 or sum <= 0 are
 * skipped; HU_ERR_ARG when fewer than two remain or nfit is outside 1..R-1.  Host only. */
int hu_small_k_exponent(const double* sum, const uint64_t* cnt, hu_bins bins, int32_t nfit, double* alpha);

/* Class of Eqs. (6)-(7) for a small-k exponent alpha in dimension d: 0 hyperuniform class I
 * (alpha > 1), 1 class II (|alpha - 1| <= tol), 2 class III (0 < alpha < 1), 3 standard
 * nonhyperuniform (|alpha| <= tol), 4 antihyperuniform (-d < alpha < 0), 5 outside these ranges.
 * Host only. */
int hu_hyperuniformity_class(double alpha, int32_t d, double tol);

/* Spectrum-matching loss for fitting the filter parameters to a target spectrum (the parameter
 * optimisation named as the extension in Sec. IV):
 *   L = (1/|B|) sum_{b in B} (ln(P_b + eps) - ln(T_b + eps))^2,   dL/dP_b = 2 d_b / (|B| (P_b + eps)),
 * P_b = sum[b] / cnt[b] the bin means of a field's continuous spectrum (hu_gen_field), T_b =
 * tsum[b] / tcnt[b] those of the target (e.g. hu_filter_spectrum of the target filter), B the bins
 * of radius r >= 1 that hold modes in both (the DC row r = 0 and the corner slot are excluded).
 * sum, tsum [R*A+1] FP64, cnt, tcnt [R*A+1] uint64 (device, 8-byte aligned); loss [1] and dL_dP
 * [R*A+1] FP64 device outputs (dL_dP is 0 outside B; it feeds hu_spectrum_grad).  eps >= 0 (the
 * parity workloads use 1e-12 sigma_f^2).  One workgroup, fixed-order sums (bit-reproducible).
 * HU_ERR_ARG for bad bins, pointers or eps; HU_ERR_ALIGN for unaligned arrays. */
int hu_spectrum_loss(hu_bins bins, const double* sum, const uint64_t* cnt, const double* tsum, const uint64_t* tcnt,
                     double eps, double* loss, double* dL_dP, void* stream);

/* Adjoint of the binned continuous spectrum with respect to the filter parameters of
 * Eqs. (12)-(13) (the gradient a parameter-fitting loop of Sec. IV needs).  Inputs are the outputs
 * of hu_gen_field(dims, 1, filt, &seed, field, stats, &bins, cont_sum, cont_cnt, ...) for one
 * field, and dL_dP [R*A+1]: the gradient of a loss L with respect to the bin means
 * P_b = cont_sum_b / cont_cnt_b (the corner slot R*A and empty bins are ignored); all device.
 * Writes grad [7] = dL/d(a, b, c, p, rot, k0, w) (device FP64; the c entry is 0 in 2D).  The
 * noise spectrum is regenerated from the seed (nothing of the forward field is read), and the
 * seven sums are FP64 across tiles, reduced in a fixed order (bit-reproducible).  HU_ERR_UNSUPPORTED
 * for a filter with a nonzero offset or a tabulated radial form (only the amplitude sqrt(chi) of
 * Eq. (13) is differentiated).
 * Workspace: hu_workspace_size(HU_OP_LOSS, dims, 1, &bins, ...). */
int hu_spectrum_grad(hu_dims dims, const hu_filter* filt, uint64_t seed, hu_bins bins, const double* dL_dP,
                     const double* cont_sum, const uint64_t* cont_cnt, const double* stats, double* grad,
                     void* work, size_t work_bytes, void* stream);

/* One field of a heterogeneous batch: its own grid, filter, seed, bins and outputs (device
 * pointers, each may be NULL; at least one must be set; bins are used when cont_sum or pm1_sum is
 * set).  Array sizes as in hu_outputs for a batch of one. */
typedef struct hu_job {
  hu_dims dims;
  hu_filter filt;
  uint64_t seed;
  hu_bins bins;
  float* field;
  int8_t* pm1;
  double* stats;
  uint64_t* counts;
  double* cont_sum;
  uint64_t* cont_cnt;
  double* pm1_sum;
  uint64_t* pm1_cnt;
} hu_job;

/* Workspace bytes for hu_pipeline_batch on `jobs` (host array). */
int hu_workspace_size_batch(const hu_job* jobs, int32_t njobs, size_t* bytes);

/* The whole hot path (as hu_pipeline) for a heterogeneous batch of fields of uneven grids and
 * parameters, in one submission: the jobs are grouped by grid and bin layout, each group runs
 * the pass sequence with per-field parameters read from a table in the workspace, and the
 * groups run side by side from one captured HIP graph that is cached and replayed for later
 * batches of the same structure on the same workspace.
 *   jobs, status: host arrays of njobs; status[i] receives job i's validation result (an
 *   invalid job is skipped, the others run).  Returns HU_OK when the valid jobs were enqueued.
 * The first call for a structure captures and instantiates the graph (and builds any missing
 * per-size tables, synchronising the stream); later calls only upload the parameter table
 * (from a pinned staging buffer) and launch the graph.  Calls sharing one workspace must be
 * ordered on one stream. */
int hu_pipeline_batch(const hu_job* jobs, int32_t njobs, float near_tol, int32_t* status, void* work,
                      size_t work_bytes, void* stream);

/* Plan autotuner.  A plan has 13 entries, each 0 or 1: the tile width of the kernel families
 * rows_r2c, cols_y, cols_filter, rows_c2r, cols_bin (0 the default, 1 half of it), then three
 * schedules (0 the default, 1 the other one): bin_schedule (the +-1 binning pass one tile of one
 * field per workgroup, or persistent with a work counter and the next tile's loads overlapping the
 * binning; default one-per-workgroup in 2D, persistent in 3D), field_placement (the fields of an
 * axis-0 tile on consecutive workgroup ids of one XCD, sharing the tile's bin-table slice in its
 * L2, or field-major; default the former in 2D, the latter in 3D) and y_group (the 3D y passes give
 * groups of 16 or of 4 neighbouring tiles to one XCD); last `radix`, the radix lists of the
 * column passes (y, filter, binning): 0 each length's default Stockham plan, 1 its alternative
 * order of radices where the length has one (256: 16.4.4 for 16.16; 512: 16.8.4 for 8.8.8; 1024:
 * 8.8.16 for 16.8.8; 2048: 16.16.8 for 16.8.16), same elements per thread; then bin_exchange
 * and filter_exchange, the exchange of the axis-0 binning and filter passes: complex values
 * through LDS, or split (real and imaginary parts in two rounds through half the LDS, so more
 * workgroups are resident, at two more barriers per exchange; axis-0 lengths of 192 and more);
 * default the binning pass split in 2D and complex in 3D, the filter pass complex, 1 the other
 * one; last whole_field (2D grids with n_x / 2 in 8 .. 64 and n0 in 16 .. 128, powers of two, whose
 * half spectrum and bins fit in one workgroup's LDS): 1 runs the whole path as one kernel, one
 * workgroup per field, the spectrum never leaving LDS (HBM traffic: the outputs only); and plane
 * (3D grids with n_x / 2 in {16, 24, 32, 48, 64} and n_y in {32, 48, 64, 96, 128}): 1 runs the x
 * and y transforms of each z-plane in one kernel, so noise, the x rows and the forward y pass
 * are one pass and the inverse y pass, the last row pass and the y pass of the +-1 field another.
 * hu_autotune searches
 * the plan of a shape class (grid, bins, batch size bucket) on a synthetic batch of `batch` fields
 * of `dims` with `bins`: after about 50 ms of warm-up runs it flips one entry at a time from the
 * default plan and keeps the change when the summed mean kernel time of the whole pass sequence,
 * timed alternately with the current plan, drops by more than 1 % (the y-pass entries only in 3D,
 * the radix entry only where a column length has an alternative, the exchange entries from
 * axis-0 length 192, whole_field and plane where the grid fits),
 * sweeping the entries a second time when the first sweep changed the plan.  The plan is kept in memory and,
 * if cache_path is non-NULL, all tuned plans are written as JSON there (read back at start-up from
 * $HUFIELD_TUNE_CACHE).  ms_out (host, optional) receives 15 values: the default plan's time and
 * the tuned plan's (timed side by side after the search), and for each entry the time with it
 * flipped during the search (0 where not tried), in ms.  Allocates and frees its own device
 * buffers and synchronises.  The tile-width, schedule and exchange entries leave fields and sign
 * maps the same bit for bit (the spectra to FP64 rounding: the tile width changes how the bins' partials
 * are grouped); the radix, whole_field and plane entries change the FP32 rounding (other transforms,
 * another order of the sums), so fields under them agree with the others to FP32 rounding, not
 * bit for bit. */
int hu_autotune(hu_dims dims, int32_t batch, const hu_bins* bins, const char* cache_path, double* ms_out);

/* The plan (13 entries, 0 or 1, order as above) that calls on this shape class use. */
int hu_plan_query(hu_dims dims, int32_t batch, const hu_bins* bins, int32_t* variants);

/* Set the plan of a shape class by hand (host array of 13 entries, each 0 or 1). */
int hu_plan_set(hu_dims dims, int32_t batch, const hu_bins* bins, const int32_t* variants);

const char* hu_strerror(int code);

/* Raw Philox4x32-10 words and the derived FP32 normals for blocks first .. first+count-1 under
 * `seed` (the noise stream of every entry point).  words [4*count] uint32 and normals
 * [4*count] FP32, either may be NULL.  For parity tests. */
int hu_debug_philox(uint64_t seed, uint64_t first, uint64_t count, uint32_t* words, float* normals,
                    void* stream);

/* The host-built bin tables behind the binned spectra, for tests (host only, no device work).
 * The axis-0 passes see the half spectrum as ncol columns of n0 modes along the slowest axis
 * (column g = m_x in 2D, g = m_y (n_x/2+1) + m_x in 3D; mode e = the natural index along axis 0)
 * and take them in tiles of `width` consecutive columns (tile variant 0 or 1 of those passes).
 *   sizes [6] (host): ncol, n0, ntiles, M (partials per field), nloc_max (most distinct bins in a
 *         tile), width
 *   table [ncol][n0]: bin of each mode (r A + a, the corner slot R A)
 *   ltab  [ncol][n0]: position of the mode's bin in its tile's ascending list of distinct bins
 *   toff  [ntiles + 1]: the partials of tile t are toff[t] .. toff[t+1]-1, one per distinct bin
 *   coff  [R A + 2], cpos [M]: the partials of bin k are cpos[coff[k] .. coff[k+1]-1], tile order
 * Each array may be NULL (host arrays).  A tile's partial is the sum over its modes in that bin,
 * combined in integer arithmetic; a spectrum bin is a fixed-order sum of its partials, so the
 * spectra are the same bits on every run. */
int hu_debug_bin_tables(hu_dims dims, hu_bins bins, int32_t variant, int32_t* sizes, uint16_t* table,
                        uint16_t* ltab, uint32_t* toff, uint32_t* coff, uint32_t* cpos);

/* Kernel timing with HIP events recorded on the launch stream around every kernel the library
 * enqueues.  hu_profile_enable(1) resets the counters and starts recording; hu_profile_read
 * fills up to `cap` entries (host arrays) with each kernel family's name, launch count and
 * summed milliseconds, and returns the number of families.  hu_profile_read synchronises on
 * the recorded events. */
int hu_profile_enable(int on);
int hu_profile_read(char (*names)[48], int64_t* launches, double* total_ms, int cap);

#ifdef __cplusplus
}
#endif

#endif /* HUFIELD_H */
