// Kernel argument blocks and launcher declarations shared by the kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hu_device.hpp"
#include "hufield.h"

namespace hu {

enum { SRC_NOISE = 0, SRC_F32 = 1, SRC_I8 = 2 };
constexpr int MAX_CHUNK = 64;   // fields per launch when seeds travel in the kernel arguments
constexpr int NVARIANT = 2;     // tile-width variants per kernel: 0 = default, 1 = half width

// Per-field parameters and outputs of a heterogeneous batch, in device memory.  When a kernel's
// `io` pointer is set, field b takes everything below from io[b] instead of the uniform kernel
// arguments (base pointer + b * stride).
struct FieldIO {
  float* field;            // [N] or null
  int8_t* pm1;             // [N] or null
  double* stats;           // [4] or null
  uint64_t* counts;        // [2] or null
  double* cont_sum;        // [nb] or null
  uint64_t* cont_cnt;      // [nb] or null
  double* pm1_sum;         // [nb] or null
  uint64_t* pm1_cnt;       // [nb] or null
  uint64_t seed;
  double sigma_f;
  float near_abs;          // absolute near-zero tolerance for the count
  int pad;
  FiltDev filt;
};

// Accumulator set-up done by block 0 of each field in the first pass: dst[b * per_field + i] is
// set to src[i] (the same per-field block for every field, e.g. precomputed bin counts) or 0.
struct FillSpan {
  uint32_t* dst;
  const uint32_t* src;
  int per_field;    // 32-bit words per field
};

// Column-pass schedule: ntiles tiles per field, padded to a multiple of G (tiles sharing a
// 128-byte line), for `batch` fields; grid = ceil(batch * ntiles_pad / (8 G)) * 8 G workgroups.
struct ColSched {
  int ntiles, ntiles_pad, G, batch;
  int finner;              // 1: the fields of one tile are consecutive (G = batch, same XCD)
};

struct RowsArgs {
  float2* spec;            // half spectrum, [B][Nh] (Nh: per-field stride, padded layout)
  long long Nh, N, nrows;  // per field
  int tiled;               // 2D column-group layout (TW = 4) or row-major (3D)
  uint64_t seeds[MAX_CHUNK];
  const FieldIO* io;       // per-field seeds and accumulators (batch path) or null
  int nb;                  // with io: bins + 1, for clearing the per-field spectra
  const uint32_t* cnt_src; // with io: precomputed bin counts (nb uint64)
  const void* src;         // real input for the load variants, [B][N]
  const float2* tw;        // stage twiddle table of the row length (StageTab layout)
  const float2* tw2;       // exp(-2 pi i k / 2L), k < L
  FillSpan fill[6];
  int fill_spans;
};

struct ColsArgs {
  ColSched sc;
  float2* spec;
  long long Nh;
  int ncol;                // transforms per field
  int inner;               // element stride (complex) along the axis
  const float2* tw;        // stage twiddle table of the axis length (StageTab layout)
};

struct Axis0Geom {
  int ndim;
  int n0;                  // length of axis 0
  int ny;                  // n_y (3D)
  int nx, nxh;
  int ncol;                // columns of the axis-0 passes (n_x/2+1 in 2D, n_y (n_x/2+1) in 3D)
  int inner0;              // element stride along axis 0: 4 (2D column groups) or ncol (3D)
  float kap0, kapy, kapx;  // 2 / n_i: wavenumber step in Nyquist units
  long long dfac_0, dfac_y, dfac_x;   // D / n_i, D = lcm of the dims
};

struct FilterArgs {
  ColSched sc;
  float2* spec;
  long long Nh, N;
  Axis0Geom gm;
  FiltDev filt;
  const FieldIO* io;       // per-field filter and continuous-spectrum output (batch path) or null
  BinDev bd;
  int nb;                  // bins + 1 (corner slot)
  const uint16_t* table;   // bin of each mode, [ncol][n0], or null (computed)
  const float2* tw;        // stage twiddle table of the axis length (StageTab layout)
  double* partials;        // [B][tiles][4]: sum w |F|^2, Re F(0), max ln chi
  double* cont_sum;        // [B][nb] raw sums of w |F|^2, or null (counts are filled from the geometry)
  int want_bins;           // accumulate the continuous spectrum (LDS sized for it)
  int any_gen;             // some field uses a tabulated radial form or the FP64 filter evaluation
};

struct FinalizeArgs {
  const double* partials;  // [B][ntiles][4]
  int ntiles;
  long long N;
  double sigma_f;
  double* fstats;          // [B][8] mu, var, max ln chi, flag, scale, offset, spectrum factor, G
  double* stats;           // [B][4] user copy or null
  double* cont_sum;        // [B][nb] rescaled in place, or null
  int nb;
  const FieldIO* io;
};

struct BinArgs {
  ColSched sc;             // tiles per field and fields (the launch is persistent over them)
  const float2* spec;
  long long Nh, N;
  Axis0Geom gm;
  BinDev bd;
  int nb;
  const uint16_t* table;
  const float2* tw;        // stage twiddle table of the axis length (StageTab layout)
  double* sum;
  const FieldIO* io;       // per-field +-1 spectrum output (batch path) or null
  int hs_off;              // LDS byte offset of the histogram (set by the launcher)
};

struct BinGeomArgs {
  long long Nh;
  Axis0Geom gm;
  BinDev bd;
  int nb;
  uint16_t* table;         // [ncol][n0] or null
  unsigned long long* counts;   // [nb], zeroed before the launch
};

struct RowsZArgs {
  float2* spec;
  long long Nh, N, nrows;
  int tiled;
  const float2* tw;        // stage twiddle table of the axis length (StageTab layout)
  const float2* tw2;
  const double* fstats;
  float* field;
  int8_t* pm1;
  uint32_t* cpart;         // [B][row tiles][2]: n_pos, n_near of each tile (THRESH), or null
  float near_tol;          // absolute
  const FieldIO* io;       // per-field outputs (batch path) or null
};

// per-field totals of the last row pass's per-tile counts
struct CountFinalArgs {
  const uint32_t* cpart;   // [B][ntiles][2]
  int ntiles;
  uint64_t* counts;        // [B][2] (plain path) or null
  const FieldIO* io;       // per-field outputs (batch path) or null
};

struct ThreshArgs {
  const float* field;
  int8_t* out;
  uint64_t* counts;
  long long N;
  float near_tol;
  float level;             // +1 where field >= level (0: the sign map)
};

struct SquareArgs {
  ColSched sc;
  float2* spec;            // transformed along every axis but axis 0, [B][Nh]; rewritten in place
  long long Nh, N;
  Axis0Geom gm;
  const float2* tw;        // stage twiddle table of the axis length (StageTab layout)
  double* fstats;          // [B][8]: entries 4 and 5 (scale, offset of the last row pass) written
};

// Adjoint of the filter with respect to theta = (a, b, c, p, rot, k0, w): the axis-0 pass over the
// noise spectrum W, with the per-bin loss weights omega(k) = coef[b(k)] - coef[nb].
struct AdjointArgs {
  int ntiles;              // column tiles of the axis-0 pass
  const float2* spec;      // W transformed along every axis but axis 0, [Nh]
  long long Nh;
  Axis0Geom gm;
  FiltDev filt;
  float width;             // w (the Gaussian band width)
  BinDev bd;
  int nb;
  const uint16_t* table;   // bin of each mode or null
  const float2* tw;        // stage twiddle table of the axis length (StageTab layout)
  const double* coef;      // [nb + 1]: beta_b per bin, then gamma
  double* partials;        // [workgroups][8]: the 7 gradient partial sums
  int cf_off;              // LDS byte offset of the per-bin weights (set by the launcher)
};

struct GradCoefArgs {
  const double* dL_dP;     // [nb]: d loss / d (bin mean)
  const double* cont_sum;  // [nb]: forward's normalised continuous-spectrum bin sums
  const uint64_t* cont_cnt;   // [nb]: mode counts
  const double* stats;     // [4]: forward's mu, var (raw field)
  int nb;                  // slots incl. the corner slot (not part of the spectrum)
  long long N;
  double sigma_f;
  double* coef;            // [nb + 1] out
};

struct GradFinalArgs {
  const double* partials;  // [rows][8]
  int ntiles;              // rows
  double* grad;            // [7] out
};

struct FilterSpecArgs {
  long long Nh;            // modes (ncol * n0)
  Axis0Geom gm;
  FiltDev filt;
  BinDev bd;
  int nb;
  const uint16_t* table;
  double* sum;             // [nb] raw sums of w H^2 (zeroed before the launch)
  double* partials;        // [gridDim.x]: per-block sum of w H^2
  int nblocks;
  long long N;
  double sigma_f;
  const unsigned long long* counts;   // [nb] geometry counts, copied to cnt
  uint64_t* cnt;           // [nb] out or null
};

struct WvarArgs {
  ColSched sc;
  const float2* spec;      // transformed along every axis but axis 0, [B][Nh]
  long long Nh;
  Axis0Geom gm;
  const float2* tw;        // stage twiddle table of the axis length (StageTab layout)
  int nr;                  // radii (1..HU_MAX_RADII)
  float radii[HU_MAX_RADII];
  double* partials;        // [B][tiles][nr]
};

struct WvarFinalArgs {
  const double* partials;  // [B][ntiles][nr]
  int ntiles, nr;
  double scale;            // 1 / N^2
  double* out;             // [B][nr]
};

hipError_t launch_cols_square(int L, const SquareArgs& a, hipStream_t st);
hipError_t launch_cols_wvar(int L, const WvarArgs& a, hipStream_t st);
hipError_t launch_wvar_final(const WvarFinalArgs& a, int batch, hipStream_t st);
hipError_t launch_cols_adjoint(int L, const AdjointArgs& a, hipStream_t st, int* grid);
// workgroups of a kernel with this block size and LDS that are resident on the current device at
// once (cached per device, kernel and LDS size)
hipError_t resident_blocks(const void* kern, int threads, size_t lds, int* slots);
hipError_t launch_grad_coef(const GradCoefArgs& a, hipStream_t st);
hipError_t launch_grad_final(const GradFinalArgs& a, hipStream_t st);
hipError_t launch_filter_spectrum(const FilterSpecArgs& a, hipStream_t st);
hipError_t launch_rows_r2c(int L, int src, int variant, const RowsArgs& a, int batch, hipStream_t st);
hipError_t launch_cols(int L, bool inv, int variant, const ColsArgs& a, hipStream_t st);
hipError_t launch_cols_filter(int L, int variant, const FilterArgs& a, hipStream_t st);
hipError_t launch_finalize(const FinalizeArgs& a, int batch, hipStream_t st);
hipError_t launch_cols_bin(int L, int variant, const BinArgs& a, hipStream_t st);
hipError_t launch_rows_c2r(int L, bool thresh, int variant, const RowsZArgs& a, int batch, hipStream_t st);
int row_tiles(int L, int variant, long long nrows);
hipError_t launch_count_final(const CountFinalArgs& a, int batch, hipStream_t st);
hipError_t launch_threshold(const ThreshArgs& a, int batch, hipStream_t st);
hipError_t launch_bin_geom(const BinGeomArgs& a, hipStream_t st);
// `group` tiles in a row per XCD (see ColSched)
ColSched col_sched(int L, int variant, long long ncol, int batch, int group = 1);
ColSched col_sched_fields(int L, int variant, long long ncol, int batch);
// tile group of the 3D y passes: their columns run over x rows of n_x / 2 + 1 complex values,
// which do not start on 128-byte lines, so neighbouring tiles share lines
constexpr int Y_PASS_GROUP = 16;
hipError_t launch_zero_u64(uint64_t* p, long long n, hipStream_t st);
hipError_t launch_debug_philox(uint64_t seed, uint64_t first, uint64_t count, uint32_t* words, float* normals,
                               hipStream_t st);
int col_tiles(int L, int variant, long long ncol);

}  // namespace hu
