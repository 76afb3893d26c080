// Kernel argument blocks and launcher declarations shared by the kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hu_device.hpp"
#include "hufield.h"

namespace hu {

// lengths whose axis-0 filter and binning passes are compiled with the split exchange too
// (shorter columns have small exchange buffers)
constexpr bool split_length(int L) { return L >= 192; }


enum { SRC_NOISE = 0, SRC_F32 = 1, SRC_I8 = 2 };
constexpr int MAX_CHUNK = 64;   // fields per launch when seeds travel in the kernel arguments
// fields per launch of the whole-field kernel, which needs no workspace: enough to give every CU
// a field (its arguments stay under the 4 KB kernel-argument limit)
constexpr int MAX_WHOLE_CHUNK = 256;
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
  int nb;                  // with io: bins + 1, for the per-field bin counts
  const uint32_t* cnt_src; // with io: precomputed bin counts (nb uint64)
  const void* src;         // real input for the load variants, [B][N]
  const float2* tw;        // stage twiddle table of the row length (StageTab layout)
  const float2* tw2;       // exp(-2 pi i k / 2L), k < L
  FillSpan fill[6];
  int fill_spans;
  unsigned* zero;          // words cleared by block (0, 0) before the later passes read them
  int nzero;               // (the work counter of the persistent binning pass)
  const float2* tw_y;      // plane kernels (3D): stage table of n_y
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

// The whole path of small 2D fields, one workgroup per field (hu_small.hip).  Uniform mode
// (io null): seeds, filter and outputs at base + field * stride; batch mode: io[b].
struct SmallArgs {
  uint64_t seeds[MAX_WHOLE_CHUNK];
  const FieldIO* io;
  FiltDev filt;
  double sigma_f;
  float near_abs;
  int thresh, want_cont, want_pm1, any_gen;
  int nb;                  // bins + 1 (0: no spectra)
  long long N;
  Axis0Geom gm;
  float* field;
  int8_t* pm1;
  double* stats;
  uint64_t* counts;
  double* cont_sum;
  uint64_t* cont_cnt;
  double* pm1_sum;
  uint64_t* pm1_cnt;
  const uint16_t* table;                   // [n_x/2 + 1][n0] bin of each mode
  const unsigned long long* counts_tab;    // [nb] modes per bin
  const float2* tw_row;                    // stage table of n_x / 2
  const float2* tw2;                       // exp(-2 pi i k / n_x), k < n_x / 2
  const float2* tw_col;                    // stage table of n0
};


// Tile-local bin tables of the axis-0 passes for one tile width.  The modes of a tile touch few of
// the bins; each tile has one partial sum per distinct bin (in ascending bin order), stored grouped
// by bin so that a bin's partials are contiguous, and the partials of a bin are combined in a
// fixed order: the binned spectra are the same bits on every run.
struct TileBinDev {
  const uint16_t* ltab;    // [ncol][n0]: position of the mode's bin in its tile's list of distinct bins
  const uint32_t* toff;    // [ntiles + 1]: partials i = toff[t] .. toff[t+1]-1 belong to tile t
  const uint32_t* wpos;    // [M]: where partial i is stored: grouped by bin, tile order inside a bin
  const uint32_t* coff;    // [nb + 1]: the stored partials of bin k are coff[k] .. coff[k+1]-1
  int nloc_max;            // most distinct bins in one tile
  int M;                   // partials per field
  int sym;                 // radial bins only: modes e and n0 - e of a column share their bin
};

// Dynamic schedule of the persistent binning pass: the items (tile, field), tile-major, are
// taken in chunks (shrinking towards the end) from a counter that the first pass of the same
// launch sequence cleared.
struct ItemQueue {
  unsigned* counter;
  int nitems;              // ntiles * batch
  int chunk_max;
};

struct FilterArgs {
  ColSched sc;
  float2* spec;
  long long Nh, N;
  Axis0Geom gm;
  FiltDev filt;
  const FieldIO* io;       // per-field filter (batch path) or null
  TileBinDev tb;
  double* parts;           // [B][M] tile partials of the continuous-spectrum bins, or null (no bins)
  const float2* tw;        // stage twiddle table of the axis length (StageTab layout)
  double* partials;        // [B][tiles][4]: sum w |F|^2, Re F(0), max ln chi
  int hx_off, hq_off;      // LDS byte offsets of the tile histogram (set by the launcher)
  int any_gen;             // some field uses a tabulated radial form or the FP64 filter evaluation
};

struct FinalizeArgs {
  const double* partials;  // [B][ntiles][4]
  int ntiles;
  long long N;
  double sigma_f;
  double* fstats;          // [B][8] mu, var, max ln chi, flag, scale, offset, spectrum factor, G
  double* stats;           // [B][4] user copy or null
  const FieldIO* io;
};

struct BinArgs {
  int ntiles, batch;
  int persistent;          // 1: persistent over the items of q; 0: one item per workgroup (sc)
  ItemQueue q;
  ColSched sc;
  const float2* spec;
  long long Nh;
  Axis0Geom gm;
  TileBinDev tb;
  double* parts;           // [B][M] tile partials of the bins of sum w |X|^2
  const float2* tw;        // stage twiddle table of the axis length (StageTab layout)
  int hx_off, hq_off;      // LDS byte offsets of the tile histogram (set by the launcher)
};

// Per-field spectra from the tile partials (each bin summed over its tiles in tile order) and the
// per-field sign counts from the last row pass's per-tile counts.
struct SpecFinalArgs {
  int nb;
  const uint32_t* coff_c;  // continuous spectrum: bin ranges of the filter pass's tile width, or null
  const double* parts_c;   // [B][M_c]
  int M_c;
  const double* fstats;    // [B][8]: entry 6 turns raw sums into the normalised field's spectrum
  double* cont_sum;        // [B][nb] (uniform path) or null
  const uint32_t* coff_p;  // +-1 (or input) spectrum: bin ranges of the binning pass's tile width, or null
  const double* parts_p;   // [B][M_p]
  int M_p;
  double pscale;           // 1 / N
  double* pm1_sum;         // [B][nb] (uniform path) or null
  const uint32_t* cpart;   // [B][ntc][2]: n_pos, n_near of each row tile, or null
  int ntc;
  uint64_t* counts;        // [B][2] (uniform path) or null
  const FieldIO* io;       // per-field outputs (batch path) or null
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
  const float2* tw_y;      // plane kernels (3D): stage table of n_y
  int pm1_spec;            // plane kernels: transform the +-1 plane for its spectrum
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

// spectrum-matching loss over the bins r >= 1 with modes (the DC row and the corner slot excluded)
struct LossArgs {
  const double* sum;       // [nb]: the field's normalised continuous-spectrum bin sums
  const uint64_t* cnt;     // [nb]: its mode counts
  const double* tsum;      // [nb]: the target spectrum's bin sums
  const uint64_t* tcnt;    // [nb]: the target's mode counts
  int nb, na;              // slots incl. the corner slot; angular bins per radius
  double eps;              // added to both bin means inside the logs
  double* loss;            // [1] out
  double* dL_dP;           // [nb] out: dL / d(bin mean), 0 for the bins not used
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
  double* sum;             // [nb] output: expected bin sums
  double* partials;        // [gridDim.x]: per-workgroup sum of w H^2
  double* rows;            // [gridDim.x][nb]: per-workgroup bin sums of w H^2
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
hipError_t launch_spectrum_loss(const LossArgs& a, hipStream_t st);
hipError_t launch_grad_final(const GradFinalArgs& a, hipStream_t st);
hipError_t launch_filter_spectrum(const FilterSpecArgs& a, hipStream_t st);
hipError_t launch_rows_r2c(int L, int src, int variant, const RowsArgs& a, int batch, hipStream_t st);
// radix: the alternative radix list of L where it has one (Plan<L, 1>)
hipError_t launch_cols(int L, bool inv, int variant, const ColsArgs& a, hipStream_t st, int radix = 0);
// split: the split exchange (real and imaginary parts in two rounds, half the LDS), lengths >= 192
hipError_t launch_cols_filter(int L, int variant, const FilterArgs& a, hipStream_t st, int radix = 0, int split = 0);
// columns per tile of the axis-0 passes with tile variant `variant`
int col_width(int L, int variant);
hipError_t launch_finalize(const FinalizeArgs& a, int batch, hipStream_t st);
hipError_t launch_cols_bin(int L, int variant, const BinArgs& a, hipStream_t st, int radix = 0, int split = 0);
hipError_t launch_rows_c2r(int L, bool thresh, int variant, const RowsZArgs& a, int batch, hipStream_t st);
int row_tiles(int L, int variant, long long nrows);
hipError_t launch_spec_final(const SpecFinalArgs& a, int batch, hipStream_t st);
// the whole-field kernel for row half-length LR (8 .. 64) and n0 (16 .. 128), powers of two;
// small_lds_bytes: its LDS for nb bins (0 for an unsupported shape)
size_t small_lds_bytes(int LR, int N0, int nb);
// the plane kernels of 3D grids (hu_plane.hip) for row half-length LR and n_y = NY; their LDS (0:
// no instantiation for the shape); grid (n0 planes, batch)
size_t plane_lds_bytes(int LR, int NY);
hipError_t launch_plane_fwd(int LR, int NY, const RowsArgs& a, int n0, int batch, hipStream_t st);
hipError_t launch_plane_inv(int LR, int NY, const RowsZArgs& a, bool thresh, int n0, int batch, hipStream_t st);
hipError_t launch_field_lds(int LR, int N0, const SmallArgs& a, int batch, hipStream_t st);
hipError_t launch_threshold(const ThreshArgs& a, int batch, hipStream_t st);
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
