// Kernel argument blocks and launcher declarations shared by the kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hu_device.hpp"

namespace hu {

enum { SRC_NOISE = 0, SRC_F32 = 1, SRC_I8 = 2 };
constexpr int MAX_CHUNK = 64;   // fields per launch (seeds travel in the kernel arguments)

struct ZeroSpan {
  uint32_t* ptr;    // first word of field 0
  int per_field;    // 32-bit words per field
};

struct RowsArgs {
  float2* spec;            // half spectrum, [B][Nh]
  long long Nh, N, nrows;  // per field
  uint64_t seeds[MAX_CHUNK];
  const void* src;         // real input for the load variants, [B][N]
  const float2* tw;        // exp(-2 pi i t / L), t < L
  const float2* tw2;       // exp(-2 pi i k / 2L), k < L
  ZeroSpan zero[6];
  int zero_spans;
};

struct ColsArgs {
  float2* spec;
  long long Nh;
  long long ncol;          // transforms per field
  long long inner;         // element stride (complex) along the axis
  const float2* tw;
};

struct Axis0Geom {
  int ndim;
  int n0;                  // length of axis 0
  int ny;                  // n_y (3D)
  int nx, nxh;
  long long ncol;          // Nh / n0
  long long dfac_0, dfac_y, dfac_x;   // D / n_i, D = lcm of the dims
};

struct FilterArgs {
  float2* spec;
  long long Nh, N;
  Axis0Geom gm;
  FiltDev filt;
  BinDev bd;
  int nb;                  // bins + 1 (corner slot)
  const float2* tw;
  double* partials;        // [B][tiles][4]
  unsigned* counters;      // [B]
  double* fstats;          // [B][8] mu, var, max ln chi, flag, scale, offset, spectrum factor, G
  double* stats;           // [B][4] user copy or null
  double* cont_sum;        // [B][nb] or null
  uint64_t* cont_cnt;
  double sigma_f;
};

struct BinArgs {
  const float2* spec;
  long long Nh, N;
  Axis0Geom gm;
  BinDev bd;
  int nb;
  const float2* tw;
  double* sum;
  uint64_t* cnt;
};

struct RowsZArgs {
  float2* spec;
  long long Nh, N, nrows;
  const float2* tw;
  const float2* tw2;
  const double* fstats;
  float* field;
  int8_t* pm1;
  uint64_t* counts;
  float near_tol;          // absolute
};

struct ThreshArgs {
  const float* field;
  int8_t* out;
  uint64_t* counts;
  long long N;
  float near_tol;
};

hipError_t launch_rows_r2c(int L, int src, const RowsArgs& a, int batch, hipStream_t st);
hipError_t launch_cols(int L, bool inv, const ColsArgs& a, int batch, hipStream_t st);
hipError_t launch_cols_filter(int L, const FilterArgs& a, int batch, hipStream_t st);
hipError_t launch_cols_bin(int L, const BinArgs& a, int batch, hipStream_t st);
hipError_t launch_rows_c2r(int L, bool thresh, const RowsZArgs& a, int batch, hipStream_t st);
hipError_t launch_threshold(const ThreshArgs& a, int batch, hipStream_t st);
hipError_t launch_zero_u64(uint64_t* p, long long n, hipStream_t st);
hipError_t launch_debug_philox(uint64_t seed, uint64_t first, uint64_t count, uint32_t* words, float* normals,
                               hipStream_t st);
int col_tiles(int L, long long ncol);

}  // namespace hu
