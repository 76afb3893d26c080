// Row passes along x (the fastest axis) of the hyperuniform-field pipeline.
//
//   rows_r2c   white noise (Philox4x32-10 + Box-Muller) or a real input -> real-to-complex
//              transform of each x row: an n_x/2-point complex FFT of the packed samples
//              x[2n] + i x[2n+1] followed by the split twist;
//   rows_c2r   inverse of that for each x row, then the normalisation of Eq. (15) with the
//              statistics of the filter pass, the FP32 field and the +-1 sign map with counts,
//              and the real-to-complex transform of the +-1 row written back in place.
//
// Half-spectrum layout seen by the row passes: element k of row r sits at
//   (k / TW) * (nrows * TW) + r * TW + (k % TW),
// TW = 4 for 2D grids (column groups of four, so that a 4-column tile of the axis-0 pass and a
// 4-row tile of these passes both move whole 128-byte lines) and TW = n_x/2 + 1 for 3D grids
// (plain row-major).  Global loads and stores of the half spectrum walk this layout in address
// order, decoupled from the FFT's thread mapping, through LDS.
#include "hu_common.hpp"

namespace hu {

template <int L, bool TILED>
struct RowIO {
  static constexpr int TW = TILED ? 4 : L + 1;
  static constexpr int NG = (L + 1 + TW - 1) / TW;   // column groups
};

// R2C split twist of every row of the tile from Z in LDS (padded, natural order) to the half
// spectrum, in address order:
//   X[k] = (Z[k] + Z*[L-k])/2 - (i/2) e^{-2 pi i k / 2L} (Z[k] - Z*[L-k]),  X[L] = Re Z[0] - Im Z[0].
template <int L, int C, int T, bool TILED>
__device__ __forceinline__ void twist_store_rows(const float2* lds, const float2* __restrict__ tw2, float2* spec_f,
                                                 long long row0, int rows_here, long long nrows, int tid) {
  constexpr int TW = RowIO<L, TILED>::TW, NG = RowIO<L, TILED>::NG, RS = Region<L>::value;
  constexpr int PG = C * TW;
  for (int u = tid; u < NG * PG; u += T) {
    const int q = u / PG, w = u - q * PG, cc = w / TW, kk = w - cc * TW;
    const int k = q * TW + kk;
    if (k > L || cc >= rows_here) continue;
    const float2* lz = lds + cc * RS;
    const float2 zk = lz[lidx(k == L ? 0 : k)];
    float2 X;
    if (k == L) {
      X = make_float2(zk.x - zk.y, 0.0f);
    } else {
      const float2 zm = cconj(lz[lidx((L - k) % L)]);
      const float2 A = cadd(zk, zm), B = csub(zk, zm);
      X = cscale(cadd(A, mul_mi<false>(cmul(tw2[k], B))), 0.5f);
    }
    spec_f[((long long)q * nrows + row0 + cc) * TW + kk] = X;
  }
}

// grid (ceil(nrows / C), B), block C * P; thread (c, p) = (tid / P, tid % P) transforms row c.
template <int L, int SRC, bool TILED, int V>
__global__ void __launch_bounds__((RowTile<L, V>::T)) k_rows_r2c(RowsArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = RowTile<L, V>::C, T = RowTile<L, V>::T;
  constexpr int RS = Region<L>::value;
  using Rad = typename Plan<L>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  float* ldsf = reinterpret_cast<float*>(lds);
  const int tid = threadIdx.x;
  const int c = tid / P, p = tid % P;
  const int b = blockIdx.y;
  const long long row0 = (long long)blockIdx.x * C;
  const long long nx = 2 * L;

  if (blockIdx.x == 0) {                        // set up this field's accumulators for later passes
    if (a.io) {
      const FieldIO& io = a.io[b];
      uint32_t* dst[5] = {reinterpret_cast<uint32_t*>(io.cont_sum), reinterpret_cast<uint32_t*>(io.cont_cnt),
                          reinterpret_cast<uint32_t*>(io.pm1_sum), reinterpret_cast<uint32_t*>(io.pm1_cnt),
                          reinterpret_cast<uint32_t*>(io.counts)};
      const uint32_t* src[5] = {nullptr, a.cnt_src, nullptr, a.cnt_src, nullptr};
      const int words[5] = {2 * a.nb, 2 * a.nb, 2 * a.nb, 2 * a.nb, 4};
      for (int s = 0; s < 5; ++s)
        if (dst[s])
          for (int i = tid; i < words[s]; i += T) dst[s][i] = src[s] ? src[s][i] : 0u;
    } else {
      for (int s = 0; s < a.fill_spans; ++s) {
        uint32_t* dst = a.fill[s].dst + (long long)b * a.fill[s].per_field;
        const uint32_t* src = a.fill[s].src;
        for (int i = tid; i < a.fill[s].per_field; i += T) dst[i] = src ? src[i] : 0u;
      }
    }
  }

  // ---- the C real rows into LDS: sample x of row c goes to float 2 lidx(x / 2) + (x & 1) of region c
  const long long v0 = row0 * nx;
  const int rows_here = (int)((a.nrows - row0) < C ? (a.nrows - row0) : C);
  const int nv = rows_here * 2 * L;
  if constexpr (SRC == SRC_NOISE) {
    // voxel i of the field takes normal i mod 4 of Philox block i / 4
    const uint64_t seed = a.io ? a.io[b].seed : a.seeds[b];
    const long long m0 = v0 >> 2, m1 = (v0 + nv + 3) >> 2;
    for (long long m = m0 + tid; m < m1; m += T) {
      float z[4];
      noise4((uint64_t)m, seed, z);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int v = (int)(4 * m + q - v0);
        if (v >= 0 && v < nv) {
          const int rc = v / (2 * L), x = v - rc * (2 * L);
          ldsf[2 * (rc * RS + lidx(x >> 1)) + (x & 1)] = z[q];
        }
      }
    }
  } else {
    const long long base = (long long)b * a.N + v0;
    for (int i = tid; i < C * 2 * L; i += T) {
      float x = 0.0f;
      if (i < nv) {
        if constexpr (SRC == SRC_F32) x = reinterpret_cast<const float*>(a.src)[base + i];
        else x = (float)reinterpret_cast<const int8_t*>(a.src)[base + i];
      }
      const int rc = i / (2 * L), xx = i - rc * (2 * L);
      ldsf[2 * (rc * RS + lidx(xx >> 1)) + (xx & 1)] = x;
    }
  }
  __syncthreads();

  float2 v[E];
  float2* lrow = lds + c * RS;
  stage_load<L, R1, P, E>(v, lrow, p);
  fft_run<L, P, E, false>(Rad{}, v, lrow, p, a.tw);
  __syncthreads();
  slot_store<L, RL, P, E>(v, lrow, p);
  __syncthreads();
  twist_store_rows<L, C, T, TILED>(lds, a.tw2, a.spec + (long long)b * a.Nh, row0, rows_here, a.nrows, tid);
}

// C2R along x -> normalise -> field, sign map, counts -> R2C of the +-1 row (THRESH).
template <int L, bool THRESH, bool TILED, int V>
__global__ void __launch_bounds__((RowTile<L, V>::T)) k_rows_c2r(RowsZArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = RowTile<L, V>::C, T = RowTile<L, V>::T;
  constexpr int RS = Region<L>::value;
  constexpr int TW = RowIO<L, TILED>::TW, NG = RowIO<L, TILED>::NG, PG = C * TW;
  using Rad = typename Plan<L>::fwd;
  using RadF = Reverse<Rad>;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  __shared__ unsigned red_u[2][T / 64 > 0 ? T / 64 : 1];
  const int tid = threadIdx.x;
  const int c = tid / P, p = tid % P;
  const int b = blockIdx.y;
  const long long row0 = (long long)blockIdx.x * C;
  const int rows_here = (int)((a.nrows - row0) < C ? (a.nrows - row0) : C);
  float2* lrow = lds + c * RS;
  float2* spec_f = a.spec + (long long)b * a.Nh;

  // ---- the tile's half rows X[0..L] into LDS, in address order; X[0] and X[L] are real after
  //      the other axes' inverse transforms
  for (int u = tid; u < NG * PG; u += T) {
    const int q = u / PG, w = u - q * PG, cc = w / TW, kk = w - cc * TW;
    const int k = q * TW + kk;
    if (k > L) continue;
    float2 x = cc < rows_here ? spec_f[((long long)q * a.nrows + row0 + cc) * TW + kk] : make_float2(0.f, 0.f);
    if (k == 0 || k == L) x.y = 0.0f;
    lds[cc * RS + lidx(k)] = x;
  }
  __syncthreads();
  // ---- pre-twist: Z[k] = (X[k] + X*[L-k]) + i e^{+2 pi i k / 2L} (X[k] - X*[L-k])
  float2 v[E];
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int k = slot_index<L, R1, P>(s, p);
    const float2 xk = lrow[lidx(k)], xc = cconj(lrow[lidx(L - k)]);
    v[s] = cadd(cadd(xk, xc), mul_mi<true>(cmul(cconj(a.tw2[k]), csub(xk, xc))));
  }
  fft_run<L, P, E, true>(Rad{}, v, lrow, p, a.tw);

  // ---- normalise (Eq. (15)); stage the field in LDS (rows contiguous, unpadded)
  const double* fs = a.fstats + (long long)b * 8;
  const float scale = (float)fs[4], offset = (float)fs[5];
  float* stage = reinterpret_cast<float*>(lds);
  __syncthreads();                               // exchange buffer free
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int n = slot_index<L, RL, P>(s, p);
    const float x0 = fmaf(v[s].x, scale, offset);
    const float x1 = fmaf(v[s].y, scale, offset);
    *reinterpret_cast<float2*>(stage + c * 2 * L + 2 * n) = make_float2(x0, x1);
    if constexpr (THRESH) v[s] = make_float2(x0 >= 0.0f ? 1.0f : -1.0f, x1 >= 0.0f ? 1.0f : -1.0f);
  }
  __syncthreads();
  // ---- field and sign map out, 4 voxels (16 B of field, 4 B of map) per unit
  float* fout = a.io ? a.io[b].field : field_ptr(a.field, a.N, b);
  int8_t* tout = a.io ? a.io[b].pm1 : field_ptr(a.pm1, a.N, b);
  uint64_t* cout = a.io ? a.io[b].counts : field_ptr(a.counts, 2, b);
  const float near_tol = a.io ? a.io[b].near_abs : a.near_tol;
  const long long gbase = row0 * 2 * L;
  const int nq = rows_here * L / 2;              // units of 4 voxels in the tile
  unsigned npos = 0, nnear = 0;
  for (int u = tid; u < nq; u += T) {
    const float4 f4 = *reinterpret_cast<const float4*>(stage + 4 * u);
    if (fout) *reinterpret_cast<float4*>(fout + gbase + 4 * u) = f4;
    if constexpr (THRESH) {
      const float xs[4] = {f4.x, f4.y, f4.z, f4.w};
      uint32_t packed = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool pos = xs[q] >= 0.0f;
        npos += pos;
        nnear += fabsf(xs[q]) < near_tol;
        packed |= (uint32_t)(pos ? 0x01u : 0xFFu) << (8 * q);
      }
      if (tout) *reinterpret_cast<uint32_t*>(tout + gbase + 4 * u) = packed;
    }
  }
  // tail (rows of 6 voxels): the last rows_here * 2L mod 4 samples one by one
  for (int i = 4 * nq + tid; i < rows_here * 2 * L; i += T) {
    const float x = stage[i];
    if (fout) fout[gbase + i] = x;
    if constexpr (THRESH) {
      npos += x >= 0.0f;
      nnear += fabsf(x) < near_tol;
      if (tout) tout[gbase + i] = x >= 0.0f ? (int8_t)1 : (int8_t)-1;
    }
  }
  if constexpr (THRESH) {
    npos = wave_usum(npos);
    nnear = wave_usum(nnear);
    if ((tid & 63) == 0) { red_u[0][tid >> 6] = npos; red_u[1][tid >> 6] = nnear; }
    // forward transform of the packed +-1 row (its first radix is the inverse's last)
    fft_run<L, P, E, false>(RadF{}, v, lrow, p, a.tw);
    __syncthreads();
    constexpr int RLF = RadInfo<RadF>::last;
    slot_store<L, RLF, P, E>(v, lrow, p);
    __syncthreads();
    twist_store_rows<L, C, T, TILED>(lds, a.tw2, spec_f, row0, rows_here, a.nrows, tid);
    if (tid == 0 && cout) {
      unsigned long long np = 0, nn = 0;
      for (int w = 0; w < (T + 63) / 64; ++w) { np += red_u[0][w]; nn += red_u[1][w]; }
      atomicAdd((unsigned long long*)(cout + 0), np);
      atomicAdd((unsigned long long*)(cout + 1), nn);
    }
  }
}

#define HU_ROW_LENGTHS(X) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(1024)

static inline unsigned ceil_div_u(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

template <int L, int SRC, bool TILED, int V>
static hipError_t launch_rows_r2c_L(const RowsArgs& a, int batch, hipStream_t st) {
  constexpr int C = RowTile<L, V>::C, T = RowTile<L, V>::T;
  dim3 grid(ceil_div_u(a.nrows, C), batch);
  hipLaunchKernelGGL((k_rows_r2c<L, SRC, TILED, V>), grid, dim3(T), (size_t)C * Region<L>::value * sizeof(float2), st,
                     a);
  return hipGetLastError();
}

template <int L, int SRC>
static hipError_t launch_rows_r2c_S(int variant, const RowsArgs& a, int batch, hipStream_t st) {
  if (variant)
    return a.tiled ? launch_rows_r2c_L<L, SRC, true, 1>(a, batch, st) : launch_rows_r2c_L<L, SRC, false, 1>(a, batch, st);
  return a.tiled ? launch_rows_r2c_L<L, SRC, true, 0>(a, batch, st) : launch_rows_r2c_L<L, SRC, false, 0>(a, batch, st);
}

hipError_t launch_rows_r2c(int L, int src, int variant, const RowsArgs& a, int batch, hipStream_t st) {
  switch (L) {
#define X(LL)                                                                                 \
  case LL:                                                                                    \
    if (src == SRC_NOISE) return launch_rows_r2c_S<LL, SRC_NOISE>(variant, a, batch, st);     \
    if (src == SRC_F32) return launch_rows_r2c_S<LL, SRC_F32>(0, a, batch, st);               \
    return launch_rows_r2c_S<LL, SRC_I8>(0, a, batch, st);
    HU_ROW_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

template <int L, bool THRESH, bool TILED, int V>
static hipError_t launch_rows_c2r_L(const RowsZArgs& a, int batch, hipStream_t st) {
  constexpr int C = RowTile<L, V>::C, T = RowTile<L, V>::T;
  dim3 grid(ceil_div_u(a.nrows, C), batch);
  hipLaunchKernelGGL((k_rows_c2r<L, THRESH, TILED, V>), grid, dim3(T), (size_t)C * Region<L>::value * sizeof(float2),
                     st, a);
  return hipGetLastError();
}

template <int L, int V>
static hipError_t launch_rows_c2r_V(bool thresh, const RowsZArgs& a, int batch, hipStream_t st) {
  if (a.tiled)
    return thresh ? launch_rows_c2r_L<L, true, true, V>(a, batch, st) : launch_rows_c2r_L<L, false, true, V>(a, batch, st);
  return thresh ? launch_rows_c2r_L<L, true, false, V>(a, batch, st) : launch_rows_c2r_L<L, false, false, V>(a, batch, st);
}

hipError_t launch_rows_c2r(int L, bool thresh, int variant, const RowsZArgs& a, int batch, hipStream_t st) {
  switch (L) {
#define X(LL) \
  case LL: return variant ? launch_rows_c2r_V<LL, 1>(thresh, a, batch, st) : launch_rows_c2r_V<LL, 0>(thresh, a, batch, st);
    HU_ROW_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hu
