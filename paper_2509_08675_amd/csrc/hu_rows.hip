// Row passes along x (the fastest axis) of the hyperuniform-field pipeline.
//
//   rows_r2c   white noise (Philox4x32-10 + Box-Muller) or a real input -> real-to-complex
//              transform of each x row: an n_x/2-point complex FFT of the packed samples
//              x[2n] + i x[2n+1] followed by the split twist;
//   rows_c2r   inverse of that for each x row, then the normalisation of Eq. (15) with the
//              statistics of the filter pass, the FP32 field and the +-1 sign map with counts,
//              and the real-to-complex transform of the +-1 row written back in place.
#include "hu_common.hpp"

namespace hu {

// grid (ceil(nrows / C), B), block C * P; thread (c, p) = (tid / P, tid % P) works on row c.
template <int L, int SRC>
__global__ void __launch_bounds__(RowTile<L>::T) k_rows_r2c(RowsArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = RowTile<L>::C, T = RowTile<L>::T;
  using Rad = typename Plan<L>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  constexpr int RS = Region<L>::value;
  extern __shared__ float2 lds[];
  float* ldsf = reinterpret_cast<float*>(lds);
  const int tid = threadIdx.x;
  const int c = tid / P, p = tid % P;
  const int b = blockIdx.y;
  const long long row0 = (long long)blockIdx.x * C;
  const long long row = row0 + c;
  const bool valid = row < a.nrows;
  const long long nx = 2 * L;

  if (blockIdx.x == 0) {                        // set up this field's accumulators for later passes
    for (int s = 0; s < a.fill_spans; ++s) {
      uint32_t* dst = a.fill[s].dst + (long long)b * a.fill[s].per_field;
      const uint32_t* src = a.fill[s].src;
      for (int i = tid; i < a.fill[s].per_field; i += T) dst[i] = src ? src[i] : 0u;
    }
  }

  // ---- the C real rows into LDS: sample x of row c goes to float 2 lidx(x / 2) + (x & 1) of region c
  const long long v0 = row0 * nx;
  const long long rows_here = (a.nrows - row0) < C ? (a.nrows - row0) : C;
  const int nv = (int)(rows_here * nx);
  if constexpr (SRC == SRC_NOISE) {
    // voxel i of the field takes normal i mod 4 of Philox block i / 4
    const uint64_t seed = a.seeds[b];
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
#pragma unroll
  for (int s = 0; s < E; ++s) v[s] = lrow[lidx(slot_index<L, R1, P>(s, p))];
  fft_run<L, P, E, false>(Rad{}, v, lrow, p, a.tw);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < E; ++s) lrow[lidx(slot_index<L, RL, P>(s, p))] = v[s];
  __syncthreads();
  float2* out = a.spec + (long long)b * a.Nh + row * (L + 1);
  r2c_twist_store<L, P, E>(lrow, a.tw2, out, p, valid);
}

// C2R along x -> normalise -> field, sign map, counts -> R2C of the +-1 row (THRESH).
template <int L, bool THRESH>
__global__ void __launch_bounds__(RowTile<L>::T) k_rows_c2r(RowsZArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = RowTile<L>::C, T = RowTile<L>::T;
  using Rad = typename Plan<L>::fwd;
  using RadF = Reverse<Rad>;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  constexpr int LS = L + 1;
  constexpr int RS = Region<L>::value;
  extern __shared__ float2 lds[];
  __shared__ unsigned red_u[2][T / 64 > 0 ? T / 64 : 1];
  const int tid = threadIdx.x;
  const int c = tid / P, p = tid % P;
  const int b = blockIdx.y;
  const long long row = (long long)blockIdx.x * C + c;
  const bool valid = row < a.nrows;
  float2* lrow = lds + c * RS;
  float2* srow = a.spec + (long long)b * a.Nh + row * LS;

  // ---- the half row X[0..L] into LDS; X[0] and X[L] are real after the other axes' inverses
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int k = p + P * i;
    float2 x = valid ? srow[k] : make_float2(0.f, 0.f);
    if (k == 0) x.y = 0.0f;
    lrow[lidx(k)] = x;
  }
  if (p == 0) lrow[lidx(L)] = valid ? make_float2(srow[L].x, 0.0f) : make_float2(0.f, 0.f);
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

  // ---- normalise (Eq. (15)), write the field, threshold
  const double* fs = a.fstats + (long long)b * 8;
  const float scale = (float)fs[4], offset = (float)fs[5];
  const float tol = a.near_tol;
  unsigned npos = 0, nnear = 0;
  float* frow = a.field ? a.field + (long long)b * a.N + row * (2LL * L) : nullptr;
  int8_t* trow = a.pm1 ? a.pm1 + (long long)b * a.N + row * (2LL * L) : nullptr;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int n = slot_index<L, RL, P>(s, p);
    const float x0 = fmaf(v[s].x, scale, offset);
    const float x1 = fmaf(v[s].y, scale, offset);
    if (valid && frow) *reinterpret_cast<float2*>(frow + 2 * n) = make_float2(x0, x1);
    if constexpr (THRESH) {
      const float t0 = x0 >= 0.0f ? 1.0f : -1.0f, t1 = x1 >= 0.0f ? 1.0f : -1.0f;
      if (valid) {
        npos += (x0 >= 0.0f) + (x1 >= 0.0f);
        nnear += (fabsf(x0) < tol) + (fabsf(x1) < tol);
        if (trow) {
          char2 tt;
          tt.x = (signed char)t0;
          tt.y = (signed char)t1;
          *reinterpret_cast<char2*>(trow + 2 * n) = tt;
        }
      }
      v[s] = make_float2(t0, t1);
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
#pragma unroll
    for (int s = 0; s < E; ++s) lrow[lidx(slot_index<L, RLF, P>(s, p))] = v[s];
    __syncthreads();
    r2c_twist_store<L, P, E>(lrow, a.tw2, srow, p, valid);
    if (tid == 0 && a.counts) {
      unsigned long long np = 0, nn = 0;
      for (int w = 0; w < (T + 63) / 64; ++w) { np += red_u[0][w]; nn += red_u[1][w]; }
      atomicAdd((unsigned long long*)(a.counts + 2 * b + 0), np);
      atomicAdd((unsigned long long*)(a.counts + 2 * b + 1), nn);
    }
  }
}

#define HU_ROW_LENGTHS(X) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(1024)

static inline unsigned ceil_div_u(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

template <int L, int SRC>
static hipError_t launch_rows_r2c_L(const RowsArgs& a, int batch, hipStream_t st) {
  constexpr int C = RowTile<L>::C, T = RowTile<L>::T;
  dim3 grid(ceil_div_u(a.nrows, C), batch);
  hipLaunchKernelGGL((k_rows_r2c<L, SRC>), grid, dim3(T), (size_t)C * Region<L>::value * sizeof(float2), st, a);
  return hipGetLastError();
}

hipError_t launch_rows_r2c(int L, int src, const RowsArgs& a, int batch, hipStream_t st) {
  switch (L) {
#define X(LL)                                                                        \
  case LL:                                                                           \
    if (src == SRC_NOISE) return launch_rows_r2c_L<LL, SRC_NOISE>(a, batch, st);     \
    if (src == SRC_F32) return launch_rows_r2c_L<LL, SRC_F32>(a, batch, st);         \
    return launch_rows_r2c_L<LL, SRC_I8>(a, batch, st);
    HU_ROW_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

template <int L, bool THRESH>
static hipError_t launch_rows_c2r_L(const RowsZArgs& a, int batch, hipStream_t st) {
  constexpr int C = RowTile<L>::C, T = RowTile<L>::T;
  dim3 grid(ceil_div_u(a.nrows, C), batch);
  hipLaunchKernelGGL((k_rows_c2r<L, THRESH>), grid, dim3(T), (size_t)C * Region<L>::value * sizeof(float2), st, a);
  return hipGetLastError();
}

hipError_t launch_rows_c2r(int L, bool thresh, const RowsZArgs& a, int batch, hipStream_t st) {
  switch (L) {
#define X(LL)                                                            \
  case LL:                                                               \
    return thresh ? launch_rows_c2r_L<LL, true>(a, batch, st)            \
                  : launch_rows_c2r_L<LL, false>(a, batch, st);
    HU_ROW_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hu
