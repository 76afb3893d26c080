// The x-row and y-column transforms of one z-plane of a 3D field in one workgroup, for grids whose
// plane (n_y rows of n_x/2 + 1 modes, padded) fits in LDS; the y transforms exchange in place.
// Two kernels take the place of five passes of the 3D sequence:
//   plane_fwd: noise -> R2C rows -> forward y transform -> the plane's half spectrum to HBM
//              (replaces rows_r2c_noise and the first y pass);
//   plane_inv: the plane from HBM -> inverse y transform -> C2R rows, normalisation (Eq. (15)),
//              field, sign map and counts -> R2C of the +-1 rows -> forward y transform -> the
//              +-1 plane to HBM (replaces the inverse y pass, the last row pass and the y pass of
//              the +-1 field).
// The z transforms, the filter and the binning stay in the axis-0 passes, on the same half-spectrum
// layout (row-major (z, y, m_x)).  Plans, stage tables, twist and noise stream are those of the
// general passes; the sign counts go to one slot per plane, which k_spec_final totals.
#include "hu_common.hpp"

namespace hu {

template <int LR, int NY>
struct PlaneShape {
  static constexpr int PR = Plan<LR>::P, ER = Plan<LR>::E;      // x rows (L = n_x / 2)
  static constexpr int PC = Plan<NY>::P, EC = Plan<NY>::E;      // y columns
  static constexpr int NC = LR + 1;                             // half-spectrum columns
  static constexpr int RSR = Region<LR>::value;                 // a row's slot: exchange region, then modes
  // LR column tasks: column t, and task 0 also column LR (the two real y sequences packed into one
  // complex transform)
  static constexpr int TA = NY * PR, TB = LR * PC;
  static constexpr int T = ((TA > TB ? TA : TB) + 63) / 64 * 64;
  static_assert(RSR >= LR + 1 && T <= 1024, "plane shape");
  static constexpr size_t lds_bytes = (size_t)NY * RSR * 8;      // the plane only: columns exchange in place
};

#define HU_PLANE_SHAPES(X)                                                                          \
  X(16, 32) X(16, 48) X(16, 64) X(16, 96) X(16, 128) X(24, 32) X(24, 48) X(24, 64) X(24, 96) X(24, 128) \
  X(32, 32) X(32, 48) X(32, 64) X(32, 96) X(32, 128) X(48, 32) X(48, 48) X(48, 64) X(48, 96) X(48, 128) \
  X(64, 32) X(64, 48) X(64, 64) X(64, 96) X(64, 128)

size_t plane_lds_bytes(int LR, int NY) {
  switch (LR * 1000 + NY) {
#define X(A, B) case A * 1000 + B: return PlaneShape<A, B>::lds_bytes;
    HU_PLANE_SHAPES(X)
#undef X
    default: return 0;
  }
}

// twist of a row whose natural-order Z sits in `lz` (padded): X[0..LR] over the slot, unpadded
template <int LR, int PR, int ER>
__device__ __forceinline__ void plane_twist(float2* lz, const float2* __restrict__ tw2, int p) {
  float2 X[ER + 1];
#pragma unroll
  for (int i = 0; i < ER; ++i) {
    const int k = p + PR * i;
    const float2 zk = lz[lidx(k)];
    const float2 zm = cconj(lz[lidx(k == 0 ? 0 : LR - k)]);
    const float2 A = cadd(zk, zm), B = csub(zk, zm);
    X[i] = cscale(cadd(A, mul_mi<false>(cmul(tw2[k], B))), 0.5f);
  }
  const float2 z0 = lz[0];
  X[ER] = make_float2(z0.x - z0.y, 0.0f);
  xchg_sync<true>();
#pragma unroll
  for (int i = 0; i < ER; ++i) lz[p + PR * i] = X[i];
  if (p == 0) lz[LR] = X[ER];
  xchg_sync<true>();
}

// The y transforms (forward, or inverse with the forward radix list as the y passes do) of the
// plane held in LDS, natural order in and out, each exchanged in place inside its own column.
// Columns 0 and LR (k_x = 0 and the x Nyquist index) carry y sequences that are real before the
// forward transform (the row twist makes X[0] and X[LR] real) and real after the inverse one (the
// C2R rows use their real parts only): they share one complex transform, z = col_0 + i col_LR,
// separated afterwards by Hermitian symmetry.  So the plane needs LR column tasks, not LR + 1.
template <int LR, int NY, bool INV>
__device__ __forceinline__ void plane_cols(float2* plane, const float2* __restrict__ tw, int tid) {
  using S = PlaneShape<LR, NY>;
  constexpr int PC = S::PC, EC = S::EC, RSR = S::RSR;
  using Rad = typename Plan<NY>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  const int t = tid / PC, pc = tid % PC;
  if (t >= LR) return;
  float2* col = plane + t;
  float2* colL = plane + LR;
  float2 v[EC];
#pragma unroll
  for (int s = 0; s < EC; ++s) {
    const int e = slot_index<NY, R1, PC>(s, pc);
    if (t == 0) {
      const float2 y0 = col[e * RSR], yl = colL[e * RSR];
      // forward: the real sequences a + i c; inverse: Y0 + i YL
      v[s] = INV ? make_float2(y0.x - yl.y, y0.y + yl.x) : make_float2(y0.x, yl.x);
    } else {
      v[s] = col[e * RSR];
    }
  }
  fft_run<NY, PC, EC, INV, true>(Rad{}, v, reinterpret_cast<Strided<RSR>*>(col), pc, tw);
  xchg_sync<true>();
  if (t != 0) {
#pragma unroll
    for (int s = 0; s < EC; ++s) col[slot_index<NY, RL, PC>(s, pc) * RSR] = v[s];
    return;
  }
  if constexpr (INV) {
    // y0 + i yL: both real
#pragma unroll
    for (int s = 0; s < EC; ++s) {
      const int e = slot_index<NY, RL, PC>(s, pc);
      col[e * RSR] = make_float2(v[s].x, 0.0f);
      colL[e * RSR] = make_float2(v[s].y, 0.0f);
    }
  } else {
    // Z = A + i C with A, C Hermitian: A[k] = (Z[k] + conj Z[-k]) / 2, C[k] = -i (Z[k] - conj Z[-k]) / 2,
    // and A[-k] = conj A[k], C[-k] = conj C[k]: each thread takes the pairs (k, NY - k), k <= NY / 2,
    // reading and writing only their own positions (no barrier, no register arrays)
#pragma unroll
    for (int s = 0; s < EC; ++s) col[slot_index<NY, RL, PC>(s, pc) * RSR] = v[s];
    xchg_sync<true>();
    for (int k = pc; k <= NY / 2; k += PC) {
      const int m = k == 0 ? 0 : NY - k;
      const float2 zk = col[k * RSR];
      const float2 zm = cconj(col[m * RSR]);
      const float2 ak = cscale(cadd(zk, zm), 0.5f);
      const float2 ck = cscale(mul_mi<false>(csub(zk, zm)), 0.5f);
      col[k * RSR] = ak;
      colL[k * RSR] = ck;
      col[m * RSR] = cconj(ak);
      colL[m * RSR] = cconj(ck);
    }
  }
}

template <int LR, int NY>
__device__ __forceinline__ void plane_copy(float2* __restrict__ dst_hbm, const float2* __restrict__ src_hbm,
                                           float2* plane, int tid, bool to_lds) {
  using S = PlaneShape<LR, NY>;
  constexpr int NC = S::NC;
  for (int i = tid; i < NY * NC; i += S::T) {
    const int y = i / NC, g = i - y * NC;
    if (to_lds) plane[y * S::RSR + g] = src_hbm[i];
    else dst_hbm[i] = plane[y * S::RSR + g];
  }
}

// grid (n0 planes, B fields)
template <int LR, int NY>
__global__ void __launch_bounds__((PlaneShape<LR, NY>::T)) k_plane_fwd(RowsArgs a) {
  using S = PlaneShape<LR, NY>;
  constexpr int PR = S::PR, ER = S::ER, T = S::T, RSR = S::RSR, NX = 2 * LR;
  using RadR = typename Plan<LR>::fwd;
  constexpr int R1R = RadInfo<RadR>::first, RLR = RadInfo<RadR>::last;
  extern __shared__ float2 lds[];
  float2* plane = lds;
  const int tid = threadIdx.x, z = blockIdx.x, b = blockIdx.y;
  if (z == 0) {                                  // the first row pass's set-up duties for this field
    if (b == 0)
      for (int i = tid; i < a.nzero; i += T) a.zero[i] = 0u;
    if (a.io) {
      const FieldIO& io = a.io[b];
      uint32_t* dst[2] = {reinterpret_cast<uint32_t*>(io.cont_cnt), reinterpret_cast<uint32_t*>(io.pm1_cnt)};
      for (int s = 0; s < 2; ++s)
        if (dst[s] && a.cnt_src)
          for (int i = tid; i < 2 * a.nb; i += T) dst[s][i] = a.cnt_src[i];
    } else {
      for (int s = 0; s < a.fill_spans; ++s) {
        uint32_t* dst = a.fill[s].dst + (long long)b * a.fill[s].per_field;
        const uint32_t* src = a.fill[s].src;
        for (int i = tid; i < a.fill[s].per_field; i += T) dst[i] = src ? src[i] : 0u;
      }
    }
  }
  // rows: noise of row z n_y + r (voxel i takes normal i mod 4 of Philox block i / 4), R2C
  const int r = tid / PR, pr = tid % PR;
  if (r < NY) {
    uint64_t seed = 0;                            // scalar select: no run-time index into the arguments
    if (a.io) {
      seed = a.io[b].seed;
    } else {
#pragma unroll
      for (int i = 0; i < MAX_CHUNK; ++i) seed = i == b ? a.seeds[i] : seed;
    }
    seed = uniform_u64(seed);
    float2* lrow = plane + r * RSR;
    const uint64_t m0 = ((uint64_t)z * NY + (uint64_t)r) * (NX / 4);
    static_assert((NX % 4) == 0, "a row holds whole Philox blocks");
    for (int j = pr; j < NX / 4; j += PR) {
      float zz[4];
      noise4(m0 + (uint64_t)j, seed, zz);
      lrow[lidx(2 * j)] = make_float2(zz[0], zz[1]);
      lrow[lidx(2 * j + 1)] = make_float2(zz[2], zz[3]);
    }
    xchg_sync<true>();
    float2 v[ER];
    stage_load<LR, R1R, PR, ER>(v, lrow, pr);
    fft_run<LR, PR, ER, false, true>(RadR{}, v, lrow, pr, a.tw);
    xchg_sync<true>();
    slot_store<LR, RLR, PR, ER>(v, lrow, pr);
    xchg_sync<true>();
    plane_twist<LR, PR, ER>(lrow, a.tw2, pr);
  }
  __syncthreads();
  plane_cols<LR, NY, false>(plane, a.tw_y, tid);
  __syncthreads();
  plane_copy<LR, NY>(a.spec + (long long)b * a.Nh + (long long)z * NY * S::NC, nullptr, plane, tid, false);
}

template <int LR, int NY, bool THRESH>
__global__ void __launch_bounds__((PlaneShape<LR, NY>::T)) k_plane_inv(RowsZArgs a) {
  using S = PlaneShape<LR, NY>;
  constexpr int PR = S::PR, ER = S::ER, T = S::T, RSR = S::RSR, NX = 2 * LR;
  using RadR = typename Plan<LR>::fwd;
  using RadRF = Reverse<RadR>;
  constexpr int R1R = RadInfo<RadR>::first, RLR = RadInfo<RadR>::last, RLRF = RadInfo<RadRF>::last;
  extern __shared__ float2 lds[];
  __shared__ unsigned red_u[2][T / 64];
  float2* plane = lds;
  const int tid = threadIdx.x, z = blockIdx.x, b = blockIdx.y;
  float2* sp = a.spec + (long long)b * a.Nh + (long long)z * NY * S::NC;
  plane_copy<LR, NY>(nullptr, sp, plane, tid, true);
  __syncthreads();
  plane_cols<LR, NY, true>(plane, a.tw_y, tid);
  __syncthreads();
  // rows: C2R, normalisation, field, sign map, counts, R2C of the +-1 row
  const double* fs = a.fstats + (long long)b * 8;
  const float scale = (float)fs[4], offset = (float)fs[5];
  float* fout;
  int8_t* tout;
  float near_tol;
  if (a.io) {
    fout = a.io[b].field;
    tout = a.io[b].pm1;
    near_tol = a.io[b].near_abs;
  } else {
    fout = field_ptr(a.field, a.N, b);
    tout = field_ptr(a.pm1, a.N, b);
    near_tol = a.near_tol;
  }
  const int r = tid / PR, pr = tid % PR;
  unsigned npos = 0, nnear = 0;
  if (r < NY) {
    float2* lrow = plane + r * RSR;
    float2 zv[ER];
#pragma unroll
    for (int s = 0; s < ER; ++s) {
      const int k = slot_index<LR, R1R, PR>(s, pr);
      float2 xk = lrow[k], xm = lrow[LR - k];
      if (k == 0) { xk.y = 0.0f; xm.y = 0.0f; }
      const float2 xc = cconj(xm);
      const float2 w = cconj(a.tw2[k]);
      zv[s] = cadd(cadd(xk, xc), mul_mi<true>(cmul(w, csub(xk, xc))));
    }
    fft_run<LR, PR, ER, true, true>(RadR{}, zv, lrow, pr, a.tw);
    const long long row = (long long)z * NY + r;
    float* frow = fout ? fout + row * NX : nullptr;
    int8_t* trow = (THRESH && tout) ? tout + row * NX : nullptr;
#pragma unroll
    for (int s = 0; s < ER; ++s) {
      const int k = slot_index<LR, RLR, PR>(s, pr);
      const float x0 = fmaf(zv[s].x, scale, offset), x1 = fmaf(zv[s].y, scale, offset);
      if (frow) *reinterpret_cast<float2*>(frow + 2 * k) = make_float2(x0, x1);
      if constexpr (THRESH) {
        const bool p0 = x0 >= 0.0f, p1 = x1 >= 0.0f;
        npos += (unsigned)p0 + (unsigned)p1;
        nnear += (unsigned)(fabsf(x0) < near_tol) + (unsigned)(fabsf(x1) < near_tol);
        if (trow) {
          trow[2 * k] = p0 ? (int8_t)1 : (int8_t)-1;
          trow[2 * k + 1] = p1 ? (int8_t)1 : (int8_t)-1;
        }
        zv[s] = make_float2(p0 ? 1.0f : -1.0f, p1 ? 1.0f : -1.0f);
      }
    }
    if (THRESH && a.pm1_spec) {
      fft_run<LR, PR, ER, false, true>(RadRF{}, zv, lrow, pr, a.tw);
      xchg_sync<true>();
      slot_store<LR, RLRF, PR, ER>(zv, lrow, pr);
      xchg_sync<true>();
      plane_twist<LR, PR, ER>(lrow, a.tw2, pr);
    }
  }
  if constexpr (THRESH) {
    npos = wave_usum(npos);
    nnear = wave_usum(nnear);
    if ((tid & 63) == 0) { red_u[0][tid >> 6] = npos; red_u[1][tid >> 6] = nnear; }
  }
  __syncthreads();
  if (THRESH && tid == 0 && a.cpart) {
    unsigned np = 0, nn = 0;
    for (int w = 0; w < T / 64; ++w) { np += red_u[0][w]; nn += red_u[1][w]; }
    reinterpret_cast<uint2*>(a.cpart)[(long long)b * gridDim.x + z] = make_uint2(np, nn);
  }
  if (!(THRESH && a.pm1_spec)) return;            // uniform over the workgroup
  plane_cols<LR, NY, false>(plane, a.tw_y, tid);
  __syncthreads();
  plane_copy<LR, NY>(sp, nullptr, plane, tid, false);
}

template <int LR, int NY>
static hipError_t launch_plane_fwd_L(const RowsArgs& a, int n0, int batch, hipStream_t st) {
  using S = PlaneShape<LR, NY>;
  hipLaunchKernelGGL((k_plane_fwd<LR, NY>), dim3(n0, batch), dim3(S::T), S::lds_bytes, st, a);
  return hipGetLastError();
}

template <int LR, int NY>
static hipError_t launch_plane_inv_L(const RowsZArgs& a, bool thresh, int n0, int batch, hipStream_t st) {
  using S = PlaneShape<LR, NY>;
  if (thresh) hipLaunchKernelGGL((k_plane_inv<LR, NY, true>), dim3(n0, batch), dim3(S::T), S::lds_bytes, st, a);
  else hipLaunchKernelGGL((k_plane_inv<LR, NY, false>), dim3(n0, batch), dim3(S::T), S::lds_bytes, st, a);
  return hipGetLastError();
}

hipError_t launch_plane_fwd(int LR, int NY, const RowsArgs& a, int n0, int batch, hipStream_t st) {
  switch (LR * 1000 + NY) {
#define X(A, B) case A * 1000 + B: return launch_plane_fwd_L<A, B>(a, n0, batch, st);
    HU_PLANE_SHAPES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_plane_inv(int LR, int NY, const RowsZArgs& a, bool thresh, int n0, int batch, hipStream_t st) {
  switch (LR * 1000 + NY) {
#define X(A, B) case A * 1000 + B: return launch_plane_inv_L<A, B>(a, thresh, n0, batch, st);
    HU_PLANE_SHAPES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hu
