// The whole hot path of one small 2D field in one workgroup, with the half spectrum resident in
// LDS: seeded noise -> R2C rows -> axis-0 transforms with the filter H_sym (Eqs. (8), (12)-(13)),
// the Parseval statistics of Eq. (15) and the continuous-spectrum bins -> inverse axis-0
// transforms -> C2R rows, normalisation, field, sign map and counts -> R2C of the +-1 rows ->
// axis-0 transforms and the +-1 spectrum bins.  HBM sees only the outputs (the field, the map,
// the statistics and the spectra) and the read-only tables: for grids up to 128^2 this replaces
// the six passes of the general sequence.  The arithmetic is that of the general passes (the same
// Philox stream, plans, twiddle tables, twist and filter code); the bins use the same exact
// integer combination, here per mode over the whole field.
#include "hu_common.hpp"

namespace hu {

template <int LR, int N0>
struct SmallShape {
  static constexpr int PR = Plan<LR>::P, ER = Plan<LR>::E;      // row transforms (L = n_x / 2)
  static constexpr int PC = Plan<N0>::P, EC = Plan<N0>::E;      // axis-0 transforms
  static constexpr int NC = LR + 1;                             // half-spectrum columns
  static constexpr int RSR = Region<LR>::value;                 // a row's LDS slot: its exchange
  static constexpr int RSC = Region<N0>::value;                 // region, then its LR + 1 modes
  static constexpr int TA = N0 * PR, TB = NC * PC;
  static constexpr int T = ((TA > TB ? TA : TB) + 63) / 64 * 64;
  static_assert(RSR >= LR + 1, "a row slot holds the row's half spectrum");
  static_assert(T <= 1024, "one workgroup per field");
  // LDS bytes before the histogram
  static constexpr size_t base_bytes = (size_t)(N0 * RSR + NC * RSC) * 8;
};

size_t small_lds_bytes(int LR, int N0, int nb) {
  switch (LR * 1000 + N0) {
#define X(A, B) case A * 1000 + B: return SmallShape<A, B>::base_bytes + (size_t)nb * 12;
    X(8, 16) X(8, 32) X(8, 64) X(8, 128) X(16, 16) X(16, 32) X(16, 64) X(16, 128)
    X(32, 16) X(32, 32) X(32, 64) X(32, 128) X(64, 16) X(64, 32) X(64, 64) X(64, 128)
#undef X
    default: return 0;
  }
}

// the twist of a row whose natural-order Z sits in `lz`: X[k] for this thread's k = p + PR i
// (and X[LR] on thread 0), into registers first, then over the row's slot (unpadded)
template <int LR, int PR, int ER>
__device__ __forceinline__ void twist_row(float2* lz, const float2* __restrict__ tw2, int p) {
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

// pass 1 (largest exponent per bin) or 2 (fixed-point adds) of the exact bin combination of the
// values w |v|^2 of a column's modes (bins from the table, recomputed in each pass)
template <int N0, int PC, int EC, int RL, bool PASS2>
__device__ __forceinline__ void commit_modes(const float2 (&v)[EC], float wm, const uint16_t* __restrict__ tcol,
                                             int pc, int* hx, unsigned long long* hq) {
#pragma unroll
  for (int s = 0; s < EC; ++s) {
    const int e = slot_index<N0, RL, PC>(s, pc);
    run_commit<PASS2>((int)tcol[e], (double)(wm * (v[s].x * v[s].x + v[s].y * v[s].y)), hx, hq);
  }
}

template <int LR, int N0, bool GEN>
__global__ void __launch_bounds__((SmallShape<LR, N0>::T)) k_field_lds(SmallArgs a) {
  using S = SmallShape<LR, N0>;
  constexpr int PR = S::PR, ER = S::ER, PC = S::PC, EC = S::EC, NC = S::NC, T = S::T;
  constexpr int RSR = S::RSR, RSC = S::RSC;
  using RadR = typename Plan<LR>::fwd;
  using RadRF = Reverse<RadR>;
  constexpr int R1R = RadInfo<RadR>::first, RLR = RadInfo<RadR>::last, RLRF = RadInfo<RadRF>::last;
  using RadC = typename Plan<N0>::fwd;
  using RadCI = Reverse<RadC>;
  constexpr int R1C = RadInfo<RadC>::first, RLC = RadInfo<RadC>::last;
  extern __shared__ float2 lds[];
  __shared__ double red_d[T / 64], red_d0[T / 64];
  __shared__ float red_f[T / 64];
  __shared__ unsigned red_u[2][T / 64];
  __shared__ double fin[4];                       // scale, offset, continuous factor, flag
  float2* spec = lds;                             // [N0][RSR]
  float2* xr = lds + N0 * RSR;                    // [NC][RSC]
  unsigned long long* hq = reinterpret_cast<unsigned long long*>(xr + NC * RSC);
  int* hx = reinterpret_cast<int*>(hq + a.nb);
  const int tid = threadIdx.x, b = blockIdx.x;
  const FieldIO* io = a.io ? a.io + b : nullptr;
  const long long N = a.N;
  constexpr int NX = 2 * LR;

  for (int j = tid; j < a.nb; j += T) {
    hx[j] = HX_EMPTY;
    hq[j] = 0ull;
  }
  // ---- rows: noise (voxel i takes normal i mod 4 of Philox block i / 4) -> R2C
  const int r = tid / PR, pr = tid % PR;
  const bool row_ok = r < N0;
  float2* lrow = spec + r * RSR;
  if (row_ok) {
    // the uniform-mode seed picked by an unrolled scalar select: a run-time index into the
    // argument array would copy the whole argument block to scratch memory
    uint64_t seed = 0;
    if (io) {
      seed = io->seed;
    } else {
#pragma unroll
      for (int i = 0; i < MAX_WHOLE_CHUNK; ++i) seed = i == b ? a.seeds[i] : seed;
    }
    seed = uniform_u64(seed);
    const uint64_t m0 = (uint64_t)r * (NX / 4);
    for (int j = pr; j < NX / 4; j += PR) {
      float z[4];
      noise4(m0 + (uint64_t)j, seed, z);
      lrow[lidx(2 * j)] = make_float2(z[0], z[1]);
      lrow[lidx(2 * j + 1)] = make_float2(z[2], z[3]);
    }
    xchg_sync<true>();
    float2 v[ER];
    stage_load<LR, R1R, PR, ER>(v, lrow, pr);
    fft_run<LR, PR, ER, false, true>(RadR{}, v, lrow, pr, a.tw_row);
    xchg_sync<true>();
    slot_store<LR, RLR, PR, ER>(v, lrow, pr);
    xchg_sync<true>();
    twist_row<LR, PR, ER>(lrow, a.tw2, pr);
  }
  __syncthreads();

  // ---- axis 0: forward transform, filter, statistics, continuous bins, inverse transform
  const int g = tid / PC, pc = tid % PC;
  const bool col_ok = g < NC;
  FiltDev filt;
  if (io) filt = io->filt;
  else filt = a.filt;
  const ColCoord cc = col_coord(a.gm, col_ok ? g : 0);
  const uint16_t* tcol = a.table ? a.table + (long long)(col_ok ? g : 0) * N0 : nullptr;
  float2 v[EC];
  double gsum = 0.0, f0 = 0.0;
  float lmax = filt.lnoffset;
  if (col_ok) {
#pragma unroll
    for (int s = 0; s < EC; ++s) v[s] = spec[slot_index<N0, R1C, PC>(s, pc) * RSR + g];
    float2* lx = xr + g * RSC;
    fft_run<N0, PC, EC, false, true>(RadC{}, v, lx, pc, a.tw_col);
#pragma unroll
    for (int s = 0; s < EC; ++s) {
      const int e = slot_index<N0, RLC, PC>(s, pc);
      float lnc;
      const float H = amp_sym<2, GEN>(filt, a.gm, cc, e, lnc);
      const float2 F = cscale(v[s], H);
      v[s] = F;
      gsum += (double)(cc.wm * (F.x * F.x + F.y * F.y));
      lmax = fmaxf(lmax, lnc);
      if (g == 0 && e == 0) f0 = (double)F.x;
    }
    if (a.want_cont) commit_modes<N0, PC, EC, RLC, false>(v, cc.wm, tcol, pc, hx, hq);
  }
  __syncthreads();
  if (col_ok) {
    if (a.want_cont) commit_modes<N0, PC, EC, RLC, true>(v, cc.wm, tcol, pc, hx, hq);
    fft_run<N0, PC, EC, true, true>(RadCI{}, v, xr + g * RSC, pc, a.tw_col);
#pragma unroll
    for (int s = 0; s < EC; ++s) spec[slot_index<N0, R1C, PC>(s, pc) * RSR + g] = v[s];
  }
  // statistics of Eq. (15) by Parseval, in a fixed order
  gsum = wave_sum(gsum);
  f0 = wave_sum(f0);
  lmax = wave_max(lmax);
  if ((tid & 63) == 0) { red_d[tid >> 6] = gsum; red_d0[tid >> 6] = f0; red_f[tid >> 6] = lmax; }
  __syncthreads();
  if (tid == 0) {
    double G = 0.0, F0 = 0.0;
    float lm = -1.0e30f;
    for (int w = 0; w < T / 64; ++w) { G += red_d[w]; F0 += red_d0[w]; lm = fmaxf(lm, red_f[w]); }
    double sigma_f;
    if (io) sigma_f = io->sigma_f;
    else sigma_f = a.sigma_f;
    const double mu = F0 / (double)N;
    const double var = G / ((double)N * (double)N) - mu * mu;
    const double lmx = (double)lm;
    const bool degenerate = !(lmx >= -80.0) || !(var > 0.0);
    const double sd = degenerate ? 1.0 : sqrt(var);
    fin[0] = degenerate ? 0.0 : sigma_f / ((double)N * sd);
    fin[1] = degenerate ? 0.0 : -sigma_f * mu / sd;
    fin[2] = degenerate ? 0.0 : sigma_f * sigma_f / ((double)N * var);
    double* st = io ? io->stats : field_ptr(a.stats, 4, b);
    if (st) { st[0] = mu; st[1] = var; st[2] = lmx; st[3] = degenerate ? 1.0 : 0.0; }
  }
  __syncthreads();
  // the continuous spectrum of the normalised field, and the mode counts of both spectra
  {
    double* cout_ = io ? io->cont_sum : field_ptr(a.cont_sum, a.nb, b);
    uint64_t* ccnt = io ? io->cont_cnt : field_ptr(a.cont_cnt, a.nb, b);
    uint64_t* pcnt = a.thresh ? (io ? io->pm1_cnt : field_ptr(a.pm1_cnt, a.nb, b)) : nullptr;
    for (int j = tid; j < a.nb; j += T) {
      if (a.want_cont) {
        const int ex = hx[j];
        if (cout_) cout_[j] = (ex == HX_EMPTY ? 0.0 : ldexp((double)hq[j], ex - HQ_SHIFT)) * fin[2];
        hx[j] = HX_EMPTY;
        hq[j] = 0ull;
      }
      const uint64_t n = a.counts_tab ? a.counts_tab[j] : 0;
      if (ccnt) ccnt[j] = n;
      if (pcnt) pcnt[j] = n;
    }
  }

  // ---- rows: C2R, normalisation, field, sign map and counts, R2C of the +-1 row
  unsigned npos = 0, nnear = 0;
  if (row_ok) {
    float* fout = io ? io->field : field_ptr(a.field, N, b);
    int8_t* tout = a.thresh ? (io ? io->pm1 : field_ptr(a.pm1, N, b)) : nullptr;
    float near_tol;
    if (io) near_tol = io->near_abs;
    else near_tol = a.near_abs;
    const float scale = (float)fin[0], offset = (float)fin[1];
    // pre-twist: Z[k] = (X[k] + X*[LR - k]) + i e^{+i pi k / LR} (X[k] - X*[LR - k]); X[0] and X[LR]
    // are real
    float2 z[ER];
#pragma unroll
    for (int s = 0; s < ER; ++s) {
      const int k = slot_index<LR, R1R, PR>(s, pr);
      float2 xk = lrow[k], xm = lrow[LR - k];
      if (k == 0) { xk.y = 0.0f; xm.y = 0.0f; }
      const float2 xc = cconj(xm);
      const float2 w = cconj(a.tw2[k]);
      z[s] = cadd(cadd(xk, xc), mul_mi<true>(cmul(w, csub(xk, xc))));
    }
    fft_run<LR, PR, ER, true, true>(RadR{}, z, lrow, pr, a.tw_row);
    float* frow = fout ? fout + (long long)r * NX : nullptr;
    int8_t* trow = tout ? tout + (long long)r * NX : nullptr;
#pragma unroll
    for (int s = 0; s < ER; ++s) {
      const int k = slot_index<LR, RLR, PR>(s, pr);
      const float x0 = fmaf(z[s].x, scale, offset), x1 = fmaf(z[s].y, scale, offset);
      if (frow) *reinterpret_cast<float2*>(frow + 2 * k) = make_float2(x0, x1);
      if (a.thresh) {
        const bool p0 = x0 >= 0.0f, p1 = x1 >= 0.0f;
        npos += (unsigned)p0 + (unsigned)p1;
        nnear += (unsigned)(fabsf(x0) < near_tol) + (unsigned)(fabsf(x1) < near_tol);
        if (trow) {
          trow[2 * k] = p0 ? (int8_t)1 : (int8_t)-1;
          trow[2 * k + 1] = p1 ? (int8_t)1 : (int8_t)-1;
        }
        z[s] = make_float2(p0 ? 1.0f : -1.0f, p1 ? 1.0f : -1.0f);
      }
    }
    if (a.want_pm1) {
      fft_run<LR, PR, ER, false, true>(RadRF{}, z, lrow, pr, a.tw_row);
      xchg_sync<true>();
      slot_store<LR, RLRF, PR, ER>(z, lrow, pr);
      xchg_sync<true>();
      twist_row<LR, PR, ER>(lrow, a.tw2, pr);
    }
  }
  if (a.thresh) {
    npos = wave_usum(npos);
    nnear = wave_usum(nnear);
    if ((tid & 63) == 0) { red_u[0][tid >> 6] = npos; red_u[1][tid >> 6] = nnear; }
  }
  __syncthreads();
  if (a.thresh && tid == 0) {
    uint64_t* cnt = io ? io->counts : field_ptr(a.counts, 2, b);
    if (cnt) {
      unsigned long long np = 0, nn = 0;
      for (int w = 0; w < T / 64; ++w) { np += red_u[0][w]; nn += red_u[1][w]; }
      cnt[0] = np;
      cnt[1] = nn;
    }
  }
  if (!a.want_pm1) return;                        // uniform over the workgroup

  // ---- axis 0 of the +-1 field: forward transform and bins of w |X|^2 / N
  if (col_ok) {
#pragma unroll
    for (int s = 0; s < EC; ++s) v[s] = spec[slot_index<N0, R1C, PC>(s, pc) * RSR + g];
    fft_run<N0, PC, EC, false, true>(RadC{}, v, xr + g * RSC, pc, a.tw_col);
    commit_modes<N0, PC, EC, RLC, false>(v, cc.wm, tcol, pc, hx, hq);
  }
  __syncthreads();
  if (col_ok) commit_modes<N0, PC, EC, RLC, true>(v, cc.wm, tcol, pc, hx, hq);
  __syncthreads();
  double* pout = io ? io->pm1_sum : field_ptr(a.pm1_sum, a.nb, b);
  const double pscale = 1.0 / (double)N;
  if (pout)
    for (int j = tid; j < a.nb; j += T) {
      const int ex = hx[j];
      pout[j] = (ex == HX_EMPTY ? 0.0 : ldexp((double)hq[j], ex - HQ_SHIFT)) * pscale;
    }
}

template <int LR, int N0>
static hipError_t launch_small_L(const SmallArgs& a, int batch, hipStream_t st) {
  using S = SmallShape<LR, N0>;
  const size_t lds = S::base_bytes + (size_t)a.nb * 12;
  if (a.any_gen) hipLaunchKernelGGL((k_field_lds<LR, N0, true>), dim3(batch), dim3(S::T), lds, st, a);
  else hipLaunchKernelGGL((k_field_lds<LR, N0, false>), dim3(batch), dim3(S::T), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_field_lds(int LR, int N0, const SmallArgs& a, int batch, hipStream_t st) {
  switch (LR * 1000 + N0) {
#define X(A, B) case A * 1000 + B: return launch_small_L<A, B>(a, batch, st);
    X(8, 16) X(8, 32) X(8, 64) X(8, 128) X(16, 16) X(16, 32) X(16, 64) X(16, 128)
    X(32, 16) X(32, 32) X(32, 64) X(32, 128) X(64, 16) X(64, 32) X(64, 64) X(64, 128)
#undef X
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hu
