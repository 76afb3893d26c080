// Differentiation of the binned continuous spectrum with respect to the filter parameters, and the
// expected spectrum of a filter.
//
// The normalised continuous spectrum of one field, binned, is
//   P_b = sigma_f^2 N G_b / (c_b G_tot),  G_b = sum_{k in b} w_k H_sym(k)^2 |W(k)|^2,
// with W the noise spectrum, G_tot the same sum over every mode and c_b the mode count (the mean of
// the field is zero because H(0) = 0, so its variance is G_tot / N^2 by Parseval).  For any loss
// with gradient g_b = dL/dP_b the chain rule gives
//   dL/dtheta_j = sum_k w_k omega(k) 2 H_sym dH_sym/dtheta_j |W|^2,
//   omega(k)    = beta_{b(k)} - gamma,  beta_b = g_b sigma_f^2 N / (c_b G_tot),
//   gamma       = sum_b g_b P_b / G_tot,
// theta = (a, b, c, p, rot, k0, w) of Eqs. (12)-(13) (band centre k0, width w).  The constant C of
// Eq. (13) and the transform scale cancel.  W is a pure function of the seed, so the gradient pass
// regenerates it (noise, row R2C and the y pass) instead of storing it, and one axis-0 pass
// forms the seven FP64 sums.
//
// The expected spectrum of a filter: E[P] per mode is sigma_f^2 N H^2 / sum_k w_k H^2 (Eqs. (10)-(11)
// with the normalisation of Eq. (15)), binned like the field's spectrum.
#include "hu_common.hpp"

namespace hu {

// ln H (relative) and d lnH/dtheta at one canonical wavenumber; returns H.  With
// u_i = |kappa'_i| / a_i, K = (sum_i u_i^p)^(1/p), r_i = u_i / K:
//   d lnH/dK  = (alpha / K - (K - k0) / w^2) / 2
//   dK/da_i   = -K r_i^p / a_i
//   dK/dp     = (K / p) sum_i r_i^p ln r_i
//   dK/drot   = r_x^(p-1) sgn(kappa'_x) kappa'_y / a - r_y^(p-1) sgn(kappa'_y) kappa'_x / b
//               (d kappa'_x / drot = kappa'_y, d kappa'_y / drot = -kappa'_x)
//   d lnH/dk0 = (K - k0) / (2 w^2),   d lnH/dw = (K - k0)^2 / (2 w^3)
// Terms with u_i = 0 contribute nothing.  The ratios t_i = (u_i / u_max)^p keep every power in
// range: r_i^p = t_i / S with S = sum_i t_i.
template <int NDIM>
__device__ __forceinline__ float lnh_partials(const FiltDev& f, float w, float kx, float ky, float kz, float (&d)[7]) {
  constexpr float LN2 = 0.69314718055994531f;
  const float kxr = f.cr * kx + f.sr * ky;
  const float kyr = -f.sr * kx + f.cr * ky;
  float u[3];
  u[0] = fabsf(kxr) * f.ia;
  u[1] = fabsf(kyr) * f.ib;
  u[2] = NDIM == 3 ? fabsf(kz) * f.ic : 0.0f;
  float um = fmaxf(u[0], u[1]);
  if constexpr (NDIM == 3) um = fmaxf(um, u[2]);
  if (!(um > 0.0f)) {
#pragma unroll
    for (int j = 0; j < 7; ++j) d[j] = 0.0f;
    return 0.0f;
  }
  const float inv = __builtin_amdgcn_rcpf(um);
  float l2r[3], t[3];
  float S = 0.0f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const bool on = (i < NDIM) && u[i] > 0.0f;
    l2r[i] = on ? hw_log2(u[i] * inv) : 0.0f;
    t[i] = on ? hw_exp2(f.p * l2r[i]) : 0.0f;
    S += t[i];
  }
  const float log2S = hw_log2(S);
  const float log2K = hw_log2(um) + log2S * f.ip;
  const float K = hw_exp2(log2K);
  const float dd = K - f.k0;
  const float lnc = f.alpha * (log2K * LN2) - dd * dd * f.inv2w2 - f.lnchimax;
  const float H = amp_from_lnchi(lnc);
  const float dK = 0.5f * (f.alpha * __builtin_amdgcn_rcpf(K) - 2.0f * dd * f.inv2w2);
  const float invS = __builtin_amdgcn_rcpf(S);
  float rp[3], accp = 0.0f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    rp[i] = t[i] * invS;
    accp += rp[i] > 0.0f ? rp[i] * (LN2 * (l2r[i] - log2S * f.ip)) : 0.0f;
  }
  d[0] = dK * (-K * rp[0] * f.ia);
  d[1] = dK * (-K * rp[1] * f.ib);
  d[2] = NDIM == 3 ? dK * (-K * rp[2] * f.ic) : 0.0f;
  d[3] = dK * K * f.ip * accp;
  // r_i^(p-1) = r_i^p K / u_i
  const float rx = u[0] > 0.0f ? rp[0] * K * __builtin_amdgcn_rcpf(u[0]) : 0.0f;
  const float ry = u[1] > 0.0f ? rp[1] * K * __builtin_amdgcn_rcpf(u[1]) : 0.0f;
  const float sx = kxr > 0.0f ? 1.0f : (kxr < 0.0f ? -1.0f : 0.0f);
  const float sy = kyr > 0.0f ? 1.0f : (kyr < 0.0f ? -1.0f : 0.0f);
  d[4] = dK * (rx * sx * kyr * f.ia - ry * sy * kxr * f.ib);
  d[5] = dd * f.inv2w2;
  d[6] = dd * dd * f.inv2w2 * __builtin_amdgcn_rcpf(w);
  return H;
}

// H_sym and dH_sym/dtheta at axis-0 index e of column cc: on the Nyquist planes of a rotated
// filter H_sym averages H at kappa and at kappa with its Nyquist components negated, and is
// differentiated term by term.
template <int NDIM>
__device__ __forceinline__ float hsym_partials(const FiltDev& f, float w, const Axis0Geom& gm, const ColCoord& cc,
                                               int e, float (&dH)[7]) {
  const int mt = e < gm.n0 / 2 ? e : e - gm.n0;
  const float k0c = (float)mt * gm.kap0;
  const bool nyq0 = (2 * e == gm.n0);
  const float kx = cc.kx_c;
  float ky, kz;
  bool ny_y;
  if constexpr (NDIM == 2) { ky = k0c; kz = 0.0f; ny_y = nyq0; }
  else { ky = cc.ky; kz = k0c; ny_y = cc.nyq_y; }
  float d1[7];
  const float H1 = lnh_partials<NDIM>(f, w, kx, ky, kz, d1);
  if (f.rotated && (cc.nyq_x || ny_y)) {
    float d2[7];
    const float H2 = lnh_partials<NDIM>(f, w, cc.nyq_x ? -kx : kx, ny_y ? -ky : ky, kz, d2);
#pragma unroll
    for (int j = 0; j < 7; ++j) dH[j] = 0.5f * (H1 * d1[j] + H2 * d2[j]);
    return 0.5f * (H1 + H2);
  }
#pragma unroll
  for (int j = 0; j < 7; ++j) dH[j] = H1 * d1[j];
  return H1;
}

// ---------------------------------------------------------------------------------------------
// axis-0 adjoint pass: forward FFT of each column of W, then the seven FP64 sums; per-tile
// partials, reduced in a fixed order by k_grad_final
// ---------------------------------------------------------------------------------------------
template <int L, int NDIM>
__global__ void __launch_bounds__((ColTile<L, 0>::T)) k_cols_adjoint(AdjointArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = ColTile<L, 0>::C, T = ColTile<L, 0>::T;
  using Rad = typename Plan<L>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  __shared__ double red[7][T / 64];
  int b;
  long long tile;
  if (!map_tile(a.sc, b, tile)) return;
  const int tid = threadIdx.x;
  const int c = tid % C, p = tid / C;
  const int g = (int)tile * C + c;
  const bool valid = g < a.gm.ncol;
  const ColIO io = col_io<L>(a.spec, a.Nh, a.gm.inner0, g, p);
  float2 v[E];
  col_load<L, R1, P, E>(v, io);
  fft_run<L, P, E, false>(Rad{}, v, lds + c * ColTile<L, 0>::RS, p, a.tw);

  // per-bin weights into LDS (the exchange buffer is free after the transform)
  double* cf = reinterpret_cast<double*>(lds);
  __syncthreads();
  for (int i = tid; i <= a.nb; i += T) cf[i] = a.coef[i];
  __syncthreads();
  const double gamma = cf[a.nb];
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (valid) {
    const ColCoord cc = col_coord(a.gm, g);
    const FiltDev f = a.filt;
#pragma unroll 4
    for (int s = 0; s < E; ++s) {
      const int e = slot_index<L, RL, P>(s, p);
      float dH[7];
      const float Hs = hsym_partials<NDIM>(f, a.width, a.gm, cc, e, dH);
      const int bin = (int)a.table[(unsigned)(g * L + e)];
      const float omega = (float)(cf[bin] - gamma);
      const float W2 = v[s].x * v[s].x + v[s].y * v[s].y;
      const float cfac = cc.wm * omega * 2.0f * Hs * W2;
#pragma unroll
      for (int j = 0; j < 7; ++j) acc[j] += (double)(cfac * dH[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const double sj = wave_sum(acc[j]);
    if ((tid & 63) == 0) red[j][tid >> 6] = sj;
  }
  __syncthreads();
  if (tid < 7) {
    double s = 0.0;
    for (int w = 0; w < T / 64; ++w) s += red[tid][w];
    a.partials[tile * 8 + tid] = s;
  }
}

template <int L>
static hipError_t launch_cols_adjoint_L(const AdjointArgs& a, hipStream_t st) {
  constexpr int T = ColTile<L, 0>::T;
  const size_t x = col_xchg_bytes<L, 0>();
  const size_t c = (size_t)(a.nb + 1) * 8;
  const size_t lds = x > c ? x : c;
  if (a.gm.ndim == 2)
    hipLaunchKernelGGL((k_cols_adjoint<L, 2>), dim3(sched_blocks(a.sc)), dim3(T), lds, st, a);
  else
    hipLaunchKernelGGL((k_cols_adjoint<L, 3>), dim3(sched_blocks(a.sc)), dim3(T), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_cols_adjoint(int L, const AdjointArgs& a, hipStream_t st) {
  switch (L) {
#define X(LL) case LL: return launch_cols_adjoint_L<LL>(a, st);
    HU_COL_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------------------------
// per-bin weights beta_b and gamma from the forward outputs and dL/dP (one workgroup)
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_grad_coef(GradCoefArgs a) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const double N = (double)a.N;
  const double mu = a.stats[0], var = a.stats[1];
  const double gtot = (var + mu * mu) * N * N;
  const double s = a.sigma_f * a.sigma_f * N;
  double gacc = 0.0;
  for (int b = tid; b < a.nb; b += 256) {
    double beta = 0.0;
    const unsigned long long cnt = a.cont_cnt[b];
    if (b < a.nb - 1 && cnt > 0 && gtot > 0.0) {
      const double cb = (double)cnt;
      const double gb = a.dL_dP[b];
      beta = gb * s / (cb * gtot);
      gacc += gb * (a.cont_sum[b] / cb) / gtot;
    }
    a.coef[b] = beta;
  }
  red[tid] = gacc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) a.coef[a.nb] = red[0];
}

hipError_t launch_grad_coef(const GradCoefArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_coef, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError();
}

// fixed-order sum of the per-tile partials into the seven gradient components
__global__ void __launch_bounds__(256) k_grad_final(GradFinalArgs a) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  for (int j = 0; j < 7; ++j) {
    double s = 0.0;
    for (int t = tid; t < a.ntiles; t += 256) s += a.partials[(long long)t * 8 + j];
    red[tid] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) red[tid] += red[tid + o];
      __syncthreads();
    }
    if (tid == 0) a.grad[j] = red[0];
    __syncthreads();
  }
}

hipError_t launch_grad_final(const GradFinalArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_final, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// expected spectrum of a filter: per-block LDS histogram of w H_sym^2 over runs of consecutive
// modes (column-major [g][n0] order, as the bin table), per-block totals, then one workgroup
// scales by sigma_f^2 N / sum w H^2 and copies the counts
// ---------------------------------------------------------------------------------------------
constexpr int FS_THREADS = 256, FS_RUN = 16;

template <int NDIM>
__global__ void __launch_bounds__(FS_THREADS) k_filter_spectrum(FilterSpecArgs a) {
  extern __shared__ double hs[];
  __shared__ double red[FS_THREADS / 64];
  const int tid = threadIdx.x;
  for (int i = tid; i < a.nb; i += FS_THREADS) hs[i] = 0.0;
  __syncthreads();
  const long long n0 = a.gm.n0;
  const long long chunk = (long long)FS_THREADS * FS_RUN;
  double tot = 0.0;
  for (long long base = (long long)blockIdx.x * chunk; base < a.Nh; base += (long long)gridDim.x * chunk) {
    const long long i0 = base + (long long)tid * FS_RUN;
    int cur = -1;
    double run = 0.0;
    for (int q = 0; q < FS_RUN; ++q) {
      const long long i = i0 + q;
      if (i >= a.Nh) break;
      const int g = (int)(i / n0);
      const int e = (int)(i - (long long)g * n0);
      const ColCoord cc = col_coord(a.gm, g);
      float lnc;
      const float H = amp_sym<NDIM>(a.filt, a.gm, cc, e, lnc);
      const double val = (double)(cc.wm * H * H);
      const int bin = (int)a.table[i];
      tot += val;
      if (bin != cur) {
        if (cur >= 0) atomicAdd(hs + cur, run);
        cur = bin;
        run = 0.0;
      }
      run += val;
    }
    if (cur >= 0) atomicAdd(hs + cur, run);
  }
  tot = wave_sum(tot);
  if ((tid & 63) == 0) red[tid >> 6] = tot;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < FS_THREADS / 64; ++w) s += red[w];
    a.partials[blockIdx.x] = s;
  }
  for (int i = tid; i < a.nb; i += FS_THREADS)
    if (hs[i] != 0.0) atomicAdd(a.sum + i, hs[i]);
}

__global__ void __launch_bounds__(256) k_filter_spectrum_final(FilterSpecArgs a) {
  __shared__ double red[256];
  __shared__ double fac;
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int t = tid; t < a.nblocks; t += 256) s += a.partials[t];
  red[tid] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) fac = red[0] > 0.0 ? a.sigma_f * a.sigma_f * (double)a.N / red[0] : 0.0;
  __syncthreads();
  for (int i = tid; i < a.nb; i += 256) {
    a.sum[i] *= fac;
    if (a.cnt) a.cnt[i] = a.counts[i];
  }
}

hipError_t launch_filter_spectrum(const FilterSpecArgs& a, hipStream_t st) {
  const size_t lds = (size_t)a.nb * 8;
  if (a.gm.ndim == 2)
    hipLaunchKernelGGL(k_filter_spectrum<2>, dim3(a.nblocks), dim3(FS_THREADS), lds, st, a);
  else
    hipLaunchKernelGGL(k_filter_spectrum<3>, dim3(a.nblocks), dim3(FS_THREADS), lds, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_filter_spectrum_final, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace hu
