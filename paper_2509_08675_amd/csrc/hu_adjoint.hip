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

// ln H (relative) and its derivatives.  With u_i = |kappa'_i| / a_i, K = (sum_i u_i^p)^(1/p),
// r_i = u_i / K and D = d lnH/dK = (alpha / K - (K - k0) / w^2) / 2:
//   d lnH/da_i = -D K r_i^p / a_i
//   d lnH/dp   = D (K / p) sum_i r_i^p ln r_i
//   d lnH/drot = D K (r_x^p kappa'_y / kappa'_x - r_y^p kappa'_x / kappa'_y)
//                (d kappa'_x / drot = kappa'_y, d kappa'_y / drot = -kappa'_x, r^(p-1) = r^p K / u)
//   d lnH/dk0  = (K - k0) / (2 w^2),   d lnH/dw = (K - k0)^2 / (2 w^3)
// Every K term carries the factor D K = alpha / 2 - K (K - k0) / (2 w^2), so 1/K is never formed.  Powers are taken relative to the largest u_i in the log2 domain: t_i = 2^(p (l_i - l_m)),
// l_i = log2 u_i, so r_i^p = t_i / S with S = sum_i t_i in [1, 3], and K = 2^(l_m + log2(S) / p).
// Axes with u_i = 0 contribute nothing (t_i = 0, their l_i is a finite sentinel).
constexpr float LOG_OFF = -1.0e4f;

// H and the seven derivatives of ln H without their per-filter constant factors:
//   d lnH/dtheta_j = kf_j r_j,  r = (DK t_x, DK t_y, DK t_z, DK sum_i t_i (l_i - log2 K), DK (t_x A - t_y B),
//                                    K - k0, (K - k0)^2),
//   kf = (-1/a, -1/b, -1/c, ln2 / p, 1, 1/(2 w^2), 1/(2 w^3)),  t_i = r_i^p,  DK = D K
// (A, B as in dK/drot above); the factors are applied once per thread after the sums.
struct LnhOut {
  float H;
  float r[7];
};

__device__ __forceinline__ void lnh_tail(const FiltDev& f, float lm, float S, const float (&rp)[3], const float (&l)[3],
                                         float A, float B, LnhOut& o) {
  constexpr float LN2 = 0.69314718055994531f;
  const float log2K = fmaf(hw_log2(S), f.ip, lm);
  const float K = hw_exp2(log2K);
  const float dd = K - f.k0;
  const float d5 = dd * f.inv2w2;
  o.H = amp_from_lnchi(fmaf(f.alpha, log2K * LN2, -fmaf(dd, d5, f.lnchimax)));
  const float KD = fmaf(-2.0f * K, d5, f.alpha) * 0.5f;
  const float accp = fmaf(rp[0], l[0] - log2K, fmaf(rp[1], l[1] - log2K, rp[2] * (l[2] - log2K)));
  o.r[0] = KD * rp[0];
  o.r[1] = KD * rp[1];
  o.r[2] = KD * rp[2];
  o.r[3] = KD * accp;
  o.r[4] = KD * fmaf(rp[0], A, -rp[1] * B);
  o.r[5] = dd;
  o.r[6] = dd * dd;
}

__device__ __forceinline__ void lnh_zero(LnhOut& o) {
  o.H = 0.0f;
#pragma unroll
  for (int j = 0; j < 7; ++j) o.r[j] = 0.0f;
}

// 2D: both in-plane components vary along an axis-0 column
__device__ __forceinline__ void lnh2(const FiltDev& f, float kx, float ky, LnhOut& o) {
  const float kxr = fmaf(f.cr, kx, f.sr * ky);
  const float kyr = fmaf(-f.sr, kx, f.cr * ky);
  const float u0 = fabsf(kxr) * f.ia, u1 = fabsf(kyr) * f.ib;
  const bool on0 = u0 > 0.0f, on1 = u1 > 0.0f;
  if (!(on0 || on1)) {
    lnh_zero(o);
    return;
  }
  float l[3];
  l[0] = on0 ? hw_log2(u0) : LOG_OFF;
  l[1] = on1 ? hw_log2(u1) : LOG_OFF;
  l[2] = LOG_OFF;
  const bool big0 = l[0] >= l[1];
  const float lm = big0 ? l[0] : l[1];
  const float lo = big0 ? l[1] : l[0];
  const float t = (on0 && on1) ? hw_exp2(f.p * (lo - lm)) : 0.0f;
  const float S = 1.0f + t;
  const float iS = __builtin_amdgcn_rcpf(S);
  const float rp[3] = {big0 ? iS : t * iS, big0 ? t * iS : iS, 0.0f};
  const float r = (on0 && on1) ? __builtin_amdgcn_rcpf(kxr * kyr) : 0.0f;
  lnh_tail(f, lm, S, rp, l, kyr * kyr * r, kxr * kxr * r, o);
}

// 3D: kappa_x and kappa_y are fixed along an axis-0 column, so their logs and relative powers
// are computed once per column
struct Lnh3Col {
  float l0, l1, lxy;   // log2 u_x, log2 u_y (or the sentinel), their maximum
  float c0, c1, c01;   // 2^(p (l_i - lxy)), their sum (0 when both are off)
  float A, B;          // kappa'_y / kappa'_x and kappa'_x / kappa'_y (0 for an axis that is off)
  bool on;             // u_x > 0 or u_y > 0
};

__device__ __forceinline__ Lnh3Col lnh3_col(const FiltDev& f, float kx, float ky) {
  Lnh3Col c;
  const float kxr = fmaf(f.cr, kx, f.sr * ky);
  const float kyr = fmaf(-f.sr, kx, f.cr * ky);
  const float u0 = fabsf(kxr) * f.ia, u1 = fabsf(kyr) * f.ib;
  const bool on0 = u0 > 0.0f, on1 = u1 > 0.0f;
  c.on = on0 || on1;
  c.l0 = on0 ? hw_log2(u0) : LOG_OFF;
  c.l1 = on1 ? hw_log2(u1) : LOG_OFF;
  c.lxy = fmaxf(c.l0, c.l1);
  c.c0 = on0 ? hw_exp2(f.p * (c.l0 - c.lxy)) : 0.0f;
  c.c1 = on1 ? hw_exp2(f.p * (c.l1 - c.lxy)) : 0.0f;
  c.c01 = c.c0 + c.c1;
  c.A = on0 ? kyr / kxr : 0.0f;
  c.B = on1 ? kxr / kyr : 0.0f;
  return c;
}

__device__ __forceinline__ void lnh3(const FiltDev& f, const Lnh3Col& c, float kz, LnhOut& o) {
  const float u2 = fabsf(kz) * f.ic;
  const bool on2 = u2 > 0.0f;
  if (!(on2 || c.on)) {
    lnh_zero(o);
    return;
  }
  float l[3] = {c.l0, c.l1, on2 ? hw_log2(u2) : LOG_OFF};
  // z the largest: t_z = 1 and the in-plane powers scale by 2^(p (l_xy - l_z)); else t_z = 2^(p (l_z - l_xy))
  const bool zbig = !c.on || (on2 && l[2] > c.lxy);
  const float e = hw_exp2(-f.p * fabsf(l[2] - c.lxy));
  const float g = zbig ? e : 1.0f;
  const float t2 = zbig ? 1.0f : (on2 ? e : 0.0f);
  const float lm = zbig ? l[2] : c.lxy;
  const float S = fmaf(g, c.c01, t2);
  const float iS = __builtin_amdgcn_rcpf(S);
  const float gi = g * iS;
  const float rp[3] = {c.c0 * gi, c.c1 * gi, t2 * iS};
  lnh_tail(f, lm, S, rp, l, c.A, c.B, o);
}

// ---------------------------------------------------------------------------------------------
// axis-0 adjoint pass: forward FFT of each column of W, then the seven FP64 sums; per-tile
// partials, reduced in a fixed order by k_grad_final
// ---------------------------------------------------------------------------------------------
// LDS layout of the per-mode phase: |W|^2 as [C][PS] floats, the tile's bin-table slice as [C][TS]
// entries, then the per-bin weights.  A half wave covers 16 columns x 2 threads of a column, and
// the threads of a column read neighbouring modes; a column stride of 2 mod 32 words puts the 32
// reads of a half wave into distinct banks (the table's two threads share a word).
template <int L>
struct AdjLds {
  static constexpr int C = ColTile<L, 0>::C;
  static constexpr int PS = (L + 31) / 32 * 32 + 2;
  static constexpr int TS = (L + 63) / 64 * 64 + 4;
  static constexpr size_t fixed = (size_t)C * PS * 4 + (size_t)C * TS * 2;
};

// per-mode accumulation: one evaluation of H, or the mean of two on a Nyquist plane of a rotated
// filter (H_sym, differentiated term by term); cb = w_m omega 2 |W|^2
// a mode's seven terms into the thread's FP32 partials of one tile (its E modes); the partials go
// into the FP64 sums once per tile
__device__ __forceinline__ void adj_acc(float (&acc)[7], float cb, const LnhOut& o) {
  const float wt = cb * o.H * o.H;
#pragma unroll
  for (int j = 0; j < 7; ++j) acc[j] = fmaf(wt, o.r[j], acc[j]);
}
__device__ __forceinline__ void adj_acc2(float (&acc)[7], float cb, const LnhOut& o1, const LnhOut& o2) {
  const float hs = 0.5f * (o1.H + o2.H);
  const float w1 = 0.5f * cb * hs * o1.H, w2 = 0.5f * cb * hs * o2.H;
#pragma unroll
  for (int j = 0; j < 7; ++j) acc[j] += fmaf(w1, o1.r[j], w2 * o2.r[j]);
}

// Persistent over tiles (tile = blockIdx.x + k gridDim.x, a fixed assignment, so the sums are
// reproducible): each tile's columns are transformed, |W|^2 and the tile's bin-table slice go to
// LDS, the next tile's columns are requested into the transform's registers, and the per-mode sums
// run while they arrive.  One row of partials per workgroup.
template <int L, int NDIM>
__global__ void __launch_bounds__((ColTile<L, 0>::T)) k_cols_adjoint(AdjointArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = ColTile<L, 0>::C, T = ColTile<L, 0>::T;
  constexpr int PS = AdjLds<L>::PS, TS = AdjLds<L>::TS;
  static_assert(E % 2 == 0, "the 3D pairs of modes split a thread's E modes in halves");
  using Rad = typename Plan<L>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  constexpr float LN2 = 0.69314718055994531f;
  extern __shared__ float2 lds[];
  __shared__ double red[7][T / 64];
  const int tid = threadIdx.x;
  const int c = tid % C, p = tid / C;
  const int n0 = a.gm.n0;
  float* pw = reinterpret_cast<float*>(lds);
  uint16_t* tb = reinterpret_cast<uint16_t*>(pw + C * PS);
  double* cf = reinterpret_cast<double*>(reinterpret_cast<char*>(lds) + a.cf_off);
  for (int i = tid; i <= a.nb; i += T) cf[i] = a.coef[i];
  const FiltDev f = a.filt;
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int tile = blockIdx.x;
  float2 v[E];
  col_load<L, R1, P, E>(v, col_io<L>(a.spec, a.Nh, a.gm.inner0, tile * C + c, p));
  for (; tile < a.ntiles; tile += gridDim.x) {
    const int g = tile * C + c;
    fft_run<L, P, E, false>(Rad{}, v, lds + c * ColTile<L, 0>::RS, p, a.tw);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < E; ++s) pw[c * PS + slot_index<L, RL, P>(s, p)] = v[s].x * v[s].x + v[s].y * v[s].y;
    {
      const int g0 = tile * C;
      const int ncv = a.gm.ncol - g0 < C ? a.gm.ncol - g0 : C;
      const uint16_t* src = a.table + (size_t)g0 * L;
      if constexpr (NDIM == 3 && L % 16 == 0) {
        // the pairs below read the bins of modes 0 .. L/2 only: the first L/16 + 1 chunks of 8
        constexpr int HC = L / 16 + 1;
        for (int i = tid; i < ncv * HC; i += T) {
          const int col = i / HC, ch = i - col * HC;
          const uint4 w = reinterpret_cast<const uint4*>(src + (size_t)col * L)[ch];
          uint32_t* d = reinterpret_cast<uint32_t*>(tb + col * TS + 8 * ch);
          d[0] = w.x;
          d[1] = w.y;
          d[2] = w.z;
          d[3] = w.w;
        }
      } else if constexpr (L % 8 == 0) {
        for (int i = tid; i < ncv * (L / 8); i += T) {
          const uint4 w = reinterpret_cast<const uint4*>(src)[i];
          uint32_t* d = reinterpret_cast<uint32_t*>(tb + ((8 * i) / L) * TS + (8 * i) % L);
          d[0] = w.x;
          d[1] = w.y;
          d[2] = w.z;
          d[3] = w.w;
        }
      } else {
        for (int i = tid; i < ncv * L; i += T) tb[(i / L) * TS + i % L] = src[i];
      }
    }
    __syncthreads();
    if (tile + (int)gridDim.x < a.ntiles)
      col_load<L, R1, P, E>(v, col_io<L>(a.spec, a.Nh, a.gm.inner0, (tile + (int)gridDim.x) * C + c, p));
    if (g < a.gm.ncol) {
      float pa[7] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
      const ColCoord cc = col_coord(a.gm, g);
      const double gamma = cf[a.nb];
      const float* pc = pw + c * PS;
      const uint16_t* tc = tb + c * TS;
      const float kx = cc.kx_c;
      const float wm2 = 2.0f * cc.wm;
      if constexpr (NDIM == 3) {
        // kappa_z enters ln H only through |kappa_z| (the rotation is about z) and the radial bin
        // only through kappa_z^2: the modes e and n0 - e share H, its derivatives and their bin, so
        // each pair is evaluated once with the sum of the two |W|^2.  Thread p takes the pairs
        // q = p + P k, k < E / 2 (q < n0 / 2); thread 0 also takes q = n0 / 2.  q = 0 and q = n0 / 2
        // are their own partners.
        const bool partner = f.rotated && (cc.nyq_x || cc.nyq_y);
        const Lnh3Col c1 = lnh3_col(f, kx, cc.ky);
        const Lnh3Col c2 = partner ? lnh3_col(f, cc.nyq_x ? -kx : kx, cc.nyq_y ? -cc.ky : cc.ky) : c1;
        constexpr int NP = E / 2 + 1;
#pragma unroll 2
        for (int k = 0; k < NP; ++k) {
          const int q = k < E / 2 ? p + P * k : (p == 0 ? n0 / 2 : -1);
          if (q < 0) continue;
          const float kz = (float)q * a.gm.kap0;
          const float w2 = (q == 0 || 2 * q == n0) ? pc[q] : pc[q] + pc[n0 - q];
          const float cb = wm2 * (float)(cf[tc[q]] - gamma) * w2;
          LnhOut o1;
          lnh3(f, c1, kz, o1);
          if (partner) {
            LnhOut o2;
            lnh3(f, c2, kz, o2);
            adj_acc2(pa, cb, o1, o2);
          } else {
            adj_acc(pa, cb, o1);
          }
        }
      } else {
#pragma unroll 2
        for (int k = 0; k < E; ++k) {
          const int e = p + P * k;
          const float ky = (float)(e < n0 / 2 ? e : e - n0) * a.gm.kap0;
          const float cb = wm2 * (float)(cf[tc[e]] - gamma) * pc[e];
          LnhOut o1;
          lnh2(f, kx, ky, o1);
          if (f.rotated && (cc.nyq_x || 2 * e == n0)) {
            LnhOut o2;
            lnh2(f, cc.nyq_x ? -kx : kx, 2 * e == n0 ? -ky : ky, o2);
            adj_acc2(pa, cb, o1, o2);
          } else {
            adj_acc(pa, cb, o1);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 7; ++j) acc[j] += (double)pa[j];
    }
    __syncthreads();
  }
  // the per-filter factors of the seven terms
  const double kf[7] = {-(double)f.ia, -(double)f.ib, -(double)f.ic, (double)(LN2 * f.ip), 1.0, (double)f.inv2w2,
                        (double)f.inv2w2 / (double)a.width};
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const double sj = wave_sum(acc[j] * kf[j]);
    if ((tid & 63) == 0) red[j][tid >> 6] = sj;
  }
  __syncthreads();
  if (tid < 7) {
    double s = 0.0;
    for (int w = 0; w < T / 64; ++w) s += red[tid][w];
    a.partials[(long long)blockIdx.x * 8 + tid] = s;
  }
}

template <int L>
static size_t adjoint_cf_off() {
  const size_t x = col_xchg_bytes<L, 0>();
  const size_t f = AdjLds<L>::fixed;
  return ((x > f ? x : f) + 15) / 16 * 16;
}

template <int L>
static hipError_t launch_cols_adjoint_L(AdjointArgs a, hipStream_t st, int* grid_out) {
  constexpr int T = ColTile<L, 0>::T;
  a.cf_off = (int)adjoint_cf_off<L>();
  const size_t lds = (size_t)a.cf_off + (size_t)(a.nb + 1) * 8;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const void* kern = a.gm.ndim == 2 ? reinterpret_cast<const void*>(&k_cols_adjoint<L, 2>)
                                    : reinterpret_cast<const void*>(&k_cols_adjoint<L, 3>);
  int slots = 0;
  const hipError_t e = resident_blocks(kern, T, lds, &slots);
  if (e != hipSuccess) return e;
  const int grid = a.ntiles < slots ? a.ntiles : slots;
  *grid_out = grid;
  if (a.gm.ndim == 2)
    hipLaunchKernelGGL((k_cols_adjoint<L, 2>), dim3(grid), dim3(T), lds, st, a);
  else
    hipLaunchKernelGGL((k_cols_adjoint<L, 3>), dim3(grid), dim3(T), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_cols_adjoint(int L, const AdjointArgs& a, hipStream_t st, int* grid) {
  switch (L) {
#define X(LL) case LL: return launch_cols_adjoint_L<LL>(a, st, grid);
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

// ---------------------------------------------------------------------------------------------
// spectrum-matching loss (one workgroup, fixed-order reduction):
//   L = (1/|B|) sum_{b in B} d_b^2,  d_b = ln(P_b + eps) - ln(T_b + eps),
//   dL/dP_b = 2 d_b / (|B| (P_b + eps)),
// P_b, T_b the bin means of the field's and the target's spectra, B the bins of radius r >= 1 that
// hold modes in both (the DC row and the corner slot excluded)
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_spectrum_loss(LossArgs a) {
  __shared__ double red[256];
  __shared__ unsigned cnt_used[256];
  __shared__ double nb_used;
  const int tid = threadIdx.x;
  double acc = 0.0;
  unsigned used = 0;
  for (int b = tid; b < a.nb - 1; b += 256) {
    const bool on = b >= a.na && a.cnt[b] > 0 && a.tcnt[b] > 0;
    if (on) {
      const double P = a.sum[b] / (double)a.cnt[b], T = a.tsum[b] / (double)a.tcnt[b];
      const double d = log(P + a.eps) - log(T + a.eps);
      acc += d * d;
      ++used;
    }
  }
  red[tid] = acc;
  cnt_used[tid] = used;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      red[tid] += red[tid + o];
      cnt_used[tid] += cnt_used[tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    nb_used = (double)cnt_used[0];
    a.loss[0] = cnt_used[0] ? red[0] / nb_used : 0.0;
  }
  __syncthreads();
  for (int b = tid; b < a.nb; b += 256) {
    double g = 0.0;
    if (b < a.nb - 1 && b >= a.na && a.cnt[b] > 0 && a.tcnt[b] > 0 && nb_used > 0.0) {
      const double P = a.sum[b] / (double)a.cnt[b], T = a.tsum[b] / (double)a.tcnt[b];
      g = 2.0 * (log(P + a.eps) - log(T + a.eps)) / (nb_used * (P + a.eps));
    }
    a.dL_dP[b] = g;
  }
}

hipError_t launch_spectrum_loss(const LossArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_spectrum_loss, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError();
}

// fixed-order sum of the per-tile partials into the seven gradient components: each thread sums
// whole partial rows (tiles tid, tid + 1024, ...), then waves and the workgroup reduce in a fixed
// order
constexpr int GF_THREADS = 1024;

__global__ void __launch_bounds__(GF_THREADS) k_grad_final(GradFinalArgs a) {
  __shared__ double red[7][GF_THREADS / 64];
  const int tid = threadIdx.x;
  double s[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int t = tid; t < a.ntiles; t += GF_THREADS) {
    const double2* row = reinterpret_cast<const double2*>(a.partials + (long long)t * 8);
    const double2 q0 = row[0], q1 = row[1], q2 = row[2], q3 = row[3];
    s[0] += q0.x;
    s[1] += q0.y;
    s[2] += q1.x;
    s[3] += q1.y;
    s[4] += q2.x;
    s[5] += q2.y;
    s[6] += q3.x;
  }
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const double w = wave_sum(s[j]);
    if ((tid & 63) == 0) red[j][tid >> 6] = w;
  }
  __syncthreads();
  if (tid < 7) {
    double r = 0.0;
    for (int w = 0; w < GF_THREADS / 64; ++w) r += red[tid][w];
    a.grad[tid] = r;
  }
}

hipError_t launch_grad_final(const GradFinalArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_final, dim3(1), dim3(GF_THREADS), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Expected spectrum of a filter, deterministic.  The modes in column-major [g][n0] order (the
// order of the bin table) are taken in chunks of FS_THREADS x FS_RUN, chunk c by workgroup
// c mod gridDim.x; thread t of a chunk evaluates w H_sym^2 of its FS_RUN consecutive modes (FP32,
// widened to FP64) and sums each run of equal bins in FP64 in mode order.  The runs of a chunk are
// combined per bin in integer arithmetic (largest binary exponent, then fixed-point adds at
// 2^(exponent - 48), as in the tile binning of the axis-0 passes), so the chunk's bin sums do not
// depend on the order of the atomics; each bin's slot of the workgroup's partial row is owned by
// one thread, which adds the chunk sums in chunk order.  k_filter_spectrum_final then sums the
// rows in workgroup order and scales by sigma_f^2 N / sum w H^2.
// ---------------------------------------------------------------------------------------------
constexpr int FS_THREADS = 256, FS_RUN = 16;

template <int NDIM>
__global__ void __launch_bounds__(FS_THREADS) k_filter_spectrum(FilterSpecArgs a) {
  extern __shared__ unsigned long long hq[];      // [nb] fixed-point sums, then [nb] int exponents
  int* hx = reinterpret_cast<int*>(hq + a.nb);
  __shared__ double red[FS_THREADS / 64];
  const int tid = threadIdx.x;
  double* row = a.rows + (long long)blockIdx.x * a.nb;
  for (int i = tid; i < a.nb; i += FS_THREADS) {
    hx[i] = HX_EMPTY;
    hq[i] = 0ull;
    row[i] = 0.0;
  }
  const long long n0 = a.gm.n0;
  const long long chunk = (long long)FS_THREADS * FS_RUN;
  double tot = 0.0;
  for (long long base = (long long)blockIdx.x * chunk; base < a.Nh; base += (long long)gridDim.x * chunk) {
    const long long i0 = base + (long long)tid * FS_RUN;
    int bin[FS_RUN];
    double val[FS_RUN];
#pragma unroll
    for (int q = 0; q < FS_RUN; ++q) {
      const long long i = i0 + q;
      bin[q] = -1;
      val[q] = 0.0;
      if (i < a.Nh) {
        const int g = (int)(i / n0);
        const int e = (int)(i - (long long)g * n0);
        const ColCoord cc = col_coord(a.gm, g);
        float lnc;
        const float H = amp_sym<NDIM, true>(a.filt, a.gm, cc, e, lnc);
        val[q] = (double)(cc.wm * H * H);
        bin[q] = (int)a.table[i];
        tot += val[q];
      }
    }
    __syncthreads();                               // the previous chunk's flush is done
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      int cur = -1;
      double run = 0.0;
#pragma unroll
      for (int q = 0; q < FS_RUN; ++q) {
        if (bin[q] != cur) {
          if (cur >= 0) pass ? run_commit<true>(cur, run, hx, hq) : run_commit<false>(cur, run, hx, hq);
          cur = bin[q];
          run = 0.0;
        }
        run += val[q];
      }
      if (cur >= 0) pass ? run_commit<true>(cur, run, hx, hq) : run_commit<false>(cur, run, hx, hq);
      __syncthreads();
    }
    for (int i = tid; i < a.nb; i += FS_THREADS) {
      const int ex = hx[i];
      if (ex != HX_EMPTY) {
        row[i] += ldexp((double)hq[i], ex - HQ_SHIFT);
        hx[i] = HX_EMPTY;
        hq[i] = 0ull;
      }
    }
  }
  tot = wave_sum(tot);
  if ((tid & 63) == 0) red[tid >> 6] = tot;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < FS_THREADS / 64; ++w) s += red[w];
    a.partials[blockIdx.x] = s;
  }
}

// one wave per bin: lane l adds rows l, l + 64, ... in order, then a fixed butterfly; every
// workgroup forms the same total of the per-workgroup sums
__global__ void __launch_bounds__(256) k_filter_spectrum_final(FilterSpecArgs a) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int t = tid; t < a.nblocks; t += 256) s += a.partials[t];
  red[tid] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  const double fac = red[0] > 0.0 ? a.sigma_f * a.sigma_f * (double)a.N / red[0] : 0.0;
  const int i = blockIdx.x * 4 + (tid >> 6), lane = tid & 63;
  if (i >= a.nb) return;
  double b = 0.0;
  for (int r = lane; r < a.nblocks; r += 64) b += a.rows[(long long)r * a.nb + i];
  b = wave_sum(b);
  if (lane == 0) {
    a.sum[i] = b * fac;
    if (a.cnt) a.cnt[i] = a.counts[i];
  }
}

hipError_t launch_filter_spectrum(const FilterSpecArgs& a, hipStream_t st) {
  const size_t lds = (size_t)a.nb * 12;
  if (a.gm.ndim == 2)
    hipLaunchKernelGGL(k_filter_spectrum<2>, dim3(a.nblocks), dim3(FS_THREADS), lds, st, a);
  else
    hipLaunchKernelGGL(k_filter_spectrum<3>, dim3(a.nblocks), dim3(FS_THREADS), lds, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_filter_spectrum_final, dim3((a.nb + 3) / 4), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace hu
