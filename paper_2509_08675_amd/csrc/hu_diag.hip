// Hyperuniformity diagnostics (Sec. II.A): the local variance of Eq. (1) over a spherical window,
// in its Fourier form
//   sigma^2(R) = sum_{m != 0} |X(m)|^2 / N^2 W(|k_m| R)^2,   W = 2 J_1(u)/u (2D), 3 (sin u - u cos u)/u^3 (3D),
// evaluated on the half spectrum with the multiplicities w_m in the axis-0 pass (the last forward
// axis, after the same row and y passes as the power spectrum), and the host-side exponent fit
// and class table.
#include <cmath>

#include "hu_common.hpp"

namespace hu {

// W^2 at u = |k| R in FP32.
// 2D: J_1 by the polynomial approximations of Abramowitz & Stegun (Handbook of Mathematical
// Functions, 9.4.4 for u <= 3: J_1(u)/u as a polynomial in (u/3)^2, |error| < 1.3e-8; 9.4.6 for
// u > 3: J_1(u) = u^(-1/2) f_1 cos(theta_1), f_1 and theta_1 - u polynomials in 3/u, absolute error
// of J_1 below 1e-7), so W = 2 J_1(u) / u costs a few fused multiply-adds and three hardware
// transcendentals.
// 3D: below u = 1 the closed form loses digits to cancellation, so the Taylor series
// 3 sum_{n>=1} (-1)^(n+1) 2n u^(2n-2) / (2n+1)! (through u^10; the next term is below 3.3e-11 at
// u = 1) is used there; above, the closed form with the hardware sine and cosine.
template <int NDIM>
__device__ __forceinline__ float window_w2(float u) {
  float w;
  if constexpr (NDIM == 2) {
    if (u <= 3.0f) {
      const float t = (u * (1.0f / 3.0f)) * (u * (1.0f / 3.0f));
      w = 2.0f * (0.5f + t * (-0.56249985f + t * (0.21093573f + t * (-0.03954289f +
                                     t * (0.00443319f + t * (-0.00031761f + t * 0.00001109f))))));
    } else {
      const float y = 3.0f * __builtin_amdgcn_rcpf(u);
      const float f1 = 0.79788456f + y * (0.00000156f + y * (0.01659667f + y * (0.00017105f +
                                     y * (-0.00249511f + y * (0.00113653f + y * (-0.00020033f))))));
      const float th = (u - 2.35619449f) + y * (0.12499612f + y * (0.00005650f + y * (-0.00637879f +
                                     y * (0.00074348f + y * (0.00079824f + y * (-0.00029166f))))));
      const float ru = __builtin_amdgcn_rsqf(u);
      w = 2.0f * f1 * __cosf(th) * ru * ru * ru;
    }
  } else {
    if (u < 1.0f) {
      const float t = u * u;
      w = 1.0f + t * (-1.0f / 10.0f + t * (1.0f / 280.0f + t * (-1.0f / 15120.0f +
                                              t * (1.0f / 1330560.0f + t * (-1.0f / 172972800.0f)))));
    } else {
      float s, c;
      __sincosf(u, &s, &c);           // hardware sin / cos: ~1e-7 absolute, W is O(u^-2) beyond
      const float ri = __builtin_amdgcn_rcpf(u);
      w = 3.0f * (s - u * c) * (ri * ri * ri);
    }
  }
  return w * w;
}

template <int L, int NDIM>
__global__ void __launch_bounds__((ColTile<L, 0>::T)) k_cols_wvar(WvarArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = ColTile<L, 0>::C, T = ColTile<L, 0>::T;
  using Rad = typename Plan<L>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  constexpr float PI = 3.14159265358979323846f;
  extern __shared__ float2 lds[];
  __shared__ double red[HU_MAX_RADII][T / 64];
  int b;
  long long tile;
  if (!map_tile(a.sc, b, tile)) return;
  const int tid = threadIdx.x;
  const int c = tid % C, p = tid / C;
  const int g = (int)tile * C + c;
  const bool valid = g < a.gm.ncol;
  const ColIO io = col_io<L>(a.spec + (long long)b * a.Nh, a.Nh, a.gm.inner0, g, p);
  float2 v[E];
  col_load<L, R1, P, E>(v, io);
  fft_run<L, P, E, false>(Rad{}, v, lds + c * ColTile<L, 0>::RS, p, a.tw);
  // per slot: w_m |X|^2 (0 for the mean mode and for columns past the end) and |k| = pi |kappa|
  const ColCoord cc = col_coord(a.gm, valid ? g : 0);
  const float kfix2 = NDIM == 3 ? cc.kx_c * cc.kx_c + cc.ky * cc.ky : cc.kx_c * cc.kx_c;
  const bool col0 = cc.mx == 0 && (NDIM == 2 || cc.my == 0);
  float pw[E], kk[E];
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int e = slot_index<L, RL, P>(s, p);
    const int mt = e < a.gm.n0 / 2 ? e : e - a.gm.n0;
    const float k0 = (float)mt * a.gm.kap0;
    kk[s] = PI * sqrtf(fmaf(k0, k0, kfix2));
    pw[s] = (valid && !(col0 && e == 0)) ? cc.wm * (v[s].x * v[s].x + v[s].y * v[s].y) : 0.0f;
  }
  for (int j = 0; j < a.nr; ++j) {
    const float R = a.radii[j];
    double acc = 0.0;
#pragma unroll 4
    for (int s = 0; s < E; ++s) acc += (double)(pw[s] * window_w2<NDIM>(kk[s] * R));
    acc = wave_sum(acc);
    if ((tid & 63) == 0) red[j][tid >> 6] = acc;
  }
  __syncthreads();
  if (tid < a.nr) {
    double s = 0.0;
    for (int w = 0; w < T / 64; ++w) s += red[tid][w];
    a.partials[((long long)b * a.sc.ntiles + tile) * a.nr + tid] = s;
  }
}

template <int L>
static hipError_t launch_cols_wvar_L(const WvarArgs& a, hipStream_t st) {
  constexpr int T = ColTile<L, 0>::T;
  if (a.gm.ndim == 2)
    hipLaunchKernelGGL((k_cols_wvar<L, 2>), dim3(sched_blocks(a.sc)), dim3(T), (col_xchg_bytes<L, 0>()), st, a);
  else
    hipLaunchKernelGGL((k_cols_wvar<L, 3>), dim3(sched_blocks(a.sc)), dim3(T), (col_xchg_bytes<L, 0>()), st, a);
  return hipGetLastError();
}

hipError_t launch_cols_wvar(int L, const WvarArgs& a, hipStream_t st) {
  switch (L) {
#define X(LL) case LL: return launch_cols_wvar_L<LL>(a, st);
    HU_COL_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

// out[b][j] = scale * (sum over the tiles of field b, in tile order, of partial j): one workgroup
// per field; thread t sums tiles t, t + 256, ... for every radius, then waves and the workgroup
// reduce in a fixed order
__global__ void __launch_bounds__(256) k_wvar_final(WvarFinalArgs a) {
  __shared__ double red[HU_MAX_RADII][4];
  const int b = blockIdx.x, tid = threadIdx.x;
  const double* part = a.partials + (long long)b * a.ntiles * a.nr;
  for (int j = 0; j < a.nr; ++j) {
    double s = 0.0;
    for (int t = tid; t < a.ntiles; t += 256) s += part[(long long)t * a.nr + j];
    s = wave_sum(s);
    if ((tid & 63) == 0) red[j][tid >> 6] = s;
  }
  __syncthreads();
  if (tid < a.nr) a.out[(long long)b * a.nr + tid] = a.scale * (((red[tid][0] + red[tid][1]) + red[tid][2]) + red[tid][3]);
}

hipError_t launch_wvar_final(const WvarFinalArgs& a, int batch, hipStream_t st) {
  hipLaunchKernelGGL(k_wvar_final, dim3(batch), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace hu
