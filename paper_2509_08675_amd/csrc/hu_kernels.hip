// HIP kernels of the hyperuniform-field hot path (gfx950).
//
// Passes over the FP32 half spectrum S (per field: n_0 x ... x n_{d-2} x (n_x/2+1) complex, row-major):
//   rows_r2c   white noise (or a real input) -> real-to-complex transform of each x row
//              (an n_x/2-point complex FFT on the packed even/odd samples plus the split twist);
//   cols       complex transform along a strided axis, forward or inverse, in place;
//   cols_filter forward transform along axis 0, multiply by the symmetrised amplitude
//              (Eq. (8) with Eqs. (12)-(13)), FP64 Parseval statistics, the continuous-field
//              spectrum bins, inverse transform along axis 0 -- one read and one write;
//   cols_bin   forward transform along axis 0 and the binned periodogram, read only;
//   rows_c2r   complex-to-real transform of each x row, normalisation (Eq. (15)) with the
//              statistics of the filter pass, FP32 field out, sign map out with counts, and the
//              real-to-complex transform of the +-1 row back into S.
#include "hu_device.hpp"
#include "hu_internal.hpp"

namespace hu {

// ---------------------------------------------------------------------------------------------
// tile widths: transforms per workgroup
// ---------------------------------------------------------------------------------------------
template <int L>
struct RowTile {
  static constexpr int P = Plan<L>::P;
  static constexpr int c0 = 256 / P > 0 ? 256 / P : 1;
  static constexpr int cl = 8192 / (L + 1) > 0 ? 8192 / (L + 1) : 1;
  static constexpr int C = c0 < cl ? c0 : cl;
  static constexpr int T = C * P;
};

template <int L>
struct ColTile {
  static constexpr int P = Plan<L>::P;
  static constexpr int a = 8192 / L < 32 ? 8192 / L : 32;
  static constexpr int b = 64 / P > a ? 64 / P : a;
  static constexpr int C = b * P > 1024 ? 1024 / P : b;
  static constexpr int T = C * P;
};

// ---------------------------------------------------------------------------------------------
// block reductions
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ unsigned wave_usum(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------------------------
// R2C split twist: from Z = FFT_L(x[2n] + i x[2n+1]) held in LDS (natural order), write
// X[k] = (Z[k] + Z*[L-k])/2 - (i/2) e^{-2 pi i k / 2L} (Z[k] - Z*[L-k]), k = 0..L, to `out`.
// ---------------------------------------------------------------------------------------------
template <int L, int P, int E>
__device__ __forceinline__ void r2c_twist_store(const float2* lz, const float2* __restrict__ tw2, float2* out,
                                                int p, bool valid) {
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int k = p + P * i;
    const float2 zk = lz[k];
    const float2 zm = cconj(lz[(L - k) % L]);
    const float2 A = cadd(zk, zm), B = csub(zk, zm);
    const float2 X = cscale(cadd(A, mul_mi<false>(cmul(tw2[k], B))), 0.5f);
    if (valid) out[k] = X;
    if (k == 0 && valid) out[L] = make_float2(zk.x - zk.y, 0.0f);
  }
}

// =============================================================================================
// rows_r2c: source -> R2C along x.   grid (ceil(nrows / C), B), block C * P.
// =============================================================================================
template <int L, int SRC>
__global__ void __launch_bounds__(RowTile<L>::T) k_rows_r2c(RowsArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = RowTile<L>::C, T = RowTile<L>::T;
  using Rad = typename Plan<L>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  float* ldsf = reinterpret_cast<float*>(lds);
  const int tid = threadIdx.x;
  const int c = tid / P, p = tid % P;
  const int b = blockIdx.y;
  const long long row0 = (long long)blockIdx.x * C;
  const long long row = row0 + c;
  const bool valid = row < a.nrows;
  const long long nx = 2 * L;

  if (blockIdx.x == 0) {                        // clear this field's accumulators for later passes
    for (int s = 0; s < a.zero_spans; ++s) {
      uint32_t* dst = a.zero[s].ptr + (long long)b * a.zero[s].per_field;
      for (int i = tid; i < a.zero[s].per_field; i += T) dst[i] = 0u;
    }
  }

  // ---- fill LDS with the C real rows (as floats)
  const long long v0 = row0 * nx;
  const long long rows_here = (a.nrows - row0) < C ? (a.nrows - row0) : C;
  const long long v1 = v0 + rows_here * nx;
  if constexpr (SRC == SRC_NOISE) {
    const uint64_t seed = a.seeds[b];
    const long long m0 = v0 >> 2, m1 = (v1 + 3) >> 2;
    for (long long m = m0 + tid; m < m1; m += T) {
      float z[4];
      noise4((uint64_t)m, seed, z);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const long long v = 4 * m + q;
        if (v >= v0 && v < v1) ldsf[v - v0] = z[q];
      }
    }
  } else {
    const long long base = (long long)b * a.N + v0;
    for (long long i = tid; i < C * nx; i += T) {
      float x = 0.0f;
      if (i < v1 - v0) {
        if constexpr (SRC == SRC_F32) x = reinterpret_cast<const float*>(a.src)[base + i];
        else x = (float)reinterpret_cast<const int8_t*>(a.src)[base + i];
      }
      ldsf[i] = x;
    }
  }
  __syncthreads();

  float2 v[E];
  float2* lrow = lds + c * L;
#pragma unroll
  for (int s = 0; s < E; ++s) v[s] = lrow[slot_index<L, R1, P>(s, p)];
  fft_run<L, P, E, false>(Rad{}, v, lrow, p, a.tw);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < E; ++s) lrow[slot_index<L, RL, P>(s, p)] = v[s];
  __syncthreads();
  float2* out = a.spec + (long long)b * a.Nh + row * (L + 1);
  r2c_twist_store<L, P, E>(lrow, a.tw2, out, p, valid);
}

// =============================================================================================
// cols: C2C along a strided axis, forward or inverse, in place.  grid (ceil(ncol / C), B).
// element e of column g lives at (g / inner) * (L * inner) + (g % inner) + e * inner.
// =============================================================================================
template <int L, bool INV>
__global__ void __launch_bounds__(ColTile<L>::T) k_cols(ColsArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = ColTile<L>::C;
  using Rad = typename Plan<L>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const int c = tid % C, p = tid / C;
  const int b = blockIdx.y;
  const long long g = (long long)blockIdx.x * C + c;
  const bool valid = g < a.ncol;
  const long long inner = a.inner;
  float2* base = a.spec + (long long)b * a.Nh + (g / inner) * (L * inner) + (g % inner);
  float2 v[E];
#pragma unroll
  for (int s = 0; s < E; ++s)
    v[s] = valid ? base[(long long)slot_index<L, R1, P>(s, p) * inner] : make_float2(0.f, 0.f);
  fft_run<L, P, E, INV>(Rad{}, v, lds + c * L, p, a.tw);
  if (valid) {
#pragma unroll
    for (int s = 0; s < E; ++s) base[(long long)slot_index<L, RL, P>(s, p) * inner] = v[s];
  }
}

// ---------------------------------------------------------------------------------------------
// shared pieces of the axis-0 passes: the column's fixed wavenumber components and bin pieces
// ---------------------------------------------------------------------------------------------
struct ColCoord {
  int mx;            // half-spectrum x index (>= 0)
  int my;            // y index (3D only)
  float kx_c;        // canonical kappa_x (-1 at the x Nyquist index)
  float ky;          // canonical kappa_y (3D only)
  bool nyq_x, nyq_y; // x / y component on a Nyquist index (3D y)
  long long qx, qy;  // bin integers (3D: qy is the y component)
  long long sfix;    // sum of the fixed q_i^2
  float wm;          // multiplicity 1 or 2
};

__device__ __forceinline__ ColCoord col_coord(const Axis0Geom& gm, long long g) {
  ColCoord cc;
  if (gm.ndim == 2) {
    cc.mx = (int)g;
    cc.my = 0;
  } else {
    cc.mx = (int)(g % gm.nxh);
    cc.my = (int)(g / gm.nxh);
  }
  cc.nyq_x = (2 * cc.mx == gm.nx);
  cc.kx_c = cc.nyq_x ? -1.0f : (float)(2.0 * cc.mx / gm.nx);
  cc.wm = (cc.mx == 0 || cc.nyq_x) ? 1.0f : 2.0f;
  cc.qx = (long long)cc.mx * gm.dfac_x;
  if (gm.ndim == 3) {
    const int mt = cc.my < gm.ny / 2 ? cc.my : cc.my - gm.ny;
    cc.nyq_y = (2 * cc.my == gm.ny);
    cc.ky = (float)(2.0 * mt / gm.ny);
    cc.qy = (long long)mt * gm.dfac_y;
    cc.sfix = cc.qx * cc.qx + cc.qy * cc.qy;
  } else {
    cc.nyq_y = false;
    cc.ky = 0.0f;
    cc.qy = 0;
    cc.sfix = cc.qx * cc.qx;
  }
  return cc;
}

// symmetrised amplitude at axis-0 index e of column cc; also returns ln chi (unsymmetrised)
__device__ __forceinline__ float amp_sym(const FiltDev& f, const Axis0Geom& gm, const ColCoord& cc, int e,
                                         float& lnc) {
  const int mt = e < gm.n0 / 2 ? e : e - gm.n0;
  const float k0c = (float)(2.0 * mt / gm.n0);   // canonical kappa along axis 0 (-1 at Nyquist)
  const bool nyq0 = (2 * e == gm.n0);
  float kx = cc.kx_c, ky, kz;
  bool ny_y;
  if (gm.ndim == 2) { ky = k0c; kz = 0.0f; ny_y = nyq0; }
  else { ky = cc.ky; kz = k0c; ny_y = cc.nyq_y; }
  lnc = ln_chi(f, kx, ky, kz);
  float H = __expf(0.5f * lnc);
  if (f.rotated && (cc.nyq_x || ny_y)) {
    // partner -m: by evenness, the canonical kappa with its Nyquist components negated
    const float kx2 = cc.nyq_x ? -kx : kx, ky2 = ny_y ? -ky : ky;
    const float l2 = ln_chi(f, kx2, ky2, kz);
    H = 0.5f * (H + __expf(0.5f * l2));
  }
  return H;
}

__device__ __forceinline__ int mode_bin(const BinDev& bd, const Axis0Geom& gm, const ColCoord& cc, int e) {
  const int mt = e < gm.n0 / 2 ? e : e - gm.n0;
  const long long q0 = (long long)mt * gm.dfac_0;
  const long long s = cc.sfix + q0 * q0;
  // 2D: angle of (q_x, q_y = q0); 3D: radial only
  return bin_index(bd, s, cc.qx, gm.ndim == 2 ? q0 : 0);
}

__device__ __forceinline__ void hist_clear(double* hs, unsigned* hc, int nb, int tid, int T) {
  for (int i = tid; i < nb; i += T) { hs[i] = 0.0; hc[i] = 0u; }
}

__device__ __forceinline__ void hist_flush(const double* hs, const unsigned* hc, int nb, double scale,
                                           double* out_sum, uint64_t* out_cnt, int tid, int T) {
  for (int i = tid; i < nb; i += T) {
    const unsigned n = hc[i];
    if (n) {
      atomicAdd(out_sum + i, hs[i] * scale);
      if (out_cnt) atomicAdd((unsigned long long*)(out_cnt + i), (unsigned long long)n);
    }
  }
}

// =============================================================================================
// cols_filter: axis-0 forward FFT -> x H_sym -> stats + continuous bins -> inverse FFT.
// =============================================================================================
template <int L>
__global__ void __launch_bounds__(ColTile<L>::T) k_cols_filter(FilterArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = ColTile<L>::C, T = ColTile<L>::T;
  using Rad = typename Plan<L>::fwd;
  using RadI = Reverse<Rad>;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  __shared__ double red_d[T / 64];
  __shared__ float red_f[T / 64];
  __shared__ double red_d0[T / 64];
  __shared__ int is_last;
  const int tid = threadIdx.x;
  const int c = tid % C, p = tid / C;
  const int b = blockIdx.y;
  const long long g = (long long)blockIdx.x * C + c;
  const bool valid = g < a.gm.ncol;
  const long long ncol = a.gm.ncol;
  float2* base = a.spec + (long long)b * a.Nh + g;
  float2 v[E];
#pragma unroll
  for (int s = 0; s < E; ++s)
    v[s] = valid ? base[(long long)slot_index<L, R1, P>(s, p) * ncol] : make_float2(0.f, 0.f);
  fft_run<L, P, E, false>(Rad{}, v, lds + c * L, p, a.tw);

  // ---- filter, Parseval statistics, continuous-spectrum histogram
  const bool do_bins = a.cont_sum != nullptr;
  double* hs = reinterpret_cast<double*>(lds);
  unsigned* hc = reinterpret_cast<unsigned*>(hs + a.nb);
  __syncthreads();                                // LDS exchange buffer is free from here
  if (do_bins) hist_clear(hs, hc, a.nb, tid, T);
  __syncthreads();
  const ColCoord cc = col_coord(a.gm, valid ? g : 0);
  double gsum = 0.0;
  float lmax = -1.0e30f;
  double f0 = 0.0;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int e = slot_index<L, RL, P>(s, p);
    float lnc;
    const float H = amp_sym(a.filt, a.gm, cc, e, lnc);
    const float2 F = cscale(v[s], H);
    v[s] = F;
    if (valid) {
      const double m2 = (double)F.x * (double)F.x + (double)F.y * (double)F.y;
      gsum += (double)cc.wm * m2;
      lmax = fmaxf(lmax, lnc);
      if (g == 0 && e == 0) f0 = (double)F.x;
      if (do_bins) {
        const int bi = mode_bin(a.bd, a.gm, cc, e);
        atomicAdd(hs + bi, (double)cc.wm * m2);
        atomicAdd(hc + bi, (unsigned)cc.wm);
      }
    }
  }
  // block reduction of the statistics (F(0) lives in workgroup 0 only)
  gsum = wave_sum(gsum);
  lmax = wave_max(lmax);
  f0 = wave_sum(f0);
  if ((tid & 63) == 0) { red_d[tid >> 6] = gsum; red_f[tid >> 6] = lmax; red_d0[tid >> 6] = f0; }
  __syncthreads();
  if (tid == 0) {
    double gs = 0.0, fz = 0.0;
    float lm = -1.0e30f;
    for (int w = 0; w < T / 64; ++w) { gs += red_d[w]; fz += red_d0[w]; lm = fmaxf(lm, red_f[w]); }
    double* part = a.partials + ((long long)b * gridDim.x + blockIdx.x) * 4;
    part[0] = gs;
    part[1] = fz;
    part[2] = (double)lm;
    part[3] = 0.0;
  }
  if (do_bins) {
    __syncthreads();
    hist_flush(hs, hc, a.nb, 1.0, a.cont_sum + (long long)b * a.nb,
               a.cont_cnt ? a.cont_cnt + (long long)b * a.nb : nullptr, tid, T);
  }
  // ---- last workgroup of this field: finalise mu, var, scale; rescale the continuous bins
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    const unsigned prev = atomicAdd(a.counters + b, 1u);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (is_last) {
    __threadfence();
    if (tid == 0) {
      double G = 0.0, F0 = 0.0;
      double lm = -1.0e30;
      const double* part = a.partials + (long long)b * gridDim.x * 4;
      for (unsigned w = 0; w < gridDim.x; ++w) {
        G += __hip_atomic_load(part + 4 * w + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        F0 += __hip_atomic_load(part + 4 * w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        lm = fmax(lm, __hip_atomic_load(part + 4 * w + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      }
      const double N = (double)a.N;
      const double mu = F0 / N;
      const double var = G / (N * N) - mu * mu;
      const bool degenerate = !(lm >= -80.0) || !(var > 0.0);
      const double sd = degenerate ? 1.0 : sqrt(var);
      double* fs = a.fstats + (long long)b * 8;
      fs[0] = mu;
      fs[1] = var;
      fs[2] = lm;
      fs[3] = degenerate ? 1.0 : 0.0;
      fs[4] = degenerate ? 0.0 : a.sigma_f / (N * sd);         // scale on the unnormalised inverse
      fs[5] = degenerate ? 0.0 : -a.sigma_f * mu / sd;          // offset
      fs[6] = degenerate ? 0.0 : a.sigma_f * a.sigma_f / (N * var);  // continuous-spectrum factor
      fs[7] = G;
      if (a.stats) {
        double* st = a.stats + (long long)b * 4;
        st[0] = mu; st[1] = var; st[2] = lm; st[3] = fs[3];
      }
      red_d[0] = fs[6];
      __hip_atomic_store(a.counters + b, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (do_bins) {
      const double fac = red_d[0];
      double* cs = a.cont_sum + (long long)b * a.nb;
      for (int i = tid; i < a.nb; i += T) {
        const double x = __hip_atomic_load(cs + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(cs + i, x * fac, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }

  // ---- inverse transform along axis 0 (first radix = last forward radix: no exchange needed)
  fft_run<L, P, E, true>(RadI{}, v, lds + c * L, p, a.tw);
  if (valid) {
#pragma unroll
    for (int s = 0; s < E; ++s) base[(long long)slot_index<L, R1, P>(s, p) * ncol] = v[s];
  }
}

// =============================================================================================
// cols_bin: axis-0 forward FFT and binned periodogram |X|^2 / N; nothing written back.
// =============================================================================================
template <int L>
__global__ void __launch_bounds__(ColTile<L>::T) k_cols_bin(BinArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = ColTile<L>::C, T = ColTile<L>::T;
  using Rad = typename Plan<L>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const int c = tid % C, p = tid / C;
  const int b = blockIdx.y;
  const long long g = (long long)blockIdx.x * C + c;
  const bool valid = g < a.gm.ncol;
  const long long ncol = a.gm.ncol;
  const float2* base = a.spec + (long long)b * a.Nh + g;
  float2 v[E];
#pragma unroll
  for (int s = 0; s < E; ++s)
    v[s] = valid ? base[(long long)slot_index<L, R1, P>(s, p) * ncol] : make_float2(0.f, 0.f);
  fft_run<L, P, E, false>(Rad{}, v, lds + c * L, p, a.tw);
  double* hs = reinterpret_cast<double*>(lds);
  unsigned* hc = reinterpret_cast<unsigned*>(hs + a.nb);
  __syncthreads();
  hist_clear(hs, hc, a.nb, tid, T);
  __syncthreads();
  if (valid) {
    const ColCoord cc = col_coord(a.gm, g);
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int e = slot_index<L, RL, P>(s, p);
      const double m2 = (double)v[s].x * (double)v[s].x + (double)v[s].y * (double)v[s].y;
      const int bi = mode_bin(a.bd, a.gm, cc, e);
      atomicAdd(hs + bi, (double)cc.wm * m2);
      atomicAdd(hc + bi, (unsigned)cc.wm);
    }
  }
  __syncthreads();
  hist_flush(hs, hc, a.nb, 1.0 / (double)a.N, a.sum + (long long)b * a.nb,
             a.cnt ? a.cnt + (long long)b * a.nb : nullptr, tid, T);
}

// =============================================================================================
// rows_c2r: C2R along x -> normalise -> field, sign map, counts -> R2C of the +-1 row.
// =============================================================================================
template <int L, bool THRESH>
__global__ void __launch_bounds__(RowTile<L>::T) k_rows_c2r(RowsZArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = RowTile<L>::C, T = RowTile<L>::T;
  using Rad = typename Plan<L>::fwd;
  using RadF = Reverse<Rad>;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  constexpr int LS = L + 1;
  extern __shared__ float2 lds[];
  __shared__ unsigned red_u[2][T / 64 > 0 ? T / 64 : 1];
  const int tid = threadIdx.x;
  const int c = tid / P, p = tid % P;
  const int b = blockIdx.y;
  const long long row = (long long)blockIdx.x * C + c;
  const bool valid = row < a.nrows;
  float2* lrow = lds + c * LS;
  float2* srow = a.spec + (long long)b * a.Nh + row * LS;

  // ---- load the half row X[0..L] into LDS
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int k = p + P * i;
    float2 x = valid ? srow[k] : make_float2(0.f, 0.f);
    if (k == 0) x.y = 0.0f;
    lrow[k] = x;
  }
  if (p == 0) lrow[L] = valid ? make_float2(srow[L].x, 0.0f) : make_float2(0.f, 0.f);
  __syncthreads();
  // ---- pre-twist: Z[k] = (X[k] + X*[L-k]) + i e^{+2 pi i k / 2L} (X[k] - X*[L-k])
  float2 v[E];
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int k = slot_index<L, R1, P>(s, p);
    const float2 xk = lrow[k], xc = cconj(lrow[L - k]);
    v[s] = cadd(cadd(xk, xc), mul_mi<true>(cmul(cconj(a.tw2[k]), csub(xk, xc))));
  }
  fft_run<L, P, E, true>(Rad{}, v, lrow, p, a.tw);

  // ---- normalise (Eq. (15)), write the field, threshold
  const double* fs = a.fstats + (long long)b * 8;
  const float scale = (float)fs[4], offset = (float)fs[5];
  const float tol = a.near_tol;
  unsigned npos = 0, nnear = 0;
  const long long rbase = (long long)b * a.N + row * (2LL * L);
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int n = slot_index<L, RL, P>(s, p);
    const float x0 = fmaf(v[s].x, scale, offset);
    const float x1 = fmaf(v[s].y, scale, offset);
    if (valid && a.field) *reinterpret_cast<float2*>(a.field + rbase + 2 * n) = make_float2(x0, x1);
    if constexpr (THRESH) {
      const float t0 = x0 >= 0.0f ? 1.0f : -1.0f, t1 = x1 >= 0.0f ? 1.0f : -1.0f;
      if (valid) {
        npos += (x0 >= 0.0f) + (x1 >= 0.0f);
        nnear += (fabsf(x0) < tol) + (fabsf(x1) < tol);
        if (a.pm1) {
          char2 tt;
          tt.x = (signed char)t0;
          tt.y = (signed char)t1;
          *reinterpret_cast<char2*>(a.pm1 + rbase + 2 * n) = tt;
        }
      }
      v[s] = make_float2(t0, t1);
    }
  }
  if constexpr (THRESH) {
    // counts
    npos = wave_usum(npos);
    nnear = wave_usum(nnear);
    if ((tid & 63) == 0) { red_u[0][tid >> 6] = npos; red_u[1][tid >> 6] = nnear; }
    // forward transform of the packed +-1 row (its first radix is the inverse's last)
    fft_run<L, P, E, false>(RadF{}, v, lrow, p, a.tw);
    __syncthreads();
    constexpr int RLF = RadInfo<RadF>::last;
#pragma unroll
    for (int s = 0; s < E; ++s) lrow[slot_index<L, RLF, P>(s, p)] = v[s];
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

// =============================================================================================
// threshold: standalone sign map with counts.  grid-stride over B * N values.
// =============================================================================================
__global__ void __launch_bounds__(256) k_threshold(ThreshArgs a) {
  __shared__ unsigned red[2][4];
  const int b = blockIdx.y;
  const float* f = a.field + (long long)b * a.N;
  int8_t* t = a.out + (long long)b * a.N;
  unsigned np = 0, nn = 0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < a.N; i += (long long)gridDim.x * 256) {
    const float x = f[i];
    const bool pos = x >= 0.0f;
    t[i] = pos ? (int8_t)1 : (int8_t)-1;
    np += pos;
    nn += fabsf(x) < a.near_tol;
  }
  np = wave_usum(np);
  nn = wave_usum(nn);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = np; red[1][threadIdx.x >> 6] = nn; }
  __syncthreads();
  if (threadIdx.x == 0 && a.counts) {
    atomicAdd((unsigned long long*)(a.counts + 2 * b + 0),
              (unsigned long long)(red[0][0] + red[0][1] + red[0][2] + red[0][3]));
    atomicAdd((unsigned long long*)(a.counts + 2 * b + 1),
              (unsigned long long)(red[1][0] + red[1][1] + red[1][2] + red[1][3]));
  }
}

__global__ void k_zero_u64(uint64_t* p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void k_debug_philox(uint64_t seed, uint64_t first, uint64_t count, uint32_t* words, float* normals) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const U4 w = philox4x32_10(first + i, seed);
  if (words) {
    words[4 * i + 0] = w.x; words[4 * i + 1] = w.y; words[4 * i + 2] = w.z; words[4 * i + 3] = w.w;
  }
  if (normals) {
    float z0, z1, z2, z3;
    box_muller(w.x, w.y, z0, z1);
    box_muller(w.z, w.w, z2, z3);
    normals[4 * i + 0] = z0; normals[4 * i + 1] = z1; normals[4 * i + 2] = z2; normals[4 * i + 3] = z3;
  }
}

// =============================================================================================
// launchers: dispatch the runtime length to the compile-time instantiation
// =============================================================================================
#define HU_ROW_LENGTHS(X) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(1024)
#define HU_COL_LENGTHS(X) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(2048)

static inline int ceil_div_ll(long long a, long long b) { return (int)((a + b - 1) / b); }

template <int L, int SRC>
static hipError_t launch_rows_r2c_L(const RowsArgs& a, int batch, hipStream_t st) {
  constexpr int C = RowTile<L>::C, T = RowTile<L>::T;
  dim3 grid(ceil_div_ll(a.nrows, C), batch);
  const size_t lds = (size_t)C * L * sizeof(float2);
  hipLaunchKernelGGL((k_rows_r2c<L, SRC>), grid, dim3(T), lds, st, a);
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

template <int L, bool INV>
static hipError_t launch_cols_L(const ColsArgs& a, int batch, hipStream_t st) {
  constexpr int C = ColTile<L>::C, T = ColTile<L>::T;
  dim3 grid(ceil_div_ll(a.ncol, C), batch);
  hipLaunchKernelGGL((k_cols<L, INV>), grid, dim3(T), (size_t)C * L * sizeof(float2), st, a);
  return hipGetLastError();
}

hipError_t launch_cols(int L, bool inv, const ColsArgs& a, int batch, hipStream_t st) {
  switch (L) {
#define X(LL) \
  case LL: return inv ? launch_cols_L<LL, true>(a, batch, st) : launch_cols_L<LL, false>(a, batch, st);
    HU_COL_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

template <int L>
static size_t col_lds_bytes(int nb) {
  const size_t fft = (size_t)ColTile<L>::C * L * sizeof(float2);
  const size_t hist = (size_t)nb * (sizeof(double) + sizeof(unsigned));
  return fft > hist ? fft : hist;
}

int col_tiles(int L, long long ncol) {
  switch (L) {
#define X(LL) case LL: return ceil_div_ll(ncol, ColTile<LL>::C);
    HU_COL_LENGTHS(X)
#undef X
    default: return -1;
  }
}

template <int L>
static hipError_t launch_cols_filter_L(const FilterArgs& a, int batch, hipStream_t st) {
  constexpr int C = ColTile<L>::C, T = ColTile<L>::T;
  dim3 grid(ceil_div_ll(a.gm.ncol, C), batch);
  hipLaunchKernelGGL((k_cols_filter<L>), grid, dim3(T), col_lds_bytes<L>(a.cont_sum ? a.nb : 0), st, a);
  return hipGetLastError();
}

hipError_t launch_cols_filter(int L, const FilterArgs& a, int batch, hipStream_t st) {
  switch (L) {
#define X(LL) case LL: return launch_cols_filter_L<LL>(a, batch, st);
    HU_COL_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

template <int L>
static hipError_t launch_cols_bin_L(const BinArgs& a, int batch, hipStream_t st) {
  constexpr int C = ColTile<L>::C, T = ColTile<L>::T;
  dim3 grid(ceil_div_ll(a.gm.ncol, C), batch);
  hipLaunchKernelGGL((k_cols_bin<L>), grid, dim3(T), col_lds_bytes<L>(a.nb), st, a);
  return hipGetLastError();
}

hipError_t launch_cols_bin(int L, const BinArgs& a, int batch, hipStream_t st) {
  switch (L) {
#define X(LL) case LL: return launch_cols_bin_L<LL>(a, batch, st);
    HU_COL_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

template <int L, bool THRESH>
static hipError_t launch_rows_c2r_L(const RowsZArgs& a, int batch, hipStream_t st) {
  constexpr int C = RowTile<L>::C, T = RowTile<L>::T;
  dim3 grid(ceil_div_ll(a.nrows, C), batch);
  hipLaunchKernelGGL((k_rows_c2r<L, THRESH>), grid, dim3(T), (size_t)C * (L + 1) * sizeof(float2), st, a);
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

hipError_t launch_threshold(const ThreshArgs& a, int batch, hipStream_t st) {
  long long blocks = (a.N + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_threshold, dim3((unsigned)blocks, batch), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_zero_u64(uint64_t* p, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_debug_philox(uint64_t seed, uint64_t first, uint64_t count, uint32_t* words, float* normals,
                               hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_debug_philox, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, seed, first, count,
                     words, normals);
  return hipGetLastError();
}

}  // namespace hu
