// The fused axis-0 pass of the generator: forward FFT along the slowest axis, multiplication by
// the symmetrised amplitude H_sym = sqrt(chi) (Eq. (8) with Eqs. (12)-(13)), the FP64 Parseval
// statistics of Eq. (15), the continuous-field spectrum bins, and the inverse FFT along the same
// axis -- one read and one write of the half spectrum.  Each workgroup leaves its partial sums
// and its tile's bin partials; k_finalize turns the sums into (mu, var, scale, offset) in a fixed
// order, and k_spec_final assembles the bins of the normalised field.
#include "hu_common.hpp"

namespace hu {

// One tile of C columns of one field per workgroup.
template <int L, int NDIM, int V, bool GEN, int RV, bool SPLIT>
__global__ void __launch_bounds__((ColTile<L, V>::T)) k_cols_filter(FilterArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = ColTile<L, V>::C, T = ColTile<L, V>::T;
  constexpr int LP = ColTile<L, V>::LP;
  using Rad = typename Plan<L, RV>::fwd;
  using RadI = Reverse<Rad>;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  __shared__ double red_d[T / 64], red_d0[T / 64];
  __shared__ float red_f[T / 64];
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
  fft_run<L, P, E, false, false, RV>(Rad{}, v, col_region<L, V, SPLIT>(lds, c), p, a.tw);

  // ---- filter and per-thread statistics
  const bool do_bins = a.parts != nullptr;
  const FiltDev filt = a.io ? a.io[b].filt : a.filt;
  const ColCoord cc = col_coord(a.gm, valid ? g : 0);
  Col3 c3a{}, c3b{};
  if constexpr (NDIM == 3) {                       // the column's x / y terms of the filter
    c3a = col3(filt, cc.kx_c, cc.ky);
    c3b = (filt.rotated && (cc.nyq_x || cc.nyq_y)) ? col3(filt, cc.nyq_x ? -cc.kx_c : cc.kx_c, cc.nyq_y ? -cc.ky : cc.ky)
                                                   : c3a;
  }
  double gsum = 0.0, f0 = 0.0;
  float lmax = filt.lnoffset;             // the lattice maximum of ln(chi_rel + offset) is at least ln offset
  // the exchange buffer is free once every thread has its transform in registers: the power
  // values of the continuous spectrum go to LDS as they are computed
  float* pw = reinterpret_cast<float*>(lds);
  int* hx = reinterpret_cast<int*>(reinterpret_cast<char*>(lds) + a.hx_off);
  unsigned long long* hq = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(lds) + a.hq_off);
  if (do_bins) {
    for (int j = tid; j < a.tb.nloc_max; j += T) {
      hx[j] = HX_EMPTY;
      hq[j] = 0ull;
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int e = slot_index<L, RL, P>(s, p);
    float lnc;
    const float H = NDIM == 3 ? amp_sym3<GEN>(filt, a.gm, cc, c3a, c3b, e, lnc) : amp_sym<NDIM, GEN>(filt, a.gm, cc, e, lnc);
    const float2 F = cscale(v[s], H);
    v[s] = F;
    const float m2 = cc.wm * (F.x * F.x + F.y * F.y);
    if (do_bins) pw[c * LP + pw_index(e)] = valid ? m2 : 0.0f;
    if (valid) {
      gsum += (double)m2;
      lmax = fmaxf(lmax, lnc);
      if (g == 0 && e == 0) f0 = (double)F.x;
    }
  }
  // ---- workgroup statistics -> partials[b][tile] (reduced by k_finalize after this kernel)
  gsum = wave_sum(gsum);
  lmax = wave_max(lmax);
  f0 = wave_sum(f0);
  if ((tid & 63) == 0) { red_d[tid >> 6] = gsum; red_f[tid >> 6] = lmax; red_d0[tid >> 6] = f0; }
  __syncthreads();
  if (tid == 0) {
    double gs = 0.0, fz = 0.0;
    float lm = -1.0e30f;
    for (int w = 0; w < T / 64; ++w) { gs += red_d[w]; fz += red_d0[w]; lm = fmaxf(lm, red_f[w]); }
    double* part = a.partials + ((long long)b * a.sc.ntiles + tile) * 4;
    part[0] = gs;
    part[1] = fz;
    part[2] = (double)lm;
    part[3] = 0.0;
  }
  // ---- continuous-spectrum bins of the tile -> parts[b][toff[tile] ..] (deterministic)
  if (do_bins) {
    tile_bins<L, E, C, LP, T>(pw, hx, hq, a.tb, (int)tile, a.gm.ncol, a.parts + (long long)b * a.tb.M, tid);
  }

  // ---- inverse transform along axis 0 (first radix = last forward radix: no exchange needed)
  fft_run<L, P, E, true, false, RV>(RadI{}, v, col_region<L, V, SPLIT>(lds, c), p, a.tw);
  __builtin_amdgcn_s_setprio(2);                 // the stores out ahead of other workgroups' transforms
  if (valid) col_store<L, R1, P, E>(v, io);
  __builtin_amdgcn_s_setprio(0);
}

// ---------------------------------------------------------------------------------------------
// finalize: one workgroup per field turns the filter pass's partials into mu, var and the
// normalisation constants (Eq. (15) via Parseval) with a fixed-order reduction, and the factor
// that turns the continuous-field bins into the spectrum of the normalised field.
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_finalize(FinalizeArgs a) {
  __shared__ double sg[256], sf[256];
  __shared__ float sm[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  const double* part = a.partials + (long long)b * a.ntiles * 4;
  const double sigma_f = a.io ? a.io[b].sigma_f : a.sigma_f;
  double* stats_out = a.io ? a.io[b].stats : field_ptr(a.stats, 4, b);
  double G = 0.0, F0 = 0.0;
  float lm = -1.0e30f;
#pragma unroll 4
  for (int w = tid; w < a.ntiles; w += 256) {
    G += part[4 * w + 0];
    F0 += part[4 * w + 1];
    lm = fmaxf(lm, (float)part[4 * w + 2]);
  }
  sg[tid] = G;
  sf[tid] = F0;
  sm[tid] = lm;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      sg[tid] += sg[tid + o];
      sf[tid] += sf[tid + o];
      sm[tid] = fmaxf(sm[tid], sm[tid + o]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double N = (double)a.N;
    const double Gt = sg[0];
    const double mu = sf[0] / N;                  // Re F(0) / N
    const double var = Gt / (N * N) - mu * mu;    // Parseval, population variance
    const double lmx = (double)sm[0];
    const bool degenerate = !(lmx >= -80.0) || !(var > 0.0);
    const double sd = degenerate ? 1.0 : sqrt(var);
    double* fs = a.fstats + (long long)b * 8;
    fs[0] = mu;
    fs[1] = var;
    fs[2] = lmx;
    fs[3] = degenerate ? 1.0 : 0.0;
    fs[4] = degenerate ? 0.0 : sigma_f / (N * sd);             // scale of the unnormalised inverse
    fs[5] = degenerate ? 0.0 : -sigma_f * mu / sd;              // offset
    fs[6] = degenerate ? 0.0 : sigma_f * sigma_f / (N * var);   // continuous-spectrum factor
    fs[7] = Gt;
    if (stats_out) {
      stats_out[0] = mu; stats_out[1] = var; stats_out[2] = lmx; stats_out[3] = fs[3];
    }
  }
}

hipError_t launch_finalize(const FinalizeArgs& a, int batch, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(batch), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int L, int V, int RV, bool SPLIT>
static hipError_t launch_cols_filter_L(FilterArgs a, hipStream_t st) {
  constexpr int T = ColTile<L, V>::T;
  size_t lds = col_xchg_bytes<L, V, SPLIT>();
  if (a.parts) {
    a.hx_off = (int)col_bin_base<L, V, SPLIT>();
    a.hq_off = a.hx_off + (a.tb.nloc_max * 4 + 15) / 16 * 16;
    lds = (size_t)a.hq_off + (size_t)a.tb.nloc_max * 8;
  }
  // the tabulated-form and FP64 branches only in the instantiation launched when a field may use one
  const dim3 grid(sched_blocks(a.sc));
  if (a.gm.ndim == 2) {
    if (a.any_gen) hipLaunchKernelGGL((k_cols_filter<L, 2, V, true, RV, SPLIT>), grid, dim3(T), lds, st, a);
    else hipLaunchKernelGGL((k_cols_filter<L, 2, V, false, RV, SPLIT>), grid, dim3(T), lds, st, a);
  } else {
    if (a.any_gen) hipLaunchKernelGGL((k_cols_filter<L, 3, V, true, RV, SPLIT>), grid, dim3(T), lds, st, a);
    else hipLaunchKernelGGL((k_cols_filter<L, 3, V, false, RV, SPLIT>), grid, dim3(T), lds, st, a);
  }
  return hipGetLastError();
}

int col_width(int L, int variant) {
  switch (L) {
#define X(LL) case LL: return variant ? ColTile<LL, 1>::C : ColTile<LL, 0>::C;
    HU_COL_LENGTHS(X)
#undef X
    default: return 0;
  }
}

hipError_t launch_cols_filter(int L, int variant, const FilterArgs& a, hipStream_t st, int radix, int split) {
  switch (L) {
#define X(LL)                                                                                             \
  case LL:                                                                                                \
    return with_choices3<LL>(variant, radix, split, [&](auto v, auto r, auto s) {                         \
      return launch_cols_filter_L<LL, decltype(v)::value, decltype(r)::value, decltype(s)::value>(a, st); \
    });
    HU_COL_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hu
