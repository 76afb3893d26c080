// Spectrum binning passes and small utility kernels.
//
//   cols_bin    forward FFT along axis 0 and the per-tile bin partials of w |X|^2 of the +-1
//               field (or of any real input), read only;
//   spec_final  the per-field binned spectra from the tile partials, and the sign counts;
//   threshold   the standalone sign map with counts;
//   debug_philox  raw Philox words and normals for the parity tests.
#include "hu_common.hpp"

namespace hu {

// Persistent (the default in 3D) over the items (tile, field), tile-major, taken from the work counter in chunks: the
// forward transform of a tile's columns, the per-mode values w |X|^2 into LDS, then (while the next
// item's columns are already being loaded into the transform's registers) the tile's deterministic
// bin partials.
template <int L, int V, int RV, bool SPLIT>
__global__ void __launch_bounds__((ColTile<L, V>::T)) k_cols_bin(BinArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = ColTile<L, V>::C, T = ColTile<L, V>::T;
  constexpr int LP = ColTile<L, V>::LP;
  using Rad = typename Plan<L, RV>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  __shared__ int grab[2];
  float* pw = reinterpret_cast<float*>(lds);
  int* hx = reinterpret_cast<int*>(reinterpret_cast<char*>(lds) + a.hx_off);
  unsigned long long* hq = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(lds) + a.hq_off);
  const int tid = threadIdx.x;
  const int c = tid % C, p = tid / C;
  for (int j = tid; j < a.tb.nloc_max; j += T) {
    hx[j] = HX_EMPTY;
    hq[j] = 0ull;
  }
  int last = 0;
  float2 v[E];
  for (;;) {
    if (tid == 0) {
      int ch = (a.q.nitems - last) / (2 * (int)gridDim.x);
      ch = ch < 1 ? 1 : (ch > a.q.chunk_max ? a.q.chunk_max : ch);
      const int s0 = (int)atomicAdd(a.q.counter, (unsigned)ch);
      grab[0] = s0;
      grab[1] = s0 + ch < a.q.nitems ? s0 + ch : a.q.nitems;
    }
    __syncthreads();
    const int i0 = grab[0], i1 = grab[1];
    if (i0 >= a.q.nitems) break;
    last = i0;
    {
      const int tile = i0 / a.batch, b = i0 - tile * a.batch;
      col_load<L, R1, P, E>(v, col_io<L>(a.spec + (long long)b * a.Nh, a.Nh, a.gm.inner0, tile * C + c, p));
    }
    for (int it = i0; it < i1; ++it) {
      const int tile = it / a.batch, b = it - tile * a.batch;
      const int g = tile * C + c;
      const bool valid = g < a.gm.ncol;
      fft_run<L, P, E, false, false, RV>(Rad{}, v, col_region<L, V, SPLIT>(lds, c), p, a.tw);
      const float wm = (valid && col_coord(a.gm, g).wm > 1.5f) ? 2.0f : 1.0f;
      __syncthreads();                              // the exchange buffer is free from here
#pragma unroll
      for (int s = 0; s < E; ++s)
        pw[c * LP + pw_index(slot_index<L, RL, P>(s, p))] = valid ? wm * (v[s].x * v[s].x + v[s].y * v[s].y) : 0.0f;
      if (it + 1 < i1) {                            // the next item's columns, in flight during the binning
        const int tn = (it + 1) / a.batch, bn = it + 1 - tn * a.batch;
        col_load<L, R1, P, E>(v, col_io<L>(a.spec + (long long)bn * a.Nh, a.Nh, a.gm.inner0, tn * C + c, p));
      }
      __syncthreads();
      tile_bins<L, E, C, LP, T>(pw, hx, hq, a.tb, tile, a.gm.ncol, a.parts + (long long)b * a.tb.M, tid);
    }
  }
}

// One item per workgroup (the default in 2D, where the schedule's XCD mapping puts the fields of a
// tile on one XCD, which then reads the tile's slice of the bin table once).
template <int L, int V, int RV, bool SPLIT>
__global__ void __launch_bounds__((ColTile<L, V>::T)) k_cols_bin_tile(BinArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = ColTile<L, V>::C, T = ColTile<L, V>::T;
  constexpr int LP = ColTile<L, V>::LP;
  using Rad = typename Plan<L, RV>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  int b;
  long long tile;
  if (!map_tile(a.sc, b, tile)) return;
  float* pw = reinterpret_cast<float*>(lds);
  int* hx = reinterpret_cast<int*>(reinterpret_cast<char*>(lds) + a.hx_off);
  unsigned long long* hq = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(lds) + a.hq_off);
  const int tid = threadIdx.x;
  const int c = tid % C, p = tid / C;
  const int g = (int)tile * C + c;
  const bool valid = g < a.gm.ncol;
  float2 v[E];
  col_load<L, R1, P, E>(v, col_io<L>(a.spec + (long long)b * a.Nh, a.Nh, a.gm.inner0, g, p));
  fft_run<L, P, E, false, false, RV>(Rad{}, v, col_region<L, V, SPLIT>(lds, c), p, a.tw);
  const float wm = (valid && col_coord(a.gm, g).wm > 1.5f) ? 2.0f : 1.0f;
  for (int j = tid; j < a.tb.nloc_max; j += T) {
    hx[j] = HX_EMPTY;
    hq[j] = 0ull;
  }
  __syncthreads();                                  // the exchange buffer is free from here
#pragma unroll
  for (int s = 0; s < E; ++s)
    pw[c * LP + pw_index(slot_index<L, RL, P>(s, p))] = valid ? wm * (v[s].x * v[s].x + v[s].y * v[s].y) : 0.0f;
  __syncthreads();
  tile_bins<L, E, C, LP, T>(pw, hx, hq, a.tb, (int)tile, a.gm.ncol, a.parts + (long long)b * a.tb.M, tid);
}

template <int L, int V, int RV, bool SPLIT>
static hipError_t launch_cols_bin_L(BinArgs a, hipStream_t st) {
  constexpr int T = ColTile<L, V>::T;
  if (a.q.nitems <= 0) return hipSuccess;
  a.hx_off = (int)col_bin_base<L, V, SPLIT>();
  a.hq_off = a.hx_off + (a.tb.nloc_max * 4 + 15) / 16 * 16;
  const size_t lds = (size_t)a.hq_off + (size_t)a.tb.nloc_max * 8;
  if (!a.persistent) {
    hipLaunchKernelGGL((k_cols_bin_tile<L, V, RV, SPLIT>), dim3(sched_blocks(a.sc)), dim3(T), lds, st, a);
    return hipGetLastError();
  }
  int slots = 0;
  const hipError_t e = resident_blocks(reinterpret_cast<const void*>(&k_cols_bin<L, V, RV, SPLIT>), T, lds, &slots);
  if (e != hipSuccess) return e;
  const unsigned grid = (unsigned)(slots < a.q.nitems ? slots : a.q.nitems);
  hipLaunchKernelGGL((k_cols_bin<L, V, RV, SPLIT>), dim3(grid), dim3(T), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_cols_bin(int L, int variant, const BinArgs& a, hipStream_t st, int radix, int split) {
  switch (L) {
#define X(LL)                                                                                             \
  case LL:                                                                                                \
    return with_choices3<LL>(variant, radix, split, [&](auto v, auto r, auto s) {                         \
      return launch_cols_bin_L<LL, decltype(v)::value, decltype(r)::value, decltype(s)::value>(a, st);    \
    });
    HU_COL_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------------------------
// Per-field spectra and sign counts.  The partials of a bin are stored together, in tile order, and
// added in a fixed order by a group of G lanes of one wave: lane l of the group adds partials
// l, l + G, l + 2G, ... (loads issued four at a time, added in order), then the group combines in a
// fixed butterfly.  G = 8 when bins hold few partials (2D: about ten), 64 when they hold hundreds
// (3D); the corner slot, which every tile touches, always gets a whole wave.  The result does not
// depend on the schedule of the passes that wrote the partials.  The continuous spectrum is scaled
// to the normalised field (factor from k_finalize), the +-1 spectrum by 1 / N.  The last workgroup
// of each field's row of the grid also totals the last row pass's per-tile sign counts.
// ---------------------------------------------------------------------------------------------
constexpr int SF_T = 256;

template <int G>
__device__ __forceinline__ double bin_total(const double* __restrict__ parts, const uint32_t* __restrict__ coff,
                                            int bin, int sub) {
  const unsigned j1 = coff[bin + 1];
  unsigned j = coff[bin] + sub;
  double s = 0.0;
  for (; j + 3 * G < j1; j += 4 * G) {
    const double x0 = parts[j], x1 = parts[j + G], x2 = parts[j + 2 * G], x3 = parts[j + 3 * G];
    s += x0;
    s += x1;
    s += x2;
    s += x3;
  }
  for (; j < j1; j += G) s += parts[j];
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  return s;
}

template <int G>
__device__ __forceinline__ void bin_out(const SpecFinalArgs& a, int b, int bin, int sub, double* cout_, double* pout) {
  if (cout_ && a.coff_c) {
    const double s = bin_total<G>(a.parts_c + (long long)b * a.M_c, a.coff_c, bin, sub);
    if (sub == 0) cout_[bin] = s * a.fstats[8LL * b + 6];
  }
  if (pout && a.coff_p) {
    const double s = bin_total<G>(a.parts_p + (long long)b * a.M_p, a.coff_p, bin, sub);
    if (sub == 0) pout[bin] = s * a.pscale;
  }
}

template <int G>
__global__ void __launch_bounds__(SF_T) k_spec_final(SpecFinalArgs a) {
  __shared__ unsigned long long red[2][SF_T];
  constexpr int PER = SF_T / G;                        // bins per workgroup
  const int b = blockIdx.y, tid = threadIdx.x;
  double* cout_ = a.io ? a.io[b].cont_sum : field_ptr(a.cont_sum, a.nb, b);
  double* pout = a.io ? a.io[b].pm1_sum : field_ptr(a.pm1_sum, a.nb, b);
  const int last = (int)gridDim.x - 1;
  if ((int)blockIdx.x < last) {
    // bins 0 .. nb - 2, G lanes each (a group lies inside one wave: the shuffles stay uniform)
    const int bin = (int)blockIdx.x * PER + tid / G;
    if (bin < a.nb - 1) bin_out<G>(a, b, bin, tid % G, cout_, pout);
    return;
  }
  if (a.nb >= 1 && tid < 64) bin_out<64>(a, b, a.nb - 1, tid, cout_, pout);   // the corner slot: one wave
  if (!a.cpart) return;                                           // uniform over the workgroup
  uint64_t* out = a.io ? a.io[b].counts : field_ptr(a.counts, 2, b);
  if (!out) return;
  const uint2* part = reinterpret_cast<const uint2*>(a.cpart) + (long long)b * a.ntc;
  unsigned long long np = 0, nn = 0;
  for (int t = tid; t < a.ntc; t += SF_T) {
    const uint2 v = part[t];
    np += v.x;
    nn += v.y;
  }
  red[0][tid] = np;
  red[1][tid] = nn;
  __syncthreads();
  for (int o = SF_T / 2; o > 0; o >>= 1) {
    if (tid < o) {
      red[0][tid] += red[0][tid + o];
      red[1][tid] += red[1][tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
  }
}

hipError_t launch_spec_final(const SpecFinalArgs& a, int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  // partials per bin (the larger of the two spectra's): a wave per bin from 64 on
  const long long mc = a.coff_c ? a.M_c : 0, mp = a.coff_p ? a.M_p : 0;
  const bool wide = (mc > mp ? mc : mp) > 64LL * a.nb;
  const int per = wide ? SF_T / 64 : SF_T / 8;
  // the regular bins (none without spectra), then the corner slot and the counts
  const unsigned gx = (unsigned)((a.nb > 1 ? (a.nb - 1 + per - 1) / per : 0) + 1);
  if (wide) hipLaunchKernelGGL((k_spec_final<64>), dim3(gx, (unsigned)batch), dim3(SF_T), 0, st, a);
  else hipLaunchKernelGGL((k_spec_final<8>), dim3(gx, (unsigned)batch), dim3(SF_T), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// standalone threshold: grid-stride over N values of each field
// ---------------------------------------------------------------------------------------------
constexpr int THR_UNROLL = 4;                 // 16-byte vectors per thread per step, loads first

__global__ void __launch_bounds__(256) k_threshold(ThreshArgs a) {
  __shared__ unsigned red[2][4];
  const int b = blockIdx.y;
  const float* f = a.field + (long long)b * a.N;
  int8_t* t = a.out + (long long)b * a.N;
  unsigned np = 0, nn = 0;
  // four voxels per vector (N is a multiple of 4 on every supported grid): a 16-byte load, one
  // 4-byte store of the four signs
  const long long n4 = a.N >> 2;
  const float4* f4 = reinterpret_cast<const float4*>(f);
  uint32_t* t4 = reinterpret_cast<uint32_t*>(t);
  const long long step = (long long)gridDim.x * 256 * THR_UNROLL;
  for (long long i0 = (long long)blockIdx.x * 256 * THR_UNROLL + threadIdx.x; i0 < n4; i0 += step) {
    float4 x4[THR_UNROLL];
#pragma unroll
    for (int u = 0; u < THR_UNROLL; ++u) {
      const long long i = i0 + u * 256;
      x4[u] = i < n4 ? f4[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
#pragma unroll
    for (int u = 0; u < THR_UNROLL; ++u) {
      const long long i = i0 + u * 256;
      if (i >= n4) break;
      const float xs[4] = {x4[u].x, x4[u].y, x4[u].z, x4[u].w};
      uint32_t packed = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool pos = xs[q] >= a.level;
        packed |= (pos ? 0x01u : 0xFFu) << (8 * q);
        np += pos;
        nn += fabsf(xs[q] - a.level) < a.near_tol;
      }
      t4[i] = packed;
    }
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

hipError_t launch_threshold(const ThreshArgs& a, int batch, hipStream_t st) {
  if (a.N % 4 != 0) return hipErrorInvalidValue;   // every supported grid has an even x and another even axis
  if (batch <= 0) return hipSuccess;
  // one step per workgroup; with counts, about 1024 workgroups over the whole batch instead:
  // still enough loads in flight to stream, and few count atomics per field (they serialise on
  // the counters' cache line: one workgroup per 1024 voxels took 1 ms for 16 x 2048^2)
  long long blocks = (a.N / 4 + 256 * THR_UNROLL - 1) / (256 * THR_UNROLL);
  const long long cap = 1024 / batch > 0 ? 1024 / batch : 1;
  if (a.counts && blocks > cap) blocks = cap;
  hipLaunchKernelGGL(k_threshold, dim3((unsigned)blocks, batch), dim3(256), 0, st, a);
  return hipGetLastError();
}

__global__ void k_zero_u64(uint64_t* p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

hipError_t launch_zero_u64(uint64_t* p, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
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

hipError_t launch_debug_philox(uint64_t seed, uint64_t first, uint64_t count, uint32_t* words, float* normals,
                               hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_debug_philox, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, seed, first, count,
                     words, normals);
  return hipGetLastError();
}

}  // namespace hu
