// Spectrum binning passes and small utility kernels.
//
//   cols_bin    forward FFT along axis 0 and the binned periodogram |X|^2 / N of the +-1 field
//               (or of any real input), read only;
//   bin_geom    once per grid and bin layout: the bin of every half-spectrum mode (optionally
//               stored as a table, column-major for the axis-0 passes) and the per-bin mode counts;
//   threshold   the standalone sign map with counts;
//   debug_philox  raw Philox words and normals for the parity tests.
#include "hu_common.hpp"

namespace hu {

// One tile per workgroup; the FP64 histogram shares the exchange buffer and is flushed per tile.
template <int L, int V>
__global__ void __launch_bounds__((ColTile<L, V>::T)) k_cols_bin(BinArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = ColTile<L, V>::C, T = ColTile<L, V>::T;
  constexpr int LP = ColTile<L, V>::LP;
  using Rad = typename Plan<L>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
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
  fft_run<L, P, E, false>(Rad{}, v, lds + c * ColTile<L, V>::RS, p, a.tw);
  const float wm = (valid && col_coord(a.gm, g).wm > 1.5f) ? 2.0f : 1.0f;
  float* pw = reinterpret_cast<float*>(lds);
  double* hs = reinterpret_cast<double*>(pw + ((C * LP + 1) & ~1));
  __syncthreads();                                  // the exchange buffer is free from here
#pragma unroll
  for (int s = 0; s < E; ++s)
    pw[c * LP + pw_index(slot_index<L, RL, P>(s, p))] = wm * (v[s].x * v[s].x + v[s].y * v[s].y);
  for (int i = tid; i < a.nb; i += T) hs[i] = 0.0;
  __syncthreads();
  bin_tile<L, E, C, LP>(pw, hs, a.table, (int)tile * C, a.gm.ncol, tid);
  __syncthreads();
  double* out = a.io ? a.io[b].pm1_sum : field_ptr(a.sum, a.nb, b);
  if (out) hist_flush(hs, a.nb, 1.0 / (double)a.N, out, tid, T);
}

// Persistent, when the FP64 histogram fits beyond the exchange buffer with two workgroups per CU:
// each workgroup takes a contiguous chunk of (field, tile) pairs, keeps one histogram per field
// (flushed when the field changes) and requests the next tile's columns into the transform's
// registers once the current power values are in LDS, so their loads overlap the binning.
template <int L, int V>
__global__ void __launch_bounds__((ColTile<L, V>::T)) k_cols_bin_keep(BinArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = ColTile<L, V>::C, T = ColTile<L, V>::T;
  constexpr int LP = ColTile<L, V>::LP;
  using Rad = typename Plan<L>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  const int total = a.sc.batch * a.sc.ntiles;
  const int per = (total + (int)gridDim.x - 1) / (int)gridDim.x;
  int lin = (int)blockIdx.x * per;
  const int end = lin + per < total ? lin + per : total;
  if (lin >= end) return;
  const int tid = threadIdx.x;
  const int c = tid % C, p = tid / C;
  float* pw = reinterpret_cast<float*>(lds);
  double* hs = reinterpret_cast<double*>(reinterpret_cast<char*>(lds) + a.hs_off);
  const double scale = 1.0 / (double)a.N;
  int b = lin / a.sc.ntiles;
  int tile = lin - b * a.sc.ntiles;
  for (int i = tid; i < a.nb; i += T) hs[i] = 0.0;
  float2 v[E];
  col_load<L, R1, P, E>(v, col_io<L>(a.spec + (long long)b * a.Nh, a.Nh, a.gm.inner0, tile * C + c, p));
  for (;;) {
    const int g = tile * C + c;
    const bool valid = g < a.gm.ncol;
    fft_run<L, P, E, false>(Rad{}, v, lds + c * ColTile<L, V>::RS, p, a.tw);
    const float wm = (valid && col_coord(a.gm, g).wm > 1.5f) ? 2.0f : 1.0f;
    __syncthreads();                                // the exchange buffer is free from here
#pragma unroll
    for (int s = 0; s < E; ++s)
      pw[c * LP + pw_index(slot_index<L, RL, P>(s, p))] = wm * (v[s].x * v[s].x + v[s].y * v[s].y);
    __syncthreads();
    ++lin;
    const int bn = lin / a.sc.ntiles, tn = lin - bn * a.sc.ntiles;
    if (lin < end) col_load<L, R1, P, E>(v, col_io<L>(a.spec + (long long)bn * a.Nh, a.Nh, a.gm.inner0, tn * C + c, p));
    bin_tile<L, E, C, LP>(pw, hs, a.table, tile * C, a.gm.ncol, tid);
    __syncthreads();
    if (lin == end || bn != b) {
      double* out = a.io ? a.io[b].pm1_sum : field_ptr(a.sum, a.nb, b);
      if (out) hist_flush(hs, a.nb, scale, out, tid, T);
      if (lin == end) break;
      __syncthreads();                              // the flush has read hs
      for (int i = tid; i < a.nb; i += T) hs[i] = 0.0;
    }
    b = bn;
    tile = tn;
  }
}

template <int L, int V>
static hipError_t launch_cols_bin_L(BinArgs a, hipStream_t st) {
  constexpr int T = ColTile<L, V>::T;
  const long long total = (long long)a.sc.batch * a.sc.ntiles;
  if (total == 0) return hipSuccess;
  const size_t x = col_xchg_bytes<L, V>();
  const size_t pwb = (size_t)ColTile<L, V>::C * ColTile<L, V>::LP * 4;
  const size_t base = ((x > pwb ? x : pwb) + 15) / 16 * 16;
  const size_t keep = base + (size_t)a.nb * 8;
  if (keep <= LDS_PER_CU / 2) {
    a.hs_off = (int)base;
    int slots = 0;
    const hipError_t e = resident_blocks(reinterpret_cast<const void*>(&k_cols_bin_keep<L, V>), T, keep, &slots);
    if (e != hipSuccess) return e;
    const long long per = (total + slots - 1) / slots;
    const unsigned grid = (unsigned)((total + per - 1) / per);
    hipLaunchKernelGGL((k_cols_bin_keep<L, V>), dim3(grid), dim3(T), keep, st, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_cols_bin<L, V>), dim3(sched_blocks(a.sc)), dim3(T), (col_lds_bytes_t<L, V>(a.nb)), st, a);
  return hipGetLastError();
}

hipError_t launch_cols_bin(int L, int variant, const BinArgs& a, hipStream_t st) {
  switch (L) {
#define X(LL) case LL: return variant ? launch_cols_bin_L<LL, 1>(a, st) : launch_cols_bin_L<LL, 0>(a, st);
    HU_COL_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------------------------
// bin geometry: grid-stride over the Nh modes in half-spectrum order (m_0 slowest, column g
// fastest); LDS-privatised u32 counts, flushed with 64-bit atomics (integers: deterministic).
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_bin_geom(BinGeomArgs a) {
  extern __shared__ unsigned hcnt[];
  for (int i = threadIdx.x; i < a.nb; i += 256) hcnt[i] = 0u;
  __syncthreads();
  const long long ncol = a.gm.ncol;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < a.Nh; i += (long long)gridDim.x * 256) {
    const int g = (int)(i % ncol);
    const int e = (int)(i / ncol);
    const ColCoord cc = col_coord(a.gm, g);
    const int bi = mode_bin(a.bd, a.gm, cc, e);
    if (a.table) a.table[g * (long long)a.gm.n0 + e] = (uint16_t)bi;
    atomicAdd(hcnt + bi, (unsigned)cc.wm);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < a.nb; i += 256)
    if (hcnt[i]) atomicAdd(a.counts + i, (unsigned long long)hcnt[i]);
}

hipError_t launch_bin_geom(const BinGeomArgs& a, hipStream_t st) {
  long long blocks = (a.Nh + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_bin_geom, dim3((unsigned)blocks), dim3(256), (size_t)a.nb * sizeof(unsigned), st, a);
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
