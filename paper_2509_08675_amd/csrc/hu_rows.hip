// Row passes along x (the fastest axis) of the hyperuniform-field pipeline.
//
//   rows_r2c   white noise (Philox4x32-10 + Box-Muller) or a real input -> real-to-complex
//              transform of each x row: an n_x/2-point complex FFT of the packed samples
//              x[2n] + i x[2n+1] followed by the split twist;
//   rows_c2r   inverse of that for each x row, then the normalisation of Eq. (15) with the
//              statistics of the filter pass, the FP32 field and the +-1 sign map (stored from
//              the transform's registers, or through the wave's LDS regions in address order
//              when a wave holds several rows) with per-tile counts, and the real-to-complex
//              transform of the +-1 row written back in place.
//
// Half-spectrum layout seen by the row passes: element k of row r sits at
//   2D (column groups of four): (k >> 2) (nrows 4) + 4 r + (k & 3);
//   3D (row-major):             r (L + 1) + k.
// The C rows of a tile therefore occupy, in 2D, one contiguous run of 4C elements per group of
// four k (so a 4-row tile and a 4-column tile of the axis-0 pass both move whole 128-byte
// lines), and in 3D one contiguous run of C (L + 1) elements.  Global loads and stores walk these
// runs in address order through buffer descriptors, decoupled from the FFT's thread mapping by
// LDS; the walk advances by constant steps, so no per-element division or 64-bit address is
// formed.  In 2D a lane moves the pair k, k + 1 (k even) of one row as one 16-byte access.
#include "hu_common.hpp"

namespace hu {

// Address-order walk over the half rows X[0..L] of a tile.  Unit u of the tile covers element k
// of tile row cc at element offset goff from the tile's first element (2D: the first run of the
// tile; 3D: the tile's first row).  Each thread visits ITERS units with compile-time strides, so
// the walk unrolls and every global load of a thread is in flight at once.
template <int L, int C, int T, bool TILED>
struct RowWalk {
  static constexpr int GS = TILED ? 4 * C : L + 1;   // elements per run
  static constexpr int NG = TILED ? L / 4 + 1 : C;   // runs per tile
  static constexpr int NU = NG * GS;
  static constexpr int PR = T / C;                   // threads per row
  // 2D steady: each thread keeps one position w in the 4C-element run and steps over runs;
  // 3D: the threads of row cc walk its L + 1 contiguous elements
  static constexpr bool STEADY = TILED && (T % GS) == 0;
  static constexpr int QS = STEADY ? T / GS : 1;     // runs per sweep
  static constexpr int ITERS = STEADY ? (NG + QS - 1) / QS : (!TILED ? (L + 1 + PR - 1) / PR : (NU + T - 1) / T);

  // unit `it` of thread tid: tile row, element k, element offset; false when outside the tile
  __device__ __forceinline__ static bool unit(int tid, int it, unsigned run_stride, int rows_here, int& cc, int& k,
                                              unsigned& goff) {
    if constexpr (STEADY) {
      const int w = tid % GS;
      const int q = tid / GS + it * QS;
      cc = w >> 2;
      k = 4 * q + (w & 3);
      goff = (unsigned)q * run_stride + (unsigned)w;
      return q < NG && k <= L && cc < rows_here;
    } else if constexpr (!TILED) {
      cc = tid / PR;
      k = tid % PR + it * PR;
      goff = (unsigned)(cc * (L + 1) + k);
      return k <= L && cc < rows_here;
    } else {
      const int u = tid + it * T;
      const int q = u / GS, w = u - q * GS;
      cc = w >> 2;
      k = 4 * q + (w & 3);
      goff = (unsigned)q * run_stride + (unsigned)w;
      return u < NU && k <= L && cc < rows_here;
    }
  }
};

// R2C split twist of every row of the tile from Z in LDS (padded, natural order) to the half
// spectrum, in address order:
//   X[k] = (Z[k] + Z*[L-k])/2 - (i/2) e^{-2 pi i k / 2L} (Z[k] - Z*[L-k]),  X[L] = Re Z[0] - Im Z[0].
// The twist factor of element k, e^{-i pi k / L} (the table tw2), for the units of the row walk.
// Where k splits into a per-thread part and a per-iteration part (k = kt + 4 QS it in the steady
// 2D walk, k = kt + PR it in the 3D walk), FACT forms it as tw2[kt] tw2[ki]: one vector load per
// thread and a uniform (scalar) load per iteration instead of a vector load per unit.
template <int L, int C, int T, bool TILED>
struct TwistSplit {
  using W = RowWalk<L, C, T, TILED>;
  static constexpr bool ok = W::STEADY || !TILED;
  static constexpr int KI = W::STEADY ? 4 * W::QS : W::PR;   // k step per iteration
  __device__ __forceinline__ static int kt(int tid) {
    if constexpr (W::STEADY) return 4 * (tid / W::GS) + ((tid % W::GS) & 3);
    else return tid % W::PR;
  }
};

template <int L, int C, int T, bool TILED, int RS, bool FACT>
__device__ __forceinline__ void twist_store_rows(const float2* lds, rsrc_t tw2, const float2* tw2p, rsrc_t spec,
                                                 unsigned tile_off, unsigned run_stride, int rows_here, int tid) {
  using W = RowWalk<L, C, T, TILED>;
  using TS = TwistSplit<L, C, T, TILED>;
  constexpr bool SPLIT = FACT && TS::ok;
  if constexpr (W::STEADY && (L % 4) == 0 && Plan<L>::E == 16) {
    // 2D: each lane forms the pair X[k], X[k + 1] (k even) of one row and stores it as 16 bytes.
    // FACT: k = kt + KI2 it, so the twist factors are tw2[kt] tw2[KI2 it] and tw2[kt + 1]
    // tw2[KI2 it]; otherwise the pair tw2[k], tw2[k + 1] is loaded for every step (all first)
    constexpr int GP = W::GS / 2, QP = T / GP, IT2 = (W::NG + QP - 1) / QP, KI2 = 4 * QP;
    const int w = tid % GP;
    const int cc = w >> 1, kl = 2 * (w & 1);
    const int kt = 4 * (tid / GP) + kl;
    const float2 wa = buf_load2(tw2, (unsigned)(kt < L ? kt : 0) * 8u, 0);
    const float2 wb = buf_load2(tw2, (unsigned)(kt + 1 < L ? kt + 1 : 0) * 8u, 0);
    u32x4 tp[FACT ? 1 : IT2];
    if constexpr (!FACT) {
#pragma unroll
      for (int it = 0; it < IT2; ++it) {
        const int k = kt + KI2 * it;
        tp[it] = buf_load4(tw2, (unsigned)(k + 1 < L ? k : 0) * 8u, 0);
      }
    }
    const float2* lz = lds + cc * RS;
    auto twist = [&](int k, float2 tw) {
      const float2 zk = lz[lidx(k)];
      const float2 zm = cconj(lz[lidx(k == 0 ? 0 : L - k)]);
      const float2 A = cadd(zk, zm), B = csub(zk, zm);
      return cscale(cadd(A, mul_mi<false>(cmul(tw, B))), 0.5f);
    };
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
      const int q = tid / GP + it * QP;
      const int k = 4 * q + kl;
      if (!(q < W::NG && cc < rows_here) || k > L) continue;
      const unsigned off = (tile_off + (unsigned)q * run_stride + 2u * w) * 8u;
      if (k == L) {
        const float2 z0 = lz[0];
        buf_store2(spec, make_float2(z0.x - z0.y, 0.0f), off, 0);
        continue;
      }
      float2 ta, tb;
      if constexpr (FACT) {
        const float2 tu = (KI2 * it < L) ? uniform_load2(tw2p, KI2 * it) : make_float2(1.0f, 0.0f);
        ta = (KI2 * it < L) ? cmul(wa, tu) : wa;
        tb = (KI2 * it < L) ? cmul(wb, tu) : wb;
      } else {
        ta = make_float2(__uint_as_float(tp[it].x), __uint_as_float(tp[it].y));
        tb = make_float2(__uint_as_float(tp[it].z), __uint_as_float(tp[it].w));
      }
      const float2 X0 = twist(k, ta);
      const float2 X1 = twist(k + 1, tb);
      buf_store4(spec, u32x4{__float_as_uint(X0.x), __float_as_uint(X0.y), __float_as_uint(X1.x), __float_as_uint(X1.y)},
                 off, 0);
    }
    return;
  }
  constexpr int NW = SPLIT ? 1 : W::ITERS;
  float2 w[NW];
  if constexpr (SPLIT) {
    const int kt = TS::kt(tid);
    w[0] = buf_load2(tw2, (unsigned)(kt < L ? kt : 0) * 8u, 0);
  } else {
#pragma unroll
    for (int it = 0; it < W::ITERS; ++it) {        // the twiddles first: all loads in flight together
      int cc, k;
      unsigned goff;
      const bool in = W::unit(tid, it, run_stride, rows_here, cc, k, goff);
      w[it] = buf_load2(tw2, (unsigned)(in && k < L ? k : 0) * 8u, 0);
    }
  }
#pragma unroll
  for (int it = 0; it < W::ITERS; ++it) {
    int cc, k;
    unsigned goff;
    if (!W::unit(tid, it, run_stride, rows_here, cc, k, goff)) continue;
    const float2* lz = lds + cc * RS;
    float2 X;
    if (k == L) {
      const float2 z0 = lz[0];
      X = make_float2(z0.x - z0.y, 0.0f);
    } else {
      const float2 zk = lz[lidx(k)];
      const float2 zm = cconj(lz[lidx(k == 0 ? 0 : L - k)]);
      const float2 A = cadd(zk, zm), B = csub(zk, zm);
      float2 tw;
      if constexpr (SPLIT) {
        tw = (TS::KI * it < L) ? cmul(w[0], uniform_load2(tw2p, TS::KI * it)) : w[0];
      } else {
        tw = w[it];
      }
      X = cscale(cadd(A, mul_mi<false>(cmul(tw, B))), 0.5f);
    }
    buf_store2(spec, X, (tile_off + goff) * 8u, 0);
  }
}

// The tile's half rows X[0..L] from the half spectrum into LDS (padded, natural order), in
// address order; X[0] and X[L] are made real (the other axes' inverse transforms leave them so up
// to rounding).
template <int L, int C, int T, bool TILED, int RS>
__device__ __forceinline__ void load_rows(float2* lds, rsrc_t spec, unsigned tile_off, unsigned run_stride,
                                          int rows_here, int tid) {
  using W = RowWalk<L, C, T, TILED>;
  if constexpr (W::STEADY && (L % 4) == 0 && Plan<L>::E == 16) {
    // 2D: 16-byte loads, each the pair k, k + 1 (k even) of one row inside a run of the tile
    constexpr int GP = W::GS / 2;                  // pairs per run
    constexpr int QP = T / GP;                     // runs per sweep
    constexpr int IT2 = (W::NG + QP - 1) / QP;
    const int w = tid % GP;
    const int cc = w >> 1, kl = 2 * (w & 1);       // row and k & 3 of the pair's first element
    u32x4 x[IT2];
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
      const int q = tid / GP + it * QP;
      const bool in = q < W::NG && cc < rows_here;
      x[it] = buf_load4(spec, in ? (tile_off + (unsigned)q * run_stride + 2u * w) * 8u : 0xFFFFFFF0u, 0);
    }
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
      const int q = tid / GP + it * QP;
      if (!(q < W::NG && cc < rows_here)) continue;
      const int k = 4 * q + kl;                    // k + 1 is odd, so never L
      if (k > L) continue;
      float2 v0 = make_float2(__uint_as_float(x[it].x), __uint_as_float(x[it].y));
      const float2 v1 = make_float2(__uint_as_float(x[it].z), __uint_as_float(x[it].w));
      if (k == 0 || k == L) v0.y = 0.0f;
      lds[cc * RS + lidx(k)] = v0;
      if (k < L) lds[cc * RS + lidx(k + 1)] = v1;
    }
    return;
  }
  float2 x[W::ITERS];
#pragma unroll
  for (int it = 0; it < W::ITERS; ++it) {
    int cc, k;
    unsigned goff;
    const bool in = W::unit(tid, it, run_stride, rows_here, cc, k, goff);
    x[it] = buf_load2(spec, in ? (tile_off + goff) * 8u : 0xFFFFFFF0u, 0);   // outside: past the end, reads 0
  }
#pragma unroll
  for (int it = 0; it < W::ITERS; ++it) {
    int cc, k;
    unsigned goff;
    if (!W::unit(tid, it, run_stride, rows_here, cc, k, goff)) continue;
    float2 v = x[it];
    if (k == 0 || k == L) v.y = 0.0f;
    lds[cc * RS + lidx(k)] = v;
  }
}

// LDS positions of element L - (p + P b + r L/R): the mirrored read of the C2R pre-twist, from one
// per-thread base when the offsets are thread-independent (checked at compile time).
template <int L, int R, int P, int E>
struct MirrorMap {
  static constexpr int off(int p, int b, int r) { return lidx(L - (p + P * b + r * (L / R))) - lidx(L - p); }
  static constexpr bool check() {
    for (int p = 0; p < P; ++p)
      for (int b = 0; b < E / R; ++b)
        for (int r = 0; r < R; ++r)
          if (off(p, b, r) != off(0, b, r)) return false;
    return true;
  }
  static constexpr bool lin = check();
};

// Tile geometry of the half spectrum: the element offset of the tile's first element and the
// element stride between consecutive runs.
template <bool TILED, int L>
__device__ __forceinline__ void tile_geom(long long row0, long long nrows, unsigned& tile_off, unsigned& run_stride) {
  if constexpr (TILED) {
    tile_off = (unsigned)(row0 * 4);
    run_stride = (unsigned)(nrows * 4);
  } else {
    tile_off = (unsigned)(row0 * (L + 1));
    run_stride = 0u;
  }
}

// grid (ceil(nrows / C), B), block C * P; thread (c, p) = (tid / P, tid % P) transforms row c.
template <int L, int SRC, bool TILED, int V>
__global__ void __launch_bounds__((RowTile<L, V>::T)) k_rows_r2c(RowsArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = RowTile<L, V>::C, T = RowTile<L, V>::T;
  constexpr int RS = RowTile<L, V>::RS;
  using Rad = typename Plan<L>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  float* ldsf = reinterpret_cast<float*>(lds);
  const int tid = threadIdx.x;
  const int c = tid / P, p = tid % P;
  const int b = blockIdx.y;
  const long long row0 = (long long)blockIdx.x * C;
  const long long nx = 2 * L;

  if (blockIdx.x == 0) {                        // set up this field's outputs and counters for later passes
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

  // ---- the C real rows into LDS: sample x of row c goes to float 2 lidx(x / 2) + (x & 1) of region c
  const long long v0 = row0 * nx;
  const int rows_here = (int)((a.nrows - row0) < C ? (a.nrows - row0) : C);
  const int nv = rows_here * 2 * L;
  if constexpr (SRC == SRC_NOISE) {
    // voxel i of the field takes normal i mod 4 of Philox block i / 4
    uint64_t seed;
    if (a.io) seed = a.io[b].seed;
    else seed = a.seeds[b];
    seed = uniform_u64(seed);
    if constexpr ((L % 2) == 0) {
      // rows of 2L voxels, a multiple of 4: each block lies in one row and fills complex
      // elements 2j, 2j + 1 of it, which are adjacent in LDS (2j + 1 never starts a padded group)
      constexpr int BPR = L / 2;                    // blocks per row
      const uint64_t m0 = (uint64_t)(v0 >> 2);
      const int nblk = rows_here * BPR;
      for (int i = tid; i < nblk; i += T) {
        float z[4];
        noise4(m0 + (uint64_t)i, seed, z);
        const int rc = i / BPR, j = i - rc * BPR;
        float2* d = lds + rc * RS + lidx(2 * j);
        d[0] = make_float2(z[0], z[1]);
        d[1] = make_float2(z[2], z[3]);
      }
    } else {
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
    }
  } else if constexpr ((SRC == SRC_F32 && L % 2 == 0) || (SRC == SRC_I8 && L % 8 == 0)) {
    // the tile's rows are contiguous and every row is a whole number of 16-byte vectors: all of a
    // thread's vector loads are issued first (rows past the field read 0), then written to LDS as
    // complex pairs (a vector never crosses a row, and a pair never straddles a padded group)
    constexpr int ESZ = SRC == SRC_F32 ? 4 : 1;
    constexpr int SPV = 16 / ESZ;                 // samples per vector
    constexpr int NV = C * 2 * L / SPV;           // vectors per full tile
    constexpr int IT = (NV + T - 1) / T;
    const char* src = reinterpret_cast<const char*>(a.src) + ((long long)b * a.N + v0) * ESZ;
    const rsrc_t rs = make_rsrc(src, (unsigned)nv * ESZ);
    u32x4 w[IT];
    __builtin_amdgcn_s_setprio(2);                // as in the last row pass: loads in flight early
#pragma unroll
    for (int it = 0; it < IT; ++it) w[it] = buf_load4(rs, (unsigned)(tid + it * T) * 16u, 0);
    __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int iv = tid + it * T;
      if (NV % T != 0 && iv >= NV) break;
      const int s0 = iv * SPV;
      const int rc = s0 / (2 * L), j0 = (s0 - rc * 2 * L) >> 1;
      float2* d = lds + rc * RS;
      if constexpr (SRC == SRC_F32) {
        using f32x4 = __attribute__((ext_vector_type(4))) float;
        const f32x4 f = __builtin_bit_cast(f32x4, w[it]);   // the whole vector (not per element)
        d[lidx(j0)] = make_float2(f.x, f.y);
        d[lidx(j0 + 1)] = make_float2(f.z, f.w);
      } else {
        const unsigned ws[4] = {w[it].x, w[it].y, w[it].z, w[it].w};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const unsigned u = ws[q >> 1] >> (16 * (q & 1));
          d[lidx(j0 + q)] = make_float2((float)(int8_t)(u & 0xFFu), (float)(int8_t)((u >> 8) & 0xFFu));
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

  constexpr bool WV = (64 % P) == 0;             // each row inside one wave
  float2 v[E];
  float2* lrow = lds + c * RS;
  stage_load<L, R1, P, E>(v, lrow, p);
  fft_run<L, P, E, false, WV>(Rad{}, v, lrow, p, a.tw);
  xchg_sync<WV>();
  slot_store<L, RL, P, E>(v, lrow, p);
  __syncthreads();
  unsigned tile_off, run_stride;
  tile_geom<TILED, L>(row0, a.nrows, tile_off, run_stride);
  const rsrc_t spec = make_rsrc(a.spec + (long long)b * a.Nh, (unsigned)(a.Nh * 8));
  const rsrc_t tw2 = make_rsrc(a.tw2, (unsigned)(L * 8));
  twist_store_rows<L, C, T, TILED, RS, false>(lds, tw2, a.tw2, spec, tile_off, run_stride, rows_here, tid);
}

// C2R along x -> normalise -> field, sign map, counts -> R2C of the +-1 row (THRESH).
template <int L, bool THRESH, bool TILED, int V>
__global__ void __launch_bounds__((RowTile<L, V>::T)) k_rows_c2r(RowsZArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = RowTile<L, V>::C, T = RowTile<L, V>::T;
  constexpr int RS = RowTile<L, V>::RS;
  using Rad = typename Plan<L>::fwd;
  using RadF = Reverse<Rad>;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  __shared__ unsigned red_u[2][T / 64 > 0 ? T / 64 : 1];
  const int tid = threadIdx.x;
  const int c = tid / P, p = tid % P;
  const int b = blockIdx.y;
  const long long row0 = (long long)blockIdx.x * C;
  const int rows_here = (int)((a.nrows - row0) < C ? (a.nrows - row0) : C);
  float2* lrow = lds + c * RS;
  unsigned tile_off, run_stride;
  tile_geom<TILED, L>(row0, a.nrows, tile_off, run_stride);
  const rsrc_t spec = make_rsrc(a.spec + (long long)b * a.Nh, (unsigned)(a.Nh * 8));
  const rsrc_t tw2 = make_rsrc(a.tw2, (unsigned)(L * 8));

  // ---- the tile's half rows X[0..L] into LDS, in address order.  The waves issue these loads at
  //      raised priority, so a workgroup starting its tile gets its loads in flight ahead of the
  //      transform work of the other resident workgroups (2D 197 -> 194 us, 3D 168 -> 160 us).
  __builtin_amdgcn_s_setprio(2);
  load_rows<L, C, T, TILED, RS>(lds, spec, tile_off, run_stride, rows_here, tid);
  __builtin_amdgcn_s_setprio(0);
  __syncthreads();
  // ---- pre-twist: Z[k] = (X[k] + X*[L-k]) + i e^{+2 pi i k / 2L} (X[k] - X*[L-k])
  float2 v[E];
  {
    const float2 tp = buf_load2(tw2, (unsigned)p * 8u, 0);
    using M = LoadMap<L, R1, P, E>;
    using MM = MirrorMap<L, R1, P, E>;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int bb = s / R1, r = s % R1;
      const int k = slot_index<L, R1, P>(s, p);
      const float2 xk = M::lin ? lrow[lidx(p) + M::off(0, bb, r)] : lrow[lidx(k)];
      const float2 xc = cconj(MM::lin ? lrow[lidx(L - p) + MM::off(0, bb, r)] : lrow[lidx(L - k)]);
      // e^{+i pi k / L} = conj(tw2[p] tw2[k - p]): the second factor is uniform (a scalar load)
      const float2 w = cconj(cmul(tp, uniform_load2(a.tw2, slot_index<L, R1, P>(s, 0))));
      v[s] = cadd(cadd(xk, xc), mul_mi<true>(cmul(w, csub(xk, xc))));
    }
  }
  constexpr bool WV = (64 % P) == 0;             // each row inside one wave
  fft_run<L, P, E, true, WV>(Rad{}, v, lrow, p, a.tw);

  // ---- normalise (Eq. (15)) in registers.  With one row per wave the field and the sign map go
  //      out straight from the slots: in slot s the P threads of a row hold P consecutive complex
  //      elements, i.e. 2P consecutive voxels, so each store instruction writes contiguous memory
  //      (with several rows per wave, see STAGE below).
  const double* fs = a.fstats + (long long)b * 8;
  const float scale = (float)fs[4], offset = (float)fs[5];
  float* fout;
  int8_t* tout;
  float near_tol;
  if (a.io) {
    const FieldIO& io = a.io[b];
    fout = io.field;
    tout = io.pm1;
    near_tol = io.near_abs;
  } else {
    fout = field_ptr(a.field, a.N, b);
    tout = field_ptr(a.pm1, a.N, b);
    near_tol = a.near_tol;
  }
  const long long gbase = row0 * 2 * L;
  // stores past the tile's rows, and all stores of an absent output (size 0), are dropped
  const unsigned tile_vox = (unsigned)rows_here * 2u * L;
  const rsrc_t fo = make_rsrc(fout ? fout + gbase : nullptr, fout ? tile_vox * 4u : 0u);
  const rsrc_t to = make_rsrc(tout ? tout + gbase : nullptr, tout ? tile_vox : 0u);
  const bool row_ok = c < rows_here;
  const unsigned vox0 = (unsigned)(c * 2 * L + 2 * p);      // voxel of this thread's slot-0 element
  unsigned npos = 0, nnear = 0;
  // STAGE: the rows of a wave are contiguous in the field and the sign map, so the wave writes its
  // normalised values to its own LDS regions and stores them back in address order, 16 bytes of
  // the field and 4 of the map per lane (rather than 2P-voxel pieces of 64 / P rows per store)
  constexpr int NRW = 64 / P;                        // rows per wave
  constexpr int NQW = NRW * 2 * L / 4;               // four-voxel groups per wave
  constexpr bool STAGE = WV && NRW > 1 && (L % 2) == 0 && (NQW % 64) == 0 && (RS >= L);
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const unsigned so = 2u * (unsigned)slot_index<L, RL, P>(s, 0);
    const float x0 = fmaf(v[s].x, scale, offset);
    const float x1 = fmaf(v[s].y, scale, offset);
    if constexpr (STAGE) lrow[slot_index<L, RL, P>(s, 0) + p] = make_float2(x0, x1);
    else buf_store2(fo, make_float2(x0, x1), vox0 * 4u, so * 4u);
    if constexpr (THRESH) {
      const bool p0 = x0 >= 0.0f, p1 = x1 >= 0.0f;
      npos += (unsigned)p0 + (unsigned)p1;
      nnear += (unsigned)(fabsf(x0) < near_tol) + (unsigned)(fabsf(x1) < near_tol);
      if constexpr (!STAGE) {
        const unsigned b0 = p0 ? 0x01u : 0xFFu, b1 = p1 ? 0x0100u : 0xFF00u;
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)(b0 | b1), to, vox0, so, 0);
      }
      v[s] = make_float2(p0 ? 1.0f : -1.0f, p1 ? 1.0f : -1.0f);
    }
  }
  if constexpr (STAGE) {
    xchg_sync<WV>();
    const int lane = tid & 63;
    const int cw = (tid >> 6) * NRW;                 // first tile row of this wave
    const float2* lw = lds + cw * RS;
#pragma unroll
    for (int k = 0; k < NQW / 64; ++k) {
      const int q = lane + 64 * k;                   // four-voxel group q of the wave's rows
      const int j = (4 * q) / (2 * L), x = 4 * q - j * (2 * L);
      const float2 a0 = lw[j * RS + x / 2], a1 = lw[j * RS + x / 2 + 1];
      const unsigned vox = (unsigned)(cw * 2 * L + 4 * q);
      buf_store4(fo, u32x4{__float_as_uint(a0.x), __float_as_uint(a0.y), __float_as_uint(a1.x), __float_as_uint(a1.y)},
                 vox * 4u, 0u);
      if constexpr (THRESH) {
        const unsigned packed = (a0.x >= 0.0f ? 0x01u : 0xFFu) | (a0.y >= 0.0f ? 0x0100u : 0xFF00u) |
                                (a1.x >= 0.0f ? 0x010000u : 0xFF0000u) | (a1.y >= 0.0f ? 0x01000000u : 0xFF000000u);
        __builtin_amdgcn_raw_buffer_store_b32(packed, to, vox, 0u, 0);
      }
    }
    xchg_sync<WV>();                                 // the regions are the next transform's exchange buffer
  }
  if constexpr (THRESH) {
    if (!row_ok) npos = nnear = 0;
    npos = wave_usum(npos);
    nnear = wave_usum(nnear);
    if ((tid & 63) == 0) { red_u[0][tid >> 6] = npos; red_u[1][tid >> 6] = nnear; }
    // forward transform of the packed +-1 row (its first radix is the inverse's last)
    fft_run<L, P, E, false, WV>(RadF{}, v, lrow, p, a.tw);
    xchg_sync<WV>();
    constexpr int RLF = RadInfo<RadF>::last;
    slot_store<L, RLF, P, E>(v, lrow, p);
    __syncthreads();
    twist_store_rows<L, C, T, TILED, RS, true>(lds, tw2, a.tw2, spec, tile_off, run_stride, rows_here, tid);
    // the tile's counts go to their own slot (k_spec_final adds them up): thousands of atomics
    // on one counter line per field would serialise in its L2 channel
    if (tid == 0 && a.cpart) {
      unsigned np = 0, nn = 0;
      for (int w = 0; w < (T + 63) / 64; ++w) { np += red_u[0][w]; nn += red_u[1][w]; }
      reinterpret_cast<uint2*>(a.cpart)[(long long)b * gridDim.x + blockIdx.x] = make_uint2(np, nn);
    }
  }
}

#define HU_ROW_LENGTHS(X) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(1024)

static inline unsigned ceil_div_u(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

template <int L, int SRC, bool TILED, int V>
static hipError_t launch_rows_r2c_L(const RowsArgs& a, int batch, hipStream_t st) {
  constexpr int C = RowTile<L, V>::C, T = RowTile<L, V>::T;
  dim3 grid(ceil_div_u(a.nrows, C), batch);
  constexpr size_t lds = (size_t)C * RowTile<L, V>::RS * sizeof(float2);
  hipLaunchKernelGGL((k_rows_r2c<L, SRC, TILED, V>), grid, dim3(T), lds, st, a);
  return hipGetLastError();
}

template <int L, int SRC>
static hipError_t launch_rows_r2c_S(int variant, const RowsArgs& a, int batch, hipStream_t st) {
  if (variant)
    return a.tiled ? launch_rows_r2c_L<L, SRC, true, 1>(a, batch, st) : launch_rows_r2c_L<L, SRC, false, 1>(a, batch, st);
  return a.tiled ? launch_rows_r2c_L<L, SRC, true, 0>(a, batch, st) : launch_rows_r2c_L<L, SRC, false, 0>(a, batch, st);
}

hipError_t launch_rows_r2c(int L, int src, int variant, const RowsArgs& a, int batch, hipStream_t st) {
  switch (L) {
#define X(LL)                                                                                 \
  case LL:                                                                                    \
    if (src == SRC_NOISE) return launch_rows_r2c_S<LL, SRC_NOISE>(variant, a, batch, st);     \
    if (src == SRC_F32) return launch_rows_r2c_S<LL, SRC_F32>(0, a, batch, st);               \
    return launch_rows_r2c_S<LL, SRC_I8>(0, a, batch, st);
    HU_ROW_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

template <int L, bool THRESH, bool TILED, int V>
static hipError_t launch_rows_c2r_L(const RowsZArgs& a, int batch, hipStream_t st) {
  constexpr int C = RowTile<L, V>::C, T = RowTile<L, V>::T;
  dim3 grid(ceil_div_u(a.nrows, C), batch);
  constexpr size_t lds = (size_t)C * RowTile<L, V>::RS * sizeof(float2);
  hipLaunchKernelGGL((k_rows_c2r<L, THRESH, TILED, V>), grid, dim3(T), lds, st, a);
  return hipGetLastError();
}

template <int L, int V>
static hipError_t launch_rows_c2r_V(bool thresh, const RowsZArgs& a, int batch, hipStream_t st) {
  if (a.tiled)
    return thresh ? launch_rows_c2r_L<L, true, true, V>(a, batch, st) : launch_rows_c2r_L<L, false, true, V>(a, batch, st);
  return thresh ? launch_rows_c2r_L<L, true, false, V>(a, batch, st) : launch_rows_c2r_L<L, false, false, V>(a, batch, st);
}

// workgroups (row tiles) per field of a row pass
int row_tiles(int L, int variant, long long nrows) {
  switch (L) {
#define X(LL)                                                                                   \
  case LL: return (int)ceil_div_u(nrows, variant ? RowTile<LL, 1>::C : RowTile<LL, 0>::C);
    HU_ROW_LENGTHS(X)
#undef X
    default: return -1;
  }
}

hipError_t launch_rows_c2r(int L, bool thresh, int variant, const RowsZArgs& a, int batch, hipStream_t st) {
  switch (L) {
#define X(LL) \
  case LL: return variant ? launch_rows_c2r_V<LL, 1>(thresh, a, batch, st) : launch_rows_c2r_V<LL, 0>(thresh, a, batch, st);
    HU_ROW_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hu
