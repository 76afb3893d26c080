// Device helpers shared by the row and column passes: tile shapes, reductions, the real-to-complex
// split twist, the XCD-aware tile schedule, per-column wavenumber pieces, the symmetrised filter
// amplitude and the run-length bin accumulation.
#pragma once

#include "hu_device.hpp"
#include "hu_internal.hpp"

// column lengths (n along a non-x axis) and row half-lengths (n_x / 2) with compiled kernels
#define HU_COL_LENGTHS(X) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(2048)

namespace hu {

constexpr size_t LDS_PER_CU = 160 * 1024;   // gfx950

// ---------------------------------------------------------------------------------------------
// tile widths: transforms per workgroup
// ---------------------------------------------------------------------------------------------
// V = 0: the default width; V = 1: half of it (more, smaller workgroups), for the autotuner.
template <int L, int V = 0>
struct RowTile {
  static constexpr int P = Plan<L>::P;
  static constexpr int c0 = 256 / P > 0 ? 256 / P : 1;
  static constexpr int cl = 8192 / Region<L>::value > 0 ? 8192 / Region<L>::value : 1;
  static constexpr int cd0 = c0 < cl ? c0 : cl;
  static constexpr int m = 64 / (P < 64 ? P : 64);       // C multiple of m: whole waves
  static constexpr int cd = cd0 / m * m > 0 ? cd0 / m * m : m;
  static constexpr int C = V == 0 ? cd : (cd / 2 / m * m >= m ? cd / 2 / m * m : cd);
  static constexpr int T = C * P;
  static_assert(T % 64 == 0, "row tiles are whole waves");
  static constexpr int RS = Region<L>::value;          // exchange region per row
};

// Offset of the split-exchange region stride beyond L + L/16 floats for the default plan of L and
// C columns per tile: the value in 0 .. 32 with the fewest LDS bank conflicts over every exchange
// store and load of the transform, counted for 32 four-byte banks and 32 lanes per LDS cycle
// (conflict-free for most tiles; 384, 512 and 768 keep some two-way conflicts).
constexpr int split_extra(int L, int C) {
  switch (L) {
    case 6: case 12: case 32: return 1;
    case 48: return C >= 32 ? 0 : 3;
    case 64: case 128: case 192: case 256: return C >= 32 ? 1 : 2;
    case 96: return C >= 32 ? 1 : 0;
    case 384: return C >= 20 ? 14 : 4;
    case 512: return C >= 16 ? 2 : 4;
    case 768: return C >= 10 ? 11 : 8;
    case 1024: return C >= 8 ? 4 : 8;
    case 2048: return C >= 4 ? 8 : 16;
    default: return 0;
  }
}
template <int L, int V = 0>
struct ColTile {
  static constexpr int P = Plan<L>::P;
  static constexpr int a = 8192 / L < 32 ? 8192 / L : 32;   // 64 KB of exchange buffer (unpadded)
  static constexpr int b = 64 / P > a ? 64 / P : a;
  static constexpr int cd0 = b * P > 1024 ? 1024 / P : b;
  static constexpr int m = 64 / (P < 64 ? P : 64);       // C multiple of m: whole waves
  static constexpr int cd = cd0 / m * m > 0 ? cd0 / m * m : m;
  static constexpr int C = V == 0 ? cd : (cd / 2 / m * m >= m ? cd / 2 / m * m : cd);
  static constexpr int T = C * P;
  static_assert(T % 64 == 0, "column tiles are whole waves");
  // exchange region per column.  Wide tiles (a wave spans many columns): the bank-staggered
  // stride.  Narrow tiles (a 16-lane phase spans 4 columns x 4 threads): L + L/16 + 4 complex,
  // i.e. 8 mod 32 words, so the four columns of a phase use disjoint banks.
  static constexpr int RS = C >= 16 ? RegionWide<L>::value : L + (L >> 4) + 4;
  // padded power-value layout for run-length binning: 4 floats after every 16, and an odd
  // number of words per column
  static constexpr int LP = (L + (L / 16) * 4 + 31) / 32 * 32 + 1;
  // split exchange (real and imaginary parts in two rounds): floats per column region
  static constexpr int RSH = L + (L >> 4) + split_extra(L, C);
};

__host__ __device__ constexpr int pw_index(int e) { return e + (e >> 4) * 4; }

// a value the whole wave holds, in scalar registers (the noise seed of a field)
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Calls f(width, radix) with the tile-width choice V and the radix choice RV as integral
// constants; a length without an alternative radix list instantiates only RV = 0.
template <int L, class F>
inline hipError_t with_choices(int variant, int radix, F&& f) {
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  if constexpr (Plan<L, 1>::alt) {
    if (radix) return variant ? f(I1{}, I1{}) : f(I0{}, I1{});
  }
  return variant ? f(I1{}, I0{}) : f(I0{}, I0{});
}
// the same with the exchange choice as a third constant (split only where split_length(L))
template <int L, class F>
inline hipError_t with_choices3(int variant, int radix, int split, F&& f) {
  if constexpr (split_length(L)) {
    if (split)
      return with_choices<L>(variant, radix, [&](auto v, auto r) { return f(v, r, std::true_type{}); });
  }
  return with_choices<L>(variant, radix, [&](auto v, auto r) { return f(v, r, std::false_type{}); });
}

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
    const float2 zk = lz[lidx(k)];
    const float2 zm = cconj(lz[lidx((L - k) % L)]);
    const float2 A = cadd(zk, zm), B = csub(zk, zm);
    const float2 X = cscale(cadd(A, mul_mi<false>(cmul(tw2[k], B))), 0.5f);
    if (valid) out[k] = X;
    if (k == 0 && valid) out[L] = make_float2(zk.x - zk.y, 0.0f);
  }
}

// ---------------------------------------------------------------------------------------------
// XCD-aware tile schedule.  Workgroups are dispatched round-robin over the 8 XCDs (id mod 8), and
// each XCD has its own L2.  Column tiles narrower than a 128-byte line share lines with their
// G - 1 neighbours; those G tiles are given ids id, id + 8, ..., id + 8 (G-1), i.e. the same XCD
// in consecutive dispatch rounds, so the line is fetched once into that XCD's L2.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ bool map_tile(const ColSched& s, int& b, long long& tile) {
  const unsigned id = blockIdx.x;
  const unsigned xcd = id & 7u, round = id >> 3;
  const unsigned j = round % (unsigned)s.G;
  const long long grp = (long long)(round / (unsigned)s.G) * 8 + xcd;
  if (s.finner) {                                 // G = batch: group grp is tile grp, j its field
    b = (int)j;
    tile = grp;
    return tile < s.ntiles;
  }
  const long long lin = grp * s.G + j;
  b = (int)(lin / s.ntiles_pad);
  tile = lin % s.ntiles_pad;
  return b < s.batch && tile < s.ntiles;
}

// workgroups launched for a schedule: whole groups of 8 G ids
inline unsigned sched_blocks(const ColSched& s) {
  const long long unit = 8LL * s.G;
  const long long n = (long long)s.batch * s.ntiles_pad;
  return (unsigned)(((n + unit - 1) / unit) * unit);
}

// ---------------------------------------------------------------------------------------------
// per-column pieces of the axis-0 passes
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

__device__ __forceinline__ ColCoord col_coord(const Axis0Geom& gm, int g) {
  ColCoord cc;
  if (gm.ndim == 2) {
    cc.mx = g;
    cc.my = 0;
  } else {
    cc.my = (int)((unsigned)g / (unsigned)gm.nxh);
    cc.mx = g - cc.my * gm.nxh;
  }
  cc.nyq_x = (2 * cc.mx == gm.nx);
  cc.kx_c = cc.nyq_x ? -1.0f : (float)cc.mx * gm.kapx;
  cc.wm = (cc.mx == 0 || cc.nyq_x) ? 1.0f : 2.0f;
  cc.qx = (long long)cc.mx * gm.dfac_x;
  if (gm.ndim == 3) {
    const int mt = cc.my < gm.ny / 2 ? cc.my : cc.my - gm.ny;
    cc.nyq_y = (2 * cc.my == gm.ny);
    cc.ky = (float)mt * gm.kapy;
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

// symmetrised amplitude at axis-0 index e of column cc (Eq. (8) with Eqs. (12)-(13));
// also returns ln chi (unsymmetrised) for the support check.  GEN: the instantiation for launches
// where some field uses a tabulated radial form or the FP64 evaluation (uniform branches on the
// field's filter); the default one evaluates Eq. (13) in FP32 only.
template <int NDIM>
__device__ __forceinline__ float amp_sym64(const FiltDev& f, const Axis0Geom& gm, const ColCoord& cc, int e,
                                           float& lnc) {
  // the canonical wavenumbers in FP64: 2 m~ / n, -1 on a Nyquist index
  const int mt = e < gm.n0 / 2 ? e : e - gm.n0;
  const double k0c = (double)(2 * mt) / (double)gm.n0;
  const bool nyq0 = (2 * e == gm.n0);
  const double kx = cc.nyq_x ? -1.0 : (double)(2 * cc.mx) / (double)gm.nx;
  double ky, kz;
  bool ny_y;
  if constexpr (NDIM == 2) { ky = k0c; kz = 0.0; ny_y = nyq0; }
  else {
    const int my = cc.my < gm.ny / 2 ? cc.my : cc.my - gm.ny;
    ky = (double)(2 * my) / (double)gm.ny;
    kz = k0c;
    ny_y = cc.nyq_y;
  }
  const double l1 = ln_chi64<NDIM>(f, kx, ky, kz);
  lnc = l1 > -1.0e299 ? (float)l1 : -1.0e30f;
  float H = amp_from_lnchi64(l1, f.doffset);
  if (f.rotated && (cc.nyq_x || ny_y)) {
    const double l2 = ln_chi64<NDIM>(f, cc.nyq_x ? -kx : kx, ny_y ? -ky : ky, kz);
    H = (float)(0.5 * ((double)H + (double)amp_from_lnchi64(l2, f.doffset)));
  }
  return H;
}

// 3D: the x and y terms of the superellipse norm are fixed along an axis-0 column (the rotation is
// about z), so they are formed once per column: lxy = log2 max(u_x, u_y) and the sum of the in-plane
// terms relative to it, c01 = 1 + (min / max)^p (0 when u_x = u_y = 0).  Per mode only the z term
// joins them, relative to the largest of the three (Eq. (12), scaled form).
struct Col3 {
  float lxy, c01;
};
constexpr float COL3_OFF = -1.0e4f;   // log2 of a zero term: its power 2^(p (COL3_OFF - l)) is 0

__device__ __forceinline__ Col3 col3(const FiltDev& f, float kx, float ky) {
  const float kxr = fmaf(f.cr, kx, f.sr * ky);
  const float kyr = fmaf(-f.sr, kx, f.cr * ky);
  const float u0 = fabsf(kxr) * f.ia, u1 = fabsf(kyr) * f.ib;
  const float um = fmaxf(u0, u1), un = fminf(u0, u1);
  Col3 c;
  if (!(um > 0.0f)) {
    c.lxy = COL3_OFF;
    c.c01 = 0.0f;
    return c;
  }
  c.lxy = hw_log2(um);
  c.c01 = 1.0f + (un > 0.0f ? hw_exp2(f.p * (hw_log2(un) - c.lxy)) : 0.0f);
  return c;
}

// ln chi (relative to its peak) at (column c, kappa_z): Eq. (13) with band centre k0, or the
// tabulated radial form (PROF); -1e30 at the DC mode
template <bool PROF>
__device__ __forceinline__ float ln_chi3(const FiltDev& f, const Col3& c, float kz) {
  const float u2 = fabsf(kz) * f.ic;
  const bool on2 = u2 > 0.0f;
  if (!on2 && !(c.c01 > 0.0f)) return -1.0e30f;
  const float l2 = on2 ? hw_log2(u2) : COL3_OFF;
  const bool zbig = l2 > c.lxy;
  const float lm = zbig ? l2 : c.lxy;
  const float t = hw_exp2(-f.p * fabsf(l2 - c.lxy));      // the smaller side relative to the larger
  const float S = zbig ? fmaf(c.c01, t, 1.0f) : c.c01 + (on2 ? t : 0.0f);
  const float log2K = fmaf(hw_log2(S), f.ip, lm);
  const float K = hw_exp2(log2K);
  if constexpr (PROF) {
    if (f.prof) return prof_lnchi(f, K);
  }
  const float d = K - f.k0;
  return fmaf(f.alpha, log2K * 0.69314718055994531f, -fmaf(d * d, f.inv2w2, f.lnchimax));
}

// the symmetrised amplitude of a 3D mode from its column's terms (c2: the column with its Nyquist
// x / y components negated, used on those planes when the filter is rotated); kappa_z enters only
// through |kappa_z|, so the z Nyquist plane needs no partner
template <bool GEN>
__device__ __forceinline__ float amp_sym3(const FiltDev& f, const Axis0Geom& gm, const ColCoord& cc, const Col3& c1,
                                          const Col3& c2, int e, float& lnc) {
  if constexpr (GEN) {
    if (f.prec64) return amp_sym64<3>(f, gm, cc, e, lnc);
  }
  const float kz = (float)(e < gm.n0 / 2 ? e : e - gm.n0) * gm.kap0;
  lnc = ln_chi3<GEN>(f, c1, kz);
  float H = amp_from_lnchi(lnc, f.offset);
  if (f.rotated && (cc.nyq_x || cc.nyq_y)) H = 0.5f * (H + amp_from_lnchi(ln_chi3<GEN>(f, c2, kz), f.offset));
  return H;
}

template <int NDIM, bool GEN = false>
__device__ __forceinline__ float amp_sym(const FiltDev& f, const Axis0Geom& gm, const ColCoord& cc, int e,
                                         float& lnc) {
  if constexpr (GEN) {
    if (f.prec64) return amp_sym64<NDIM>(f, gm, cc, e, lnc);
  }
  constexpr bool PROF = GEN;
  const int mt = e < gm.n0 / 2 ? e : e - gm.n0;
  const float k0c = (float)mt * gm.kap0;         // canonical kappa along axis 0 (-1 at Nyquist)
  const bool nyq0 = (2 * e == gm.n0);
  float kx = cc.kx_c, ky, kz;
  bool ny_y;
  if constexpr (NDIM == 2) { ky = k0c; kz = 0.0f; ny_y = nyq0; }
  else { ky = cc.ky; kz = k0c; ny_y = cc.nyq_y; }
  lnc = ln_chi<NDIM, PROF>(f, kx, ky, kz);
  float H = amp_from_lnchi(lnc, f.offset);
  if (f.rotated && (cc.nyq_x || ny_y)) {
    // partner -m: by evenness, the canonical kappa with its Nyquist components negated
    const float kx2 = cc.nyq_x ? -kx : kx, ky2 = ny_y ? -ky : ky;
    const float l2 = ln_chi<NDIM, PROF>(f, kx2, ky2, kz);
    H = 0.5f * (H + amp_from_lnchi(l2, f.offset));
  }
  return H;
}

// ---------------------------------------------------------------------------------------------
// Deterministic binning of one tile.  The per-mode power values w |X|^2 of the tile's C columns sit
// in LDS (padded layout pw_index).  Thread (column cb, segment pb) takes the E consecutive modes
// e = pb E .. pb E + E - 1 of its column, reads their tile-local bins j (the position of the mode's
// bin in the tile's ascending list of distinct bins, from the per-geometry table ltab) and sums
// each run of equal j in FP64 in mode order.  The runs of one bin are combined in integer
// arithmetic, which does not depend on the order in which the atomics land:
//   pass 1: hx[j] = the largest binary exponent of the bin's runs (integer maximum);
//   pass 2: hq[j] += each run rounded to a multiple of 2^(hx[j] - 48), as an unsigned integer.
// A run is below 2^hx[j], so it contributes less than 2^48 units, and a bin of one tile gathers
// at most T E <= 2^15 runs: the sum stays below 2^63.  The tile's partial of bin j is then
// hq[j] 2^(hx[j] - 48), the same bits for every schedule of the workgroup; its error is at most
// 2^-48 of the bin's largest run per run.
// ---------------------------------------------------------------------------------------------
constexpr int HX_EMPTY = -100000;
constexpr int HQ_SHIFT = 48;

__device__ __forceinline__ unsigned long long run_to_fixed(double s, int emax) {
  const double x = ldexp(s, HQ_SHIFT - emax);               // in [0, 2^48)
  const double y = x + 4503599627370496.0;                  // + 2^52: the low mantissa bits hold rint(x)
  return (unsigned long long)__double_as_longlong(y) - 0x4330000000000000ull;
}

template <bool PASS2>
__device__ __forceinline__ void run_commit(int j, double s, int* hx, unsigned long long* hq) {
  if (!(s > 0.0)) return;
  if constexpr (!PASS2) atomicMax(hx + j, __builtin_amdgcn_frexp_exp(s));
  else atomicAdd(hq + j, run_to_fixed(s, hx[j]));
}

template <int E, bool PASS2>
__device__ __forceinline__ void runs_commit(const int (&loc)[E], const float (&v)[E], int* hx,
                                            unsigned long long* hq) {
  int cur = loc[0];
  double acc = (double)v[0];
#pragma unroll
  for (int i = 1; i < E; ++i) {
    if (loc[i] != cur) {
      run_commit<PASS2>(cur, acc, hx, hq);
      cur = loc[i];
      acc = 0.0;
    }
    acc += (double)v[i];
  }
  run_commit<PASS2>(cur, acc, hx, hq);
}

// the E tile-local bins and power values of binning thread (cb, pb), all loads issued first
template <int L, int E>
__device__ __forceinline__ void seg_read(const float* pwc, const uint16_t* __restrict__ ltab, int g, int pb,
                                         int (&loc)[E], float (&v)[E]) {
  const int e0 = pb * E;
  const uint16_t* t = ltab + (unsigned)(g * L + e0);
  if constexpr ((L % 8) == 0 && (E % 8) == 0) {
    uint4 w[E / 8];
#pragma unroll
    for (int q = 0; q < E / 8; ++q) w[q] = *reinterpret_cast<const uint4*>(t + 8 * q);
#pragma unroll
    for (int q = 0; q < E / 8; ++q) {
      const uint32_t ws[4] = {w[q].x, w[q].y, w[q].z, w[q].w};
#pragma unroll
      for (int h = 0; h < 8; ++h) loc[8 * q + h] = (int)((ws[h >> 1] >> (16 * (h & 1))) & 0xFFFFu);
    }
  } else {
#pragma unroll
    for (int i = 0; i < E; ++i) loc[i] = (int)t[i];
  }
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = pwc[pw_index(e0 + i)];
}

// Radial bins only (sym): the bin of a mode depends on the axis-0 index e only through its square,
// so e and n0 - e share it.  Thread (cb, pb) then takes the pairs q = pb E/2 .. pb E/2 + E/2 - 1 of
// its column with the value pw[q] + pw[n0 - q] (pw[q] alone for q = 0), the last thread also
// q = n0 / 2 (its own partner): half the runs.  Other threads carry an empty last entry.
template <int L, int E, int P>
__device__ __forceinline__ void seg_read_sym(const float* pwc, const uint16_t* __restrict__ ltab, int g, int pb,
                                             int (&loc)[E / 2 + 1], double (&v)[E / 2 + 1]) {
  constexpr int H = E / 2;
  const int q0 = pb * H;
  const uint16_t* t = ltab + (unsigned)(g * L);
#pragma unroll
  for (int i = 0; i < H; ++i) loc[i] = (int)t[q0 + i];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const int q = q0 + i;
    v[i] = q == 0 ? (double)pwc[pw_index(0)] : (double)pwc[pw_index(q)] + (double)pwc[pw_index(L - q)];
  }
  const bool nyq = pb == P - 1;
  loc[H] = nyq ? (int)t[L / 2] : loc[H - 1];
  v[H] = nyq ? (double)pwc[pw_index(L / 2)] : 0.0;
}

template <int N, bool PASS2>
__device__ __forceinline__ void runs_commit_d(const int (&loc)[N], const double (&v)[N], int* hx,
                                              unsigned long long* hq) {
  int cur = loc[0];
  double acc = v[0];
#pragma unroll
  for (int i = 1; i < N; ++i) {
    if (loc[i] != cur) {
      run_commit<PASS2>(cur, acc, hx, hq);
      cur = loc[i];
      acc = 0.0;
    }
    acc += v[i];
  }
  run_commit<PASS2>(cur, acc, hx, hq);
}

// The whole tile: both passes and the stores of the partials (thread j < nloc stores the partial of
// local bin j at its position wpos[toff[tile] + j] and clears its slots for the next tile).  Called
// by every thread of the workgroup after the power values are in LDS and a barrier; ends with the
// LDS histogram cleared, without a final barrier.
template <int L, int E, int C, int LP, int T>
__device__ __forceinline__ void tile_bins(const float* pw, int* hx, unsigned long long* hq, const TileBinDev& tb,
                                          int tile, int ncol, double* __restrict__ out, int tid) {
  constexpr int P = Plan<L>::P;
  const int cb = tid / P, pb = tid - cb * P;
  const int g = tile * C + cb;
  const bool act = cb < C && g < ncol;
  // the tile's partial range and store positions first: their loads overlap the two passes
  const unsigned j0 = tb.toff[tile];
  const int nloc = (int)(tb.toff[tile + 1] - j0);
  const unsigned wp0 = tid < nloc ? tb.wpos[j0 + tid] : 0u;
  if (tb.sym) {                                      // uniform over the launch
    static_assert(E % 2 == 0, "pairs of modes split a thread's E modes in halves");
    int loc[E / 2 + 1];
    double v[E / 2 + 1];
    if (act) {
      seg_read_sym<L, E, P>(pw + cb * LP, tb.ltab, g, pb, loc, v);
      runs_commit_d<E / 2 + 1, false>(loc, v, hx, hq);
    }
    __syncthreads();
    if (act) runs_commit_d<E / 2 + 1, true>(loc, v, hx, hq);
    __syncthreads();
  } else {
    int loc[E];
    float v[E];
    if (act) {
      seg_read<L, E>(pw + cb * LP, tb.ltab, g, pb, loc, v);
      runs_commit<E, false>(loc, v, hx, hq);
    }
    __syncthreads();
    if (act) runs_commit<E, true>(loc, v, hx, hq);
    __syncthreads();
  }
  for (int j = tid; j < nloc; j += T) {
    const int e = hx[j];
    const unsigned long long q = hq[j];
    out[j == tid ? wp0 : tb.wpos[j0 + j]] = e == HX_EMPTY ? 0.0 : ldexp((double)q, e - HQ_SHIFT);
    hx[j] = HX_EMPTY;
    hq[j] = 0ull;
  }
}

template <int L, int V, bool SPLIT = false>
__host__ __device__ constexpr size_t col_xchg_bytes() {
  return SPLIT ? (size_t)ColTile<L, V>::C * ColTile<L, V>::RSH * 4 : (size_t)ColTile<L, V>::C * ColTile<L, V>::RS * 8;
}

// LDS of an axis-0 pass that bins: the exchange buffer (the power values reuse it), then the tile
// histogram (nloc_max exponents and fixed-point sums)
template <int L, int V, bool SPLIT = false>
__host__ __device__ constexpr size_t col_bin_base() {
  return ((col_xchg_bytes<L, V, SPLIT>() > (size_t)ColTile<L, V>::C * ColTile<L, V>::LP * 4
               ? col_xchg_bytes<L, V, SPLIT>()
               : (size_t)ColTile<L, V>::C * ColTile<L, V>::LP * 4) + 15) / 16 * 16;
}

// the exchange region of column c of a tile: complex, or floats for the split exchange
template <int L, int V, bool SPLIT>
__device__ __forceinline__ auto col_region(float2* lds, int c) {
  if constexpr (SPLIT) return reinterpret_cast<float*>(lds) + c * ColTile<L, V>::RSH;
  else return lds + c * ColTile<L, V>::RS;
}

// ---------------------------------------------------------------------------------------------
// Global I/O through buffer resources: a 128-bit descriptor (base, size in bytes) in scalar
// registers, a per-thread byte offset in one vector register and a uniform per-slot byte offset
// in a scalar register, so the slots of a transform cost no vector address arithmetic.  Loads
// beyond the size return 0 and stores beyond it are dropped.
// ---------------------------------------------------------------------------------------------
using rsrc_t = __amdgpu_buffer_rsrc_t;
using u32x2 = __attribute__((ext_vector_type(2))) unsigned int;
using u32x4 = __attribute__((ext_vector_type(4))) unsigned int;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float2 buf_load2(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ u32x4 buf_load4(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
}
__device__ __forceinline__ void buf_store2(rsrc_t r, float2 v, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_store4(rsrc_t r, u32x4 v, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, soff, 0);
}

// Column g of a column pass over one field's half spectrum: element e sits at
// (g / inner) L inner + g mod inner + e inner -- in 2D (column groups of four, inner = 4) element
// (e, g) at ((g >> 2) L + e) 4 + (g & 3), in 3D axis 0 (inner = ncol) at e ncol + g, in the 3D y
// pass (inner = n_x / 2 + 1, g = z inner + m_x) within its z-plane.  Thread p of the column
// addresses element p + o at voff + o * step.
struct ColIO {
  rsrc_t r;
  unsigned voff;   // bytes, this thread's first element
  unsigned step;   // bytes per element along axis 0 (uniform)
};

template <int L>
__device__ __forceinline__ ColIO col_io(const float2* field_spec, long long nh, int inner, int g, int p) {
  ColIO io;
  io.r = make_rsrc(field_spec, (unsigned)(nh * 8));
  const unsigned go = (unsigned)g / (unsigned)inner;
  const unsigned col = go * (unsigned)(L * inner) + ((unsigned)g - go * (unsigned)inner);
  io.voff = (col + (unsigned)p * (unsigned)inner) * 8u;
  io.step = (unsigned)inner * 8u;
  return io;
}

// the E slots of a transform whose first (load) or last (store) radix is R
template <int L, int R, int P, int E>
__device__ __forceinline__ void col_load(float2 (&v)[E], const ColIO& io) {
#pragma unroll
  for (int s = 0; s < E; ++s) v[s] = buf_load2(io.r, io.voff, (unsigned)slot_index<L, R, P>(s, 0) * io.step);
}
template <int L, int R, int P, int E>
__device__ __forceinline__ void col_store(const float2 (&v)[E], const ColIO& io) {
#pragma unroll
  for (int s = 0; s < E; ++s) buf_store2(io.r, v[s], io.voff, (unsigned)slot_index<L, R, P>(s, 0) * io.step);
}

// per-field parameter and output accessors: the batch table when present, else the uniform
// arguments (base pointer + field * stride)
template <class T>
__device__ __forceinline__ T* field_ptr(T* base, long long stride, int b) {
  return base ? base + (long long)b * stride : nullptr;
}

}  // namespace hu
