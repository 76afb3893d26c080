// Device building blocks for the hyperuniform-field kernels (gfx950, wave64).
//
//  * complex helpers and radix-2/3/4/8/16 DFTs held in registers;
//  * Stockham autosort stages: butterfly j reads elements j + r L/R, applies the twiddles
//    exp(-+ 2 pi i r (j mod Ns) / (Ns R)), and writes (j / Ns) Ns R + (j mod Ns) + r Ns, so the last
//    stage leaves the transform in natural order in the same j + r L/R register pattern the
//    first stage reads; stages exchange through LDS;
//  * Philox4x32-10 (Salmon et al., SC'11) and Box-Muller for the white noise;
//  * the superellipse filter amplitude of Eqs. (12)-(13) (with band centre k0) in FP32;
//  * the exact integer radial / FP64 angular bin index.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace hu {

// ---------------------------------------------------------------------------------------------
// complex arithmetic on float2
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// The library is built without automatic multiply-add contraction, so that every instantiation
// of a formula rounds the same way; the fused forms used are written out.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// multiply by exp(-+ i 2 pi m / 16) for the compile-time m
template <int M, bool INV>
__device__ __forceinline__ float2 mul_w16(float2 a) {
  constexpr double PI = 3.14159265358979323846;
  constexpr int m = M % 16;
  if constexpr (m == 0) return a;
  if constexpr (m == 4) return mul_mi<INV>(a);
  if constexpr (m == 8) return make_float2(-a.x, -a.y);
  if constexpr (m == 12) return mul_mi<!INV>(a);
  // generic constant twiddle; the constants are FP64 expressions rounded once to FP32
  constexpr float c = (float)(m == 1 ? 0.92387953251128675613 : m == 2 ? 0.70710678118654752440
                              : m == 3 ? 0.38268343236508977173 : m == 5 ? -0.38268343236508977173
                              : m == 6 ? -0.70710678118654752440 : m == 7 ? -0.92387953251128675613
                              : m == 9 ? -0.92387953251128675613 : m == 10 ? -0.70710678118654752440
                              : m == 11 ? -0.38268343236508977173 : m == 13 ? 0.38268343236508977173
                              : m == 14 ? 0.70710678118654752440 : 0.92387953251128675613);
  constexpr float s = (float)(m == 1 ? 0.38268343236508977173 : m == 2 ? 0.70710678118654752440
                              : m == 3 ? 0.92387953251128675613 : m == 5 ? 0.92387953251128675613
                              : m == 6 ? 0.70710678118654752440 : m == 7 ? 0.38268343236508977173
                              : m == 9 ? -0.38268343236508977173 : m == 10 ? -0.70710678118654752440
                              : m == 11 ? -0.92387953251128675613 : m == 13 ? -0.92387953251128675613
                              : m == 14 ? -0.70710678118654752440 : -0.38268343236508977173);
  (void)PI;
  // forward: exp(-i t) = (c, -s); inverse: (c, +s), with (c, s) = (cos t, sin t)
  const float sy = INV ? s : -s;
  return make_float2(fmaf(a.x, c, -(a.y * sy)), fmaf(a.x, sy, a.y * c));
}

// ---------------------------------------------------------------------------------------------
// small DFTs in registers, natural order in and out
// ---------------------------------------------------------------------------------------------
template <bool INV>
__device__ __forceinline__ void dft2(float2& a0, float2& a1) {
  float2 t = a0;
  a0 = cadd(t, a1);
  a1 = csub(t, a1);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  float2 t2 = cadd(a1, a3), t3 = mul_mi<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2& a0, float2& a1, float2& a2) {
  const float h = 0.86602540378443864676f;  // sqrt(3)/2
  float2 t = cadd(a1, a2), u = csub(a1, a2);
  float2 m = make_float2(fmaf(-0.5f, t.x, a0.x), fmaf(-0.5f, t.y, a0.y));
  float2 v = cscale(mul_mi<INV>(u), h);
  a0 = cadd(a0, t);
  a1 = cadd(m, v);
  a2 = csub(m, v);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* a) {
  // even / odd split: E = DFT4(a0,a2,a4,a6), O = DFT4(a1,a3,a5,a7), X_k = E_k + w8^k O_k
  float2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  float2 o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  o1 = mul_w16<2, INV>(o1);
  o2 = mul_w16<4, INV>(o2);
  o3 = mul_w16<6, INV>(o3);
  a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1); a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2); a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3); a[7] = csub(e3, o3);
}

template <bool INV>
__device__ __forceinline__ void dft16(float2* a) {
  // 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
  float2 y[16];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    float2 b0 = a[n2], b1 = a[4 + n2], b2 = a[8 + n2], b3 = a[12 + n2];
    dft4<INV>(b0, b1, b2, b3);
    y[n2 * 4 + 0] = b0; y[n2 * 4 + 1] = b1; y[n2 * 4 + 2] = b2; y[n2 * 4 + 3] = b3;
  }
  // twiddles w16^(n2 k1)
  y[1 * 4 + 1] = mul_w16<1, INV>(y[1 * 4 + 1]);
  y[1 * 4 + 2] = mul_w16<2, INV>(y[1 * 4 + 2]);
  y[1 * 4 + 3] = mul_w16<3, INV>(y[1 * 4 + 3]);
  y[2 * 4 + 1] = mul_w16<2, INV>(y[2 * 4 + 1]);
  y[2 * 4 + 2] = mul_w16<4, INV>(y[2 * 4 + 2]);
  y[2 * 4 + 3] = mul_w16<6, INV>(y[2 * 4 + 3]);
  y[3 * 4 + 1] = mul_w16<3, INV>(y[3 * 4 + 1]);
  y[3 * 4 + 2] = mul_w16<6, INV>(y[3 * 4 + 2]);
  y[3 * 4 + 3] = mul_w16<9, INV>(y[3 * 4 + 3]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 b0 = y[0 * 4 + k1], b1 = y[1 * 4 + k1], b2 = y[2 * 4 + k1], b3 = y[3 * 4 + k1];
    dft4<INV>(b0, b1, b2, b3);
    a[k1] = b0; a[k1 + 4] = b1; a[k1 + 8] = b2; a[k1 + 12] = b3;
  }
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2* a) {
  if constexpr (R == 2) dft2<INV>(a[0], a[1]);
  else if constexpr (R == 3) dft3<INV>(a[0], a[1], a[2]);
  else if constexpr (R == 4) dft4<INV>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 8) dft8<INV>(a);
  else if constexpr (R == 16) dft16<INV>(a);
  else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------------------------
// Stockham plans.  Plan<L>: E elements per thread, P = L / E threads per transform, radix list
// fwd (first radix first) and its reverse.  Every radix divides E.  Plan<L, 1>: an alternative
// order of radices with the same E (so the same tile shapes), chosen per shape class by the
// autotuner; lengths without one (alt false) keep their default list under either choice.
// ---------------------------------------------------------------------------------------------
template <int... Rs>
struct Radices {};

template <int... Rs>
struct RadProd;
template <>
struct RadProd<> { static constexpr int value = 1; };
template <int R0, int... Rs>
struct RadProd<R0, Rs...> { static constexpr int value = R0 * RadProd<Rs...>::value; };
template <int E, int... Rs>
struct RadDivE { static constexpr bool value = ((E % Rs == 0) && ...); };

template <int L, int RV = 0>
struct Plan;
#define HU_PLAN(LEN, EPT, ...)                                                               \
  template <>                                                                                \
  struct Plan<LEN, 0> {                                                                      \
    static constexpr int E = EPT;                                                            \
    static constexpr int P = LEN / EPT;                                                      \
    static constexpr bool alt = false;                                                       \
    using fwd = Radices<__VA_ARGS__>;                                                        \
    static_assert(RadProd<__VA_ARGS__>::value == LEN && RadDivE<EPT, __VA_ARGS__>::value, \
                  "radices multiply to the length and divide E");                           \
  };
HU_PLAN(2, 2, 2)
HU_PLAN(3, 3, 3)
HU_PLAN(4, 4, 4)
HU_PLAN(6, 6, 3, 2)
HU_PLAN(8, 8, 8)
HU_PLAN(12, 12, 3, 4)
HU_PLAN(16, 16, 16)
HU_PLAN(24, 24, 3, 8)
HU_PLAN(32, 16, 8, 4)
HU_PLAN(48, 12, 3, 4, 4)
HU_PLAN(64, 16, 16, 4)
HU_PLAN(96, 24, 3, 4, 8)
HU_PLAN(128, 16, 16, 8)
HU_PLAN(192, 24, 3, 8, 8)
HU_PLAN(256, 16, 16, 16)
HU_PLAN(384, 24, 3, 8, 8, 2)
HU_PLAN(512, 16, 8, 8, 8)
HU_PLAN(768, 24, 3, 8, 8, 4)
HU_PLAN(1024, 16, 16, 8, 8)
HU_PLAN(1536, 24, 3, 8, 8, 8)
HU_PLAN(2048, 16, 16, 8, 16)
#undef HU_PLAN

template <int L>
struct Plan<L, 1> : Plan<L, 0> {};
#define HU_ALT_PLAN(LEN, ...)                                                                  \
  template <>                                                                                  \
  struct Plan<LEN, 1> {                                                                        \
    static constexpr int E = Plan<LEN, 0>::E;                                                  \
    static constexpr int P = Plan<LEN, 0>::P;                                                  \
    static constexpr bool alt = true;                                                          \
    using fwd = Radices<__VA_ARGS__>;                                                          \
    static_assert(RadProd<__VA_ARGS__>::value == LEN && RadDivE<E, __VA_ARGS__>::value,     \
                  "radices multiply to the length and divide E");                             \
  };
HU_ALT_PLAN(256, 16, 4, 4)
HU_ALT_PLAN(512, 16, 8, 4)
HU_ALT_PLAN(1024, 8, 8, 16)
HU_ALT_PLAN(2048, 16, 16, 8)
#undef HU_ALT_PLAN

// the radix choice a kernel of length L runs under the requested one (0 where L has no alternative)
template <int L>
constexpr int radix_choice(int rv) { return rv && Plan<L, 1>::alt ? 1 : 0; }

template <int R0, int... Rs>
struct FirstR { static constexpr int value = R0; };
template <int R0, int... Rs>
struct LastR { static constexpr int value = LastR<Rs...>::value; };
template <int R0>
struct LastR<R0> { static constexpr int value = R0; };

template <typename A, typename B>
struct RevImpl;
template <int... Done>
struct RevImpl<Radices<>, Radices<Done...>> { using type = Radices<Done...>; };
template <int R0, int... Rs, int... Done>
struct RevImpl<Radices<R0, Rs...>, Radices<Done...>> {
  using type = typename RevImpl<Radices<Rs...>, Radices<R0, Done...>>::type;
};
template <typename A>
using Reverse = typename RevImpl<A, Radices<>>::type;

template <typename A>
struct RadInfo;
template <int... Rs>
struct RadInfo<Radices<Rs...>> {
  static constexpr int first = FirstR<Rs...>::value;
  static constexpr int last = LastR<Rs...>::value;
};

// ---------------------------------------------------------------------------------------------
// Stage twiddle rows.  Stage i >= 1 of a radix list (R_0, R_1, ...) with NS_i = R_0 ... R_{i-1}
// multiplies input r of butterfly j by exp(-+ 2 pi i r k / (NS_i R_i)), k = j mod NS_i.  Its rows
// k = 0 .. NS_i - 1 hold rpad(R_i) consecutive complex entries (r = 0 .. rpad - 1, R rounded up to
// even so that every row starts on 16 bytes), so one butterfly reads one row with 16-byte loads
// from a single offset.  The table of a length L holds the rows of the forward radix list, then
// those of its reverse (the plan of the inverse transforms); the first stage needs none.
// ---------------------------------------------------------------------------------------------
__host__ __device__ constexpr int rpad(int R) { return (R + 1) / 2 * 2; }

template <int NS, int... Rs>
struct TabSize;
template <int NS>
struct TabSize<NS> { static constexpr int value = 0; };
template <int NS, int R, int... Rest>
struct TabSize<NS, R, Rest...> {
  static constexpr int value = (NS > 1 ? NS * rpad(R) : 0) + TabSize<NS * R, Rest...>::value;
};
template <typename A>
struct PlanTab;
template <int... Rs>
struct PlanTab<Radices<Rs...>> { static constexpr int size = TabSize<1, Rs...>::value; };

// complex entries of the stage table of length L under radix choice RV (forward rows, then
// reversed-plan rows)
template <int L, int RV = 0>
struct StageTab {
  using F = typename Plan<L, RV>::fwd;
  static constexpr int fwd = PlanTab<F>::size;
  static constexpr int total = fwd + PlanTab<Reverse<F>>::size;
};

// One Stockham stage on the registers of thread p: butterflies j = p + P b, b < E/R; the stage's
// twiddle rows start at entry SOFF of the table.
template <int L, int R, int NS, int P, int E, bool INV, int SOFF>
__device__ __forceinline__ void stage_compute(float2 (&v)[E], int p, const float2* __restrict__ tw) {
#pragma unroll
  for (int b = 0; b < E / R; ++b) {
    if constexpr (NS > 1) {
      const int j = p + P * b;
      const unsigned k = (unsigned)(j % NS);
      const float4* row = reinterpret_cast<const float4*>(tw) + (unsigned)(SOFF / 2) + k * (unsigned)(rpad(R) / 2);
#pragma unroll
      for (int q = 0; q < rpad(R) / 2; ++q) {
        const float4 w2 = row[q];
        if (2 * q >= 1 && 2 * q < R) {
          const float2 w = make_float2(w2.x, INV ? -w2.y : w2.y);
          v[b * R + 2 * q] = cmul(v[b * R + 2 * q], w);
        }
        if (2 * q + 1 < R) {
          const float2 w = make_float2(w2.z, INV ? -w2.w : w2.w);
          v[b * R + 2 * q + 1] = cmul(v[b * R + 2 * q + 1], w);
        }
      }
    }
    dft<R, INV>(&v[b * R]);
  }
}

// LDS layout of an exchange region: one padding element after every 16, so that the strided
// stores of the early Stockham stages (stride R complex) fall on distinct banks.
__host__ __device__ constexpr int lidx(int i) { return i + (i >> 4); }
// complex elements per exchange region of a length-L transform (padding plus 8 so that
// neighbouring regions start on different banks)
template <int L>
struct Region {
  static constexpr int value = L + (L >> 4) + 8;
};
// the same rounded up to a multiple of 16 plus 1: for tiles of many transforms whose lanes in a
// wave belong to different transforms, consecutive regions then start on different banks
template <int L>
struct RegionWide {
  static constexpr int value = (L + (L >> 4) + 15) / 16 * 16 + 1;
};

// LDS positions of a stage's reads (element j + r L/R, j = p + P b) and writes (element
// (j / NS) NS R + j mod NS + r NS).  When the padded position minus that of the thread's first
// element is the same for every thread p, the stage addresses LDS from one per-thread base with
// constant offsets (`lin`); this is checked at compile time over every p.
template <int L, int R, int P, int E>
struct LoadMap {
  static constexpr int off(int p, int b, int r) { return lidx(p + P * b + r * (L / R)) - lidx(p); }
  static constexpr bool check() {
    for (int p = 0; p < P; ++p)
      for (int b = 0; b < E / R; ++b)
        for (int r = 0; r < R; ++r)
          if (off(p, b, r) != off(0, b, r)) return false;
    return true;
  }
  static constexpr bool lin = check();
};

template <int R, int NS, int P, int E>
struct StoreMap {
  static constexpr int base(int j) { return (j / NS) * NS * R + (j % NS); }
  static constexpr int off(int p, int b, int r) { return lidx(base(p + P * b) + r * NS) - lidx(base(p)); }
  static constexpr bool check() {
    for (int p = 0; p < P; ++p)
      for (int b = 0; b < E / R; ++b)
        for (int r = 0; r < R; ++r)
          if (off(p, b, r) != off(0, b, r)) return false;
    return true;
  }
  static constexpr bool lin = check();
};

template <int L, int R, int NS, int P, int E>
__device__ __forceinline__ void stage_store(const float2 (&v)[E], float2* lds, int p) {
  using M = StoreMap<R, NS, P, E>;
  if constexpr (M::lin) {
    float2* sp = lds + lidx(M::base(p));
#pragma unroll
    for (int b = 0; b < E / R; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) sp[M::off(0, b, r)] = v[b * R + r];
  } else {
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
      const int base = M::base(p + P * b);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lidx(base + r * NS)] = v[b * R + r];
    }
  }
}

// element j + r L/R of slot b R + r (the read pattern of a stage, and the natural-order pattern a
// transform starts from or ends in)
template <int L, int R, int P, int E>
__device__ __forceinline__ void stage_load(float2 (&v)[E], const float2* lds, int p) {
  using M = LoadMap<L, R, P, E>;
  if constexpr (M::lin) {
    const float2* lp = lds + lidx(p);
#pragma unroll
    for (int b = 0; b < E / R; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) v[b * R + r] = lp[M::off(0, b, r)];
  } else {
#pragma unroll
    for (int b = 0; b < E / R; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) v[b * R + r] = lds[lidx(p + P * b + r * (L / R))];
  }
}

// Split exchange: the same positions in a region of floats, one component (COMP 0: real, 1:
// imaginary) per round, so the region takes half the LDS of a complex one.
template <int COMP>
__device__ __forceinline__ float& part(float2& a) { return COMP ? a.y : a.x; }
template <int COMP>
__device__ __forceinline__ float part(const float2& a) { return COMP ? a.y : a.x; }

template <int L, int R, int NS, int P, int E, int COMP>
__device__ __forceinline__ void stage_store(const float2 (&v)[E], float* lds, int p) {
  using M = StoreMap<R, NS, P, E>;
  if constexpr (M::lin) {
    float* sp = lds + lidx(M::base(p));
#pragma unroll
    for (int b = 0; b < E / R; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) sp[M::off(0, b, r)] = part<COMP>(v[b * R + r]);
  } else {
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
      const int base = M::base(p + P * b);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lidx(base + r * NS)] = part<COMP>(v[b * R + r]);
    }
  }
}

template <int L, int R, int P, int E, int COMP>
__device__ __forceinline__ void stage_load(float2 (&v)[E], const float* lds, int p) {
  using M = LoadMap<L, R, P, E>;
  if constexpr (M::lin) {
    const float* lp = lds + lidx(p);
#pragma unroll
    for (int b = 0; b < E / R; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) part<COMP>(v[b * R + r]) = lp[M::off(0, b, r)];
  } else {
#pragma unroll
    for (int b = 0; b < E / R; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) part<COMP>(v[b * R + r]) = lds[lidx(p + P * b + r * (L / R))];
  }
}

// In-place exchange through a strided column: element i of the transform at float2 index i * S
// of the base (a column of a matrix held row by row in LDS, the column's own storage serving as
// its exchange region).
template <int S>
struct Strided {
  float2 v;
};

template <int L, int R, int NS, int P, int E, int S>
__device__ __forceinline__ void stage_store(const float2 (&v)[E], Strided<S>* lds, int p) {
  float2* base = reinterpret_cast<float2*>(lds);
#pragma unroll
  for (int b = 0; b < E / R; ++b) {
    const int j0 = StoreMap<R, NS, P, E>::base(p + P * b);
#pragma unroll
    for (int r = 0; r < R; ++r) base[(j0 + r * NS) * S] = v[b * R + r];
  }
}

template <int L, int R, int P, int E, int S>
__device__ __forceinline__ void stage_load(float2 (&v)[E], const Strided<S>* lds, int p) {
  const float2* base = reinterpret_cast<const float2*>(lds);
#pragma unroll
  for (int b = 0; b < E / R; ++b)
#pragma unroll
    for (int r = 0; r < R; ++r) v[b * R + r] = base[(p + P * b + r * (L / R)) * S];
}

template <int L, int R, int P, int E>
__device__ __forceinline__ void slot_store(const float2 (&v)[E], float2* lds, int p) {
  using M = LoadMap<L, R, P, E>;
  if constexpr (M::lin) {
    float2* lp = lds + lidx(p);
#pragma unroll
    for (int b = 0; b < E / R; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) lp[M::off(0, b, r)] = v[b * R + r];
  } else {
#pragma unroll
    for (int b = 0; b < E / R; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lidx(p + P * b + r * (L / R))] = v[b * R + r];
  }
}

// Element index held in register slot i for a transform whose first / last stage has radix R.
template <int L, int R, int P>
__device__ __forceinline__ int slot_index(int i, int p) {
  return p + P * (i / R) + (i % R) * (L / R);
}

// Exchange synchronisation.  A transform whose P threads all sit in one wave and own its LDS
// region needs no workgroup barrier: the LDS operations of a wave complete in issue order, so a
// wave-scope fence (which also keeps the compiler from moving LDS accesses across it) suffices.
template <bool WAVE>
__device__ __forceinline__ void xchg_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// X = float2: one complex exchange per stage; X = float: the split exchange, real parts then
// imaginary parts through the same float region (two more barriers, half the LDS).
template <class X, int L, int P, int E, bool INV, bool WAVE, int NS, int SOFF, int R, int... Rest>
__device__ __forceinline__ void fft_stages(float2 (&v)[E], X* lds, int p, const float2* __restrict__ tw) {
  stage_compute<L, R, NS, P, E, INV, SOFF>(v, p, tw);
  if constexpr (sizeof...(Rest) > 0) {
    constexpr int R2 = FirstR<Rest...>::value;
    if constexpr (std::is_same<X, float>::value) {
      xchg_sync<WAVE>();
      stage_store<L, R, NS, P, E, 0>(v, lds, p);
      xchg_sync<WAVE>();
      stage_load<L, R2, P, E, 0>(v, lds, p);
      xchg_sync<WAVE>();
      stage_store<L, R, NS, P, E, 1>(v, lds, p);
      xchg_sync<WAVE>();
      stage_load<L, R2, P, E, 1>(v, lds, p);
    } else {
      xchg_sync<WAVE>();
      stage_store<L, R, NS, P, E>(v, lds, p);
      xchg_sync<WAVE>();
      stage_load<L, R2, P, E>(v, lds, p);
    }
    fft_stages<X, L, P, E, INV, WAVE, NS * R, (NS > 1 ? SOFF + NS * rpad(R) : SOFF), Rest...>(v, lds, p, tw);
  }
}

// The transform with radix list Rs (the forward list of Plan<L, RV> or its reverse); tw = the
// stage table of L under radix choice RV, whose reversed-plan rows follow the forward rows.  A
// list that reads the same both ways uses the forward rows for both directions (they are the same
// rows).  WAVE: the P threads of each transform lie in one wave and the region `lds` is theirs
// alone (row passes with P dividing 64), so the exchanges synchronise the wave only.  `lds` is a
// complex region (X = float2), for the split exchange a float region of the same positions, or a
// strided column exchanged in place (X = Strided<S>).
template <int L, int P, int E, bool INV, bool WAVE = false, int RV = 0, class X = float2, int... Rs>
__device__ __forceinline__ void fft_run(Radices<Rs...>, float2 (&v)[E], X* lds, int p,
                                        const float2* __restrict__ tw) {
  using A = Radices<Rs...>;
  using F = typename Plan<L, RV>::fwd;
  constexpr bool is_fwd = std::is_same<A, F>::value;
  static_assert(is_fwd || std::is_same<A, Reverse<F>>::value, "radix list is not a plan of L");
  static_assert(!WAVE || (64 % P) == 0, "wave-local exchange needs each transform inside one wave");
  fft_stages<X, L, P, E, INV, WAVE, 1, (is_fwd ? 0 : StageTab<L, RV>::fwd), Rs...>(v, lds, p, tw);
}

// ---------------------------------------------------------------------------------------------
// Philox4x32-10 and Box-Muller
// ---------------------------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

// a ^ b ^ c as one three-input bitwise instruction (truth table 0x96: odd parity of the inputs)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U4 philox4x32_10(uint64_t block, uint64_t seed) {
  uint32_t c0 = (uint32_t)block, c1 = (uint32_t)(block >> 32), c2 = 0u, c3 = 0u;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    // one 32x32 -> 64-bit product per multiplier (a single v_mad_u64_u32 each)
    const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0), n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// u = (2 (x >> 9) + 1) 2^-24: an odd multiple of 2^-24, exact in FP32.  Formed as
// (1 + (x >> 9) 2^-23) - (1 - 2^-24): the first operand is the 23 bits under the exponent of 1,
// and the difference is exact (the operands lie within a factor of two of each other).
__device__ __forceinline__ float word_to_uniform(uint32_t x) {
  return __uint_as_float(0x3F800000u | (x >> 9)) - 0.999999940395355224609375f;
}

// Box-Muller on the hardware transcendentals: v_log_f32 (log2), v_sqrt_f32 and v_sin_f32 /
// v_cos_f32, whose argument is in revolutions, so sin(2 pi u) is one instruction.  Over all 2^23
// possible uniforms they stay within 1.3e-7 of the FP64 values (absolute for sin / cos, relative
// for ln u and sqrt(-2 ln u)), the accuracy of the library FP32 routines.
__device__ __forceinline__ void box_muller(uint32_t w0, uint32_t w1, float& z0, float& z1) {
  const float u0 = word_to_uniform(w0), u1 = word_to_uniform(w1);
  const float r = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u0));  // -2 ln 2 log2 u
  z0 = r * __builtin_amdgcn_cosf(u1);
  z1 = r * __builtin_amdgcn_sinf(u1);
}

__device__ __forceinline__ void noise4(uint64_t block, uint64_t seed, float (&z)[4]) {
  const U4 w = philox4x32_10(block, seed);
  box_muller(w.x, w.y, z[0], z[1]);
  box_muller(w.z, w.w, z[2], z[3]);
}

// ---------------------------------------------------------------------------------------------
// Filter amplitude (Eqs. (12)-(13) with band centre k0) in FP32
// ---------------------------------------------------------------------------------------------
struct FiltDev {
  float cr, sr;          // cos / sin of the rotation
  float ia, ib, ic;      // 1 / semi-axes
  float p, ip;           // p and 1/p
  float alpha, k0;
  float inv2w2;          // 1 / (2 w^2)
  float lnchimax;        // ln chi at K* (continuum peak)
  float offset;          // offset regularisation added to chi / chi(K*) (0: none)
  float lnoffset;        // ln offset, or -1e30
  int rotated;           // rot != 0 (H_sym differs from H on x / y Nyquist planes)
  const float* prof;     // tabulated ln chi(i dK), or null for Eq. (13)
  int prof_n;            // samples
  float prof_idk;        // 1 / dK
  // FP64 evaluation of Eq. (13), for filters whose ln chi terms are large enough that their FP32
  // rounding would show in the field (alpha ln K*, (K* - k0)^2 / (2 w^2) and ln chi(K*) summing to
  // more than 32 in magnitude: the paper's alpha = 20 .. 100): the parameters in FP64
  int prec64;
  double dcr, dsr, dia, dib, dic, dp, dip, dalpha, dk0, dinv2w2, dlnchimax, doffset;
};

// ln chi(K) of a tabulated radial form: linear interpolation between samples i dK, held at the
// last sample beyond the table
__device__ __forceinline__ float prof_lnchi(const FiltDev& f, float K) {
  const float x = K * f.prof_idk;
  if (!(x < (float)(f.prof_n - 1))) return f.prof[f.prof_n - 1];
  const int i = (int)x;
  const float t = x - (float)i;
  const float l0 = f.prof[i], l1 = f.prof[i + 1];
  return fmaf(t, l1 - l0, l0);
}

// Load of a read-only table entry at a wave-uniform index through the constant address space, so
// the compiler issues a scalar load (the host pass never runs device code and reads normally).
__device__ __forceinline__ float2 uniform_load2(const float2* p, int i) {
#if __HIP_DEVICE_COMPILE__
  return ((const __attribute__((address_space(4))) float2*)p)[i];
#else
  return p[i];
#endif
}

// raw hardware log2 / exp2 (v_log_f32, v_exp_f32)
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// ln chi (relative to its peak) at the (unrotated) wavenumber (kx, ky, kz), kz = 0 in 2D:
//   u_i = |kappa'_i| / a_i,  K = u_max (sum_i (u_i / u_max)^p)^(1/p)   (Eq. (12), scaled form)
//   ln chi = alpha ln K - (K - k0)^2 / (2 w^2) - ln chi(K*)            (Eq. (13) with band centre k0)
// or, for a tabulated radial form, the interpolated samples at K.
// The largest ratio is 1, so only the other one (2D) or two (3D) need a power.
template <int NDIM, bool PROF = false>
__device__ __forceinline__ float ln_chi(const FiltDev& f, float kx, float ky, float kz) {
  const float kxr = fmaf(f.cr, kx, f.sr * ky);
  const float kyr = fmaf(-f.sr, kx, f.cr * ky);
  const float ux = fabsf(kxr) * f.ia, uy = fabsf(kyr) * f.ib;
  float um, S;
  if constexpr (NDIM == 2) {
    um = fmaxf(ux, uy);
    const float un = fminf(ux, uy);
    if (!(um > 0.0f)) return -1.0e30f;
    const float r = un * __builtin_amdgcn_rcpf(um);
    S = 1.0f + (r > 0.0f ? hw_exp2(f.p * hw_log2(r)) : 0.0f);
  } else {
    const float uz = fabsf(kz) * f.ic;
    um = fmaxf(ux, fmaxf(uy, uz));
    if (!(um > 0.0f)) return -1.0e30f;
    const float lo = fminf(ux, fminf(uy, uz));
    const float mid = __builtin_amdgcn_fmed3f(ux, uy, uz);
    const float inv = __builtin_amdgcn_rcpf(um);
    const float r1 = mid * inv, r2 = lo * inv;
    S = 1.0f + (r1 > 0.0f ? hw_exp2(f.p * hw_log2(r1)) : 0.0f) + (r2 > 0.0f ? hw_exp2(f.p * hw_log2(r2)) : 0.0f);
  }
  const float log2K = fmaf(hw_log2(S), f.ip, hw_log2(um));
  const float K = hw_exp2(log2K);
  if constexpr (PROF) {                          // instantiated only where a tabulated form may occur
    if (f.prof) return prof_lnchi(f, K);
  }
  const float d = K - f.k0;
  return fmaf(f.alpha, log2K * 0.69314718055994531f, -fmaf(d * d, f.inv2w2, f.lnchimax));
}

// The same ln chi in FP64 (library log2 / exp2 in double precision) from the exact wavenumbers,
// for the filters flagged prec64.  The terms alpha ln K, (K - k0)^2 / (2 w^2) and ln chi(K*) of
// such filters reach 50 .. 150 while ln chi itself is O(1) in the band, so their FP32 rounding
// (2^-24 of each term) would be amplified into the amplitude; in FP64 it is 1e-14.
template <int NDIM>
__device__ __forceinline__ double ln_chi64(const FiltDev& f, double kx, double ky, double kz) {
  const double kxr = f.dcr * kx + f.dsr * ky;
  const double kyr = f.dcr * ky - f.dsr * kx;
  const double ux = fabs(kxr) * f.dia, uy = fabs(kyr) * f.dib;
  double um, S = 1.0;
  if constexpr (NDIM == 2) {
    um = fmax(ux, uy);
    if (!(um > 0.0)) return -1.0e300;
    const double un = fmin(ux, uy);
    if (un > 0.0) S += exp2(f.dp * log2(un / um));
  } else {
    const double uz = fabs(kz) * f.dic;
    um = fmax(ux, fmax(uy, uz));
    if (!(um > 0.0)) return -1.0e300;
    const double lo = fmin(ux, fmin(uy, uz));
    const double mid = fmax(fmin(ux, uy), fmin(fmax(ux, uy), uz));
    if (mid > 0.0) S += exp2(f.dp * log2(mid / um));
    if (lo > 0.0) S += exp2(f.dp * log2(lo / um));
  }
  const double log2K = log2(S) * f.dip + log2(um);
  const double K = exp2(log2K);
  const double d = K - f.dk0;
  return f.dalpha * (log2K * 0.69314718055994530942) - (d * d * f.dinv2w2 + f.dlnchimax);
}

// sqrt(chi_rel (+ offset)) from an FP64 ln chi; the DC mode keeps amplitude 0
__device__ __forceinline__ float amp_from_lnchi64(double lnc, double offset) {
  if (!(lnc > -1.0e299)) return 0.0f;
  if (offset > 0.0) return (float)sqrt(exp(lnc) + offset);
  return (float)exp(0.5 * lnc);
}

// exp(x / 2) for ln chi -> amplitude
__device__ __forceinline__ float amp_from_lnchi(float lnc) { return hw_exp2(lnc * 0.72134752044448170368f); }

// sqrt(chi_rel + offset) with the offset regularisation (a uniform branch); the DC mode (ln chi
// returned as -1e30) keeps amplitude 0
__device__ __forceinline__ float amp_from_lnchi(float lnc, float offset) {
  if (offset > 0.0f)
    return lnc > -1.0e29f ? __builtin_sqrtf(hw_exp2(lnc * 1.44269504088896340736f) + offset) : 0.0f;
  return amp_from_lnchi(lnc);
}

// ---------------------------------------------------------------------------------------------
// Bin index: exact integer radial rule, FP64 angular edges tested with separately rounded
// products.  q = signed index scaled to the common denominator D = lcm(n_i).
// ---------------------------------------------------------------------------------------------
struct BinDev {
  int nr, na;
  long long D2;          // D^2
  float invD2;           // 1 / D^2 (estimate only; the rule itself is exact in integers)
  long long fourR2;      // 4 R^2
  const double* ex;      // angular edge unit vectors, na - 1 of them
  const double* ey;
};

#pragma clang fp contract(off)
__device__ __forceinline__ bool edge_le(const BinDev& b, int j, double qx, double qy) {
  // angle(e_j) <= angle(q) for j in 1..na-1 (edges stored from index 0)
  const double t1 = b.ex[j - 1] * qy;
  const double t2 = b.ey[j - 1] * qx;
  return (t1 - t2) >= 0.0;
}

__device__ __forceinline__ int bin_index(const BinDev& b, long long s, long long qx, long long qy) {
  // s = sum of q_i^2; radial r = max{r : r^2 D^2 <= 4 R^2 s}
  const long long rhs = b.fourR2 * s;
  long long r = (long long)__builtin_amdgcn_sqrtf((float)rhs * b.invD2);
  if (r * r * b.D2 > rhs) --r;
  if ((r + 1) * (r + 1) * b.D2 <= rhs) ++r;
  if (r >= b.nr) return b.nr * b.na;
  int a = 0;
  if (b.na > 1 && s != 0) {
    if (qy < 0) { qy = -qy; qx = -qx; }
    const double dx = (double)qx, dy = (double)qy;
    // estimate from atan2, then settle on the exact edge tests
    float ang = atan2f((float)dy, (float)dx);                 // [0, pi]
    int g = (int)(ang * (float)b.na * 0.31830988618379067f);
    g = g < 0 ? 0 : (g > b.na - 1 ? b.na - 1 : g);
    while (g < b.na - 1 && edge_le(b, g + 1, dx, dy)) ++g;
    while (g > 0 && !edge_le(b, g, dx, dy)) --g;
    a = g;
  }
  return (int)r * b.na + a;
}
#pragma clang fp contract(on)

}  // namespace hu
