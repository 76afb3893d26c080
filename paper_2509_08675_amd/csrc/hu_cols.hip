// Plain complex transform along a strided axis (the y axis of 3D grids), forward or inverse, in
// place.  Element e of column g lives at (g / inner) * (L * inner) + (g % inner) + e * inner; a
// workgroup transforms C adjacent columns, P threads per column, E elements per thread.
#include "hu_common.hpp"

namespace hu {

template <int L, bool INV, int V, int RV>
__global__ void __launch_bounds__((ColTile<L, V>::T)) k_cols(ColsArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = ColTile<L, V>::C;
  using Rad = typename Plan<L, RV>::fwd;
  constexpr int R1 = RadInfo<Rad>::first, RL = RadInfo<Rad>::last;
  extern __shared__ float2 lds[];
  int b;
  long long tile;
  if (!map_tile(a.sc, b, tile)) return;
  const int tid = threadIdx.x;
  const int c = tid % C, p = tid / C;
  const int g = (int)tile * C + c;
  const bool valid = g < a.ncol;
  const ColIO io = col_io<L>(a.spec + (long long)b * a.Nh, a.Nh, a.inner, g, p);
  float2 v[E];
  col_load<L, R1, P, E>(v, io);
  fft_run<L, P, E, INV, false, RV>(Rad{}, v, lds + c * ColTile<L, V>::RS, p, a.tw);
  if (valid) col_store<L, RL, P, E>(v, io);
}

template <int L, int V>
static ColSched col_sched_L(long long ncol, int batch, int group) {
  constexpr int C = ColTile<L, V>::C;
  ColSched s;
  s.ntiles = (int)((ncol + C - 1) / C);
  // one workgroup per tile; `group` consecutive tiles go to the same XCD (they share the 128-byte
  // lines at their boundaries when the column index runs over rows that are not line-aligned)
  s.G = group > 0 ? group : 1;
  s.ntiles_pad = (s.ntiles + s.G - 1) / s.G * s.G;
  s.batch = batch;
  s.finner = 0;
  return s;
}

ColSched col_sched(int L, int variant, long long ncol, int batch, int group) {
  switch (L) {
#define X(LL) \
  case LL: return variant ? col_sched_L<LL, 1>(ncol, batch, group) : col_sched_L<LL, 0>(ncol, batch, group);
    HU_COL_LENGTHS(X)
#undef X
    default: return ColSched{0, 0, 1, 0, 0};
  }
}

// The B fields of a tile get consecutive ids on one XCD, so a per-geometry table slice read by the
// tile (the bin indices of its modes) is fetched into that XCD's L2 once for all the fields.
ColSched col_sched_fields(int L, int variant, long long ncol, int batch) {
  ColSched s = col_sched(L, variant, ncol, batch, 1);
  if (batch > 1) {
    s.G = batch;
    s.ntiles_pad = s.ntiles;
    s.finner = 1;
  }
  return s;
}

int col_tiles(int L, int variant, long long ncol) { return col_sched(L, variant, ncol, 1).ntiles; }

template <int L, bool INV, int V, int RV>
static hipError_t launch_cols_L(const ColsArgs& a, hipStream_t st) {
  constexpr int T = ColTile<L, V>::T;
  hipLaunchKernelGGL((k_cols<L, INV, V, RV>), dim3(sched_blocks(a.sc)), dim3(T), (col_xchg_bytes<L, V>()), st, a);
  return hipGetLastError();
}

hipError_t launch_cols(int L, bool inv, int variant, const ColsArgs& a, hipStream_t st, int radix) {
  switch (L) {
#define X(LL)                                                                                        \
  case LL:                                                                                           \
    return with_choices<LL>(variant, radix, [&](auto v, auto r) {                                    \
      constexpr int V = decltype(v)::value, RV = decltype(r)::value;                                \
      return inv ? launch_cols_L<LL, true, V, RV>(a, st) : launch_cols_L<LL, false, V, RV>(a, st); \
    });
    HU_COL_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hu
