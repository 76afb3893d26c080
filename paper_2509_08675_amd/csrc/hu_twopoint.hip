// Two-point probability function of the +1 phase of a +-1 map (Wiener-Khinchin, Eqs. (10)-(11)):
// with G the unnormalised DFT of g and m = G(0) / N,
//   S_2(r) = (1 + 2 m + C(r)) / 4,   C(r) = (1/N) sum_x g(x) g(x + r) = IDFT(|G|^2)(r) / N^2,
// IDFT unnormalised.  After the row and y passes of the power spectrum, this axis-0 pass
// transforms each column, replaces G by |G|^2 and transforms back; the thread holding the DC mode
// writes the scale 1 / (4 N^2) and the offset (1 + 2 m) / 4 that the inverse row pass applies.
#include "hu_common.hpp"

namespace hu {

template <int L>
__global__ void __launch_bounds__((ColTile<L, 0>::T)) k_cols_square(SquareArgs a) {
  constexpr int P = Plan<L>::P, E = Plan<L>::E, C = ColTile<L, 0>::C, T = ColTile<L, 0>::T;
  using Rad = typename Plan<L>::fwd;
  using RadI = Reverse<Rad>;
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
  fft_run<L, P, E, false>(Rad{}, v, lds + c * ColTile<L, 0>::RS, p, a.tw);
  if (g == 0 && p == 0) {    // slot 0 of thread 0 of column 0 holds the DC mode
    const double N = (double)a.N;
    double* fs = a.fstats + (long long)b * 8;
    fs[4] = 0.25 / (N * N);
    fs[5] = 0.25 * (1.0 + 2.0 * (double)v[0].x / N);
  }
#pragma unroll
  for (int s = 0; s < E; ++s) v[s] = make_float2(fmaf(v[s].x, v[s].x, v[s].y * v[s].y), 0.0f);
  __syncthreads();          // every read of the forward transform's last exchange is done
  fft_run<L, P, E, true>(RadI{}, v, lds + c * ColTile<L, 0>::RS, p, a.tw);
  if (valid) col_store<L, R1, P, E>(v, io);
}

template <int L>
static hipError_t launch_cols_square_L(const SquareArgs& a, hipStream_t st) {
  constexpr int T = ColTile<L, 0>::T;
  hipLaunchKernelGGL((k_cols_square<L>), dim3(sched_blocks(a.sc)), dim3(T), (col_xchg_bytes<L, 0>()), st, a);
  return hipGetLastError();
}

hipError_t launch_cols_square(int L, const SquareArgs& a, hipStream_t st) {
  switch (L) {
#define X(LL) case LL: return launch_cols_square_L<LL>(a, st);
    HU_COL_LENGTHS(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hu
