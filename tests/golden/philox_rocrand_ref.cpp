// Independent Philox4x32-10 reference for pinning the oracle's generator.
//
// Uses the header-only engine that ships with rocRAND (rocrand_philox4x32_10.h), built as
// a host program.  With seed s, subsequence 0 and offset 0 the engine's key is
// (s mod 2^32, s >> 32) and its 128-bit counter starts at 0 and steps by one per block of
// four words, which is the stream layout the oracle adopts.  Usage:
//   philox_rocrand_ref <seed> <first_block> <n_blocks>
// prints 4 * n_blocks hexadecimal words, one per line.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  unsigned long long seed = strtoull(argv[1], nullptr, 0);
  unsigned long long first = strtoull(argv[2], nullptr, 0);
  long n = atol(argv[3]);
  rocrand_device::philox4x32_10_engine eng(seed, 0, 0);
  eng.discard(4ull * first);
  for (long i = 0; i < 4 * n; ++i) printf("%08x\n", eng.next());
  return 0;
}
