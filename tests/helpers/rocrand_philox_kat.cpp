// Known-answer helper for the Philox4x32-10 pin: prints the raw 4-word block that
// ROCm's rocRAND (header-only engine, an implementation independent of this
// project) produces for a given counter and key.  Compiled and run by the CPU
// test suite; it never runs on a GPU.
//
// rocRAND's engine is seeded with key = (seed_lo, seed_hi); its subsequence
// selects counter words (z, w) and discard(4*n) advances counter words (x, y) by
// n blocks, so engine(seed, (w<<32)|z, 0) advanced by (y<<32)|x blocks yields the
// block for counter (x, y, z, w).  The advance is split into four equal parts plus
// a remainder so that 4*n never overflows 64 bits.
#include <cstdio>
#include <cstdlib>
#include <rocrand/rocrand_philox4x32_10.h>

int main(int argc, char** argv) {
  if (argc != 7) { std::fprintf(stderr, "usage: c0 c1 c2 c3 k0 k1\n"); return 2; }
  unsigned long long v[6];
  for (int i = 0; i < 6; ++i) v[i] = std::strtoull(argv[i + 1], nullptr, 0);
  const unsigned long long seed = (v[5] << 32) | v[4];
  const unsigned long long subseq = (v[3] << 32) | v[2];
  const unsigned long long blocks = (v[1] << 32) | v[0];
  rocrand_device::philox4x32_10_engine eng(seed, subseq, 0);
  const unsigned long long quarter = blocks >> 2;
  for (int i = 0; i < 4; ++i) eng.discard(4ull * quarter);
  eng.discard(4ull * (blocks - 4ull * quarter));
  uint4 r = eng.next4();
  std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  return 0;
}
