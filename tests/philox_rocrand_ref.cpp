// Third-party cross-check for the oracle's Philox4x32-10: runs rocRAND's own
// host-side Philox4x32-10 engine (a black box here) and prints its output.
// Input lines: "seed e j" (decimal).  Output lines: four hex words, the block
// for key (seed_lo, seed_hi) and 128-bit counter e + j * 2^64, i.e. the words
// (e_lo, e_hi, j, 0).  rocRAND advances the counter's low 64 bits with its
// offset (4 words per block) and the high 64 bits with its subsequence; the
// offset is advanced in steps of 2^63 words so that every e < 2^64 is reached.
// Test-only; compiled by the test suite, never part of the product.
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

int main() {
  unsigned long long seed, e, j;
  while (std::scanf("%llu %llu %llu", &seed, &e, &j) == 3) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, j, 0, &st);
    const unsigned long long step = 1ull << 61;  // blocks per skip of 2^63 words
    for (unsigned long long q = e / step; q > 0; --q) skipahead(4ull * step, &st);
    skipahead(4ull * (e % step), &st);
    unsigned w[4];
    for (int i = 0; i < 4; ++i) w[i] = rocrand(&st);
    std::printf("%08x %08x %08x %08x\n", w[0], w[1], w[2], w[3]);
  }
  return 0;
}
