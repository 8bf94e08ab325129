// The library's host-side partition code (tile counting on host threads,
// work lists, pinned list staging) against the fake device, for a build
// under the host address and undefined-behaviour sanitizers: every count
// equals the CPU oracle's, and the work lists of a generation cover every
// block of every non-empty tile once.  Exit status 0 when all checks pass.
//
//   partition_sanitize    (compiled with api.cpp, partition.cpp,
//                          fake_device.cpp and oracle/rmat_oracle.c)
#include <cinttypes>
#include <cstdio>
#include <vector>

#include "rmat.h"

extern "C" {
struct orc_table;
orc_table* orc_table_new(void);
void orc_table_delete(orc_table* t);
int orc_build_table(double a, double b, double c, double d, int k, uint64_t bound, int mode, orc_table* out);
int orc_partition_counts(const orc_table* t, uint64_t seed, uint64_t m, int tbits, uint32_t row_begin,
                         uint32_t row_end, uint64_t* counts);
int sim_failed();
void sim_whole_cover(int on);
uint64_t sim_cover_insts();
}

int main() {
  struct Case {
    double q[4];
    int k;
    uint64_t bound, seed, m;
    int tb;
    uint32_t r0, r1;
  } cases[] = {
      {{0.57, 0.19, 0.19, 0.05}, 12, 256, 3, 100000, 3, 0, 8},
      {{0.57, 0.19, 0.19, 0.05}, 26, 4096, 7, 1ull << 30, 6, 0, 64},
      {{0.45, 0.22, 0.22, 0.11}, 34, 1 << 16, 3, 1ull << 34, 8, 17, 90},
      {{0.25, 0.25, 0.25, 0.25}, 40, 1000, 11, 1ull << 53, 9, 500, 512},
      {{1.0, 0.0, 0.0, 0.0}, 20, 300, 1, 123456, 4, 0, 16},
      {{0.5, 0.5, 0.0, 0.0}, 20, 300, 2, 7, 5, 0, 32},
      {{0.6, 0.1, 0.3, 0.0}, 16, 64, 5, 0, 2, 0, 4},
      {{0.57, 0.19, 0.19, 0.05}, 24, 4096, 5, 1ull << 22, 10, 0, 4},
      {{0.25, 0.25, 0.25, 0.25}, 22, 1000, 4, 450ull << 16, 8, 7, 9},
  };
  int bad = 0;
  for (const Case& c : cases) {
    rmat_table_t t = nullptr;
    if (rmat_build_table(c.q[0], c.q[1], c.q[2], c.q[3], c.k, c.bound, RMAT_VARIABLE, &t) != RMAT_OK) {
      std::printf("build: %s\n", rmat_last_error());
      ++bad;
      continue;
    }
    const size_t n = static_cast<size_t>(c.r1 - c.r0) << c.tb;
    std::vector<uint64_t> got(n), want(n);
    if (rmat_partition_counts(t, c.seed, c.m, c.tb, c.r0, c.r1, got.data()) != RMAT_OK) {
      std::printf("counts: %s\n", rmat_last_error());
      ++bad;
    }
    orc_table* o = orc_table_new();
    orc_build_table(c.q[0], c.q[1], c.q[2], c.q[3], c.k, c.bound, 1, o);
    orc_partition_counts(o, c.seed, c.m, c.tb, c.r0, c.r1, want.data());
    orc_table_delete(o);
    if (got != want) {
      std::printf("k=%d tiles 2^%d: counts differ from the oracle\n", c.k, c.tb);
      ++bad;
    }
    uint64_t total = 0, tiles = 0;
    for (uint64_t v : got) {
      total += v;
      tiles += v > 0;
    }
    if (total > (1ull << 24)) {  // the fake device keeps a counter per edge: cover only small graphs
      rmat_free_table(t);
      continue;
    }
    uint64_t dummy[2];
    sim_whole_cover(1);
    if (rmat_generate_partition(t, c.seed, c.m, c.tb, c.r0, c.r1, dummy, dummy, total) != RMAT_OK) {
      std::printf("generate: %s\n", rmat_last_error());
      ++bad;
    } else if (total > 0 && sim_cover_insts() != tiles) {
      std::printf("k=%d: work lists cover %" PRIu64 " tiles of %" PRIu64 "\n", c.k, sim_cover_insts(), tiles);
      ++bad;
    }
    sim_whole_cover(0);
    rmat_free_table(t);
  }
  if (sim_failed()) ++bad;
  std::printf("%d failures\n", bad);
  return bad ? 1 : 0;
}
