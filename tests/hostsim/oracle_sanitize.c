/* Drives every entry of the CPU oracle (oracle/rmat_oracle.c) once or more,
 * for a build under the host address and undefined-behaviour sanitizers:
 * R-MAT tables (VARIABLE and FIXED, ties, degenerate parameters, an L2-sized
 * table), edges with both id widths and the epilogues, chunk reductions,
 * binomial draws, partitioned counts and edges, K x K tables and edges, and
 * perturbed sets.  Prints a checksum of everything it produced; exit status
 * 0 unless an entry reported an error it should not have.
 *
 *   oracle_sanitize                (compiled together with rmat_oracle.c) */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc_table orc_table;
orc_table* orc_table_new(void);
void orc_table_delete(orc_table* t);
void orc_table_info(const orc_table* t, uint64_t info[8]);
int orc_build_table(double a, double b, double c, double d, int k, uint64_t bound, int mode, orc_table* out);
int orc_generate_ex(const orc_table* t, uint64_t seed, uint64_t edge_begin, uint64_t m, void* src, void* dst,
                    int width, uint32_t* n_samples, int threads, int flags, uint64_t scramble_key);
int orc_generate_reduce(const orc_table* t, uint64_t seed, uint64_t edge_begin, uint64_t m, int hist_bits,
                        uint64_t* hist, uint64_t* xor_out, int threads);
uint64_t orc_binomial(uint64_t seed, uint32_t r, uint32_t c, int level, uint64_t n, double p);
int orc_partition_counts(const orc_table* t, uint64_t seed, uint64_t m, int tbits, uint32_t row_begin,
                         uint32_t row_end, uint64_t* counts);
int orc_generate_partition(const orc_table* t, uint64_t seed, uint64_t m, int tbits, uint32_t row_begin,
                           uint32_t row_end, void* src, void* dst, int width, const uint64_t* counts);
int orc_kron_build_table(const double* P, int K, int k, uint64_t bound, int mode, orc_table* out);
int orc_perturbed_params(double a, double b, double c, double d, int n_tables, double eps, uint64_t seed,
                         double* out);
int orc_generate_set(const orc_table* const* tables, int n_tables, uint64_t seed, uint64_t edge_begin, uint64_t m,
                     void* src, void* dst, int width);

static uint64_t g_sum = 0;
static int g_bad = 0;

static void mix(const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) g_sum = (g_sum ^ b[i]) * 0x100000001B3ull;
}

static void expect(int rc, int want, const char* what) {
  if (rc != want) {
    fprintf(stderr, "%s: status %d, want %d\n", what, rc, want);
    ++g_bad;
  }
}

static void edges(const orc_table* t, uint64_t seed, uint64_t e0, uint64_t m, int width, int flags, int threads) {
  void* s = malloc(m * 8 + 8);
  void* d = malloc(m * 8 + 8);
  uint32_t* ns = (uint32_t*)malloc(m * 4 + 4);
  expect(orc_generate_ex(t, seed, e0, m, s, d, width, ns, threads, flags, 0xC0FFEE), 0, "generate");
  mix(s, m * width);
  mix(d, m * width);
  mix(ns, m * 4);
  free(s);
  free(d);
  free(ns);
}

int main(void) {
  const double G[4] = {0.57, 0.19, 0.19, 0.05};
  struct { double q[4]; int k; uint64_t bound; int mode; } rm[] = {
      {{0.57, 0.19, 0.19, 0.05}, 16, 256, 0},     {{0.57, 0.19, 0.19, 0.05}, 26, 4096, 1},
      {{0.45, 0.22, 0.22, 0.11}, 34, 1 << 16, 1}, {{0.25, 0.25, 0.25, 0.25}, 20, 5000, 1},
      {{1.0, 0.0, 0.0, 0.0}, 26, 300, 1},         {{0.5, 0.5, 0.0, 0.0}, 64, 1000, 1},
      {{0.9, 0.025, 0.025, 0.05}, 40, 8192, 1},   {{0.57, 0.19, 0.19, 0.05}, 1, 5, 1},
      {{0.57, 0.19, 0.19, 0.05}, 30, 4, 0},       {{0.57, 0.19, 0.19, 0.05}, 28, 1 << 18, 1},
  };
  for (size_t i = 0; i < sizeof(rm) / sizeof(rm[0]); ++i) {
    orc_table* t = orc_table_new();
    expect(orc_build_table(rm[i].q[0], rm[i].q[1], rm[i].q[2], rm[i].q[3], rm[i].k, rm[i].bound, rm[i].mode, t), 0,
           "build_table");
    uint64_t info[8];
    orc_table_info(t, info);
    mix(info, sizeof(info));
    const int width = rm[i].k <= 32 ? 4 : 8;
    edges(t, 7 + i, 0, 5000, width, 0, 1);
    edges(t, 9 + i, (1ull << 32) - 777, 3000, 8, 3, 4);       /* epilogue, 64-bit slots, threads */
    edges(t, ~0ull, ~0ull - 999, 1000, 8, 1, 2);               /* the last edges of the stream */
    const int hb = rm[i].k < 16 ? rm[i].k : 16;
    uint64_t* hist = (uint64_t*)calloc((size_t)1 << hb, 8);
    uint64_t x = 0;
    expect(orc_generate_reduce(t, 3, 12345, 20000, hb, hist, &x, 3), 0, "generate_reduce");
    mix(hist, ((size_t)1 << hb) * 8);
    mix(&x, 8);
    free(hist);
    if (rm[i].k >= 4) {
      const int tb = rm[i].k > 8 ? 3 : 2;
      const uint32_t rows = 1u << tb;
      uint64_t* cnt = (uint64_t*)calloc((size_t)rows << tb, 8);
      expect(orc_partition_counts(t, 5, 30000, tb, 0, rows, cnt), 0, "partition_counts");
      uint64_t n = 0;
      for (uint64_t j = 0; j < ((uint64_t)rows << tb); ++j) n += cnt[j];
      if (n != 30000) {
        fprintf(stderr, "partition counts sum to %llu\n", (unsigned long long)n);
        ++g_bad;
      }
      void* s = malloc(n * 8);
      void* d = malloc(n * 8);
      expect(orc_generate_partition(t, 5, 30000, tb, 0, rows, s, d, 8, cnt), 0, "generate_partition");
      mix(s, n * 8);
      mix(d, n * 8);
      free(s);
      free(d);
      free(cnt);
    }
    orc_table_delete(t);
  }
  /* rejected inputs */
  orc_table* bad = orc_table_new();
  expect(orc_build_table(0.57, 0.19, 0.19, 0.05 - 9e-10, 26, 5, 1, bad) != 0, 1, "residual out of range");
  orc_table_delete(bad);
  bad = orc_table_new();
  expect(orc_build_table(0.6, 0.19, 0.19, 0.05, 26, 4096, 1, bad) != 0, 1, "sum not 1");
  orc_table_delete(bad);
  /* binomial draws in both regimes */
  for (int i = 0; i < 200; ++i) {
    const uint64_t v = orc_binomial(1000 + i, i, 3 * i, i % 7, (uint64_t)1 << (i % 41), 0.03 + 0.0047 * i);
    mix(&v, 8);
  }
  /* K x K tables and edges */
  const double P3[9] = {0.3, 0.1, 0.05, 0.1, 0.2, 0.05, 0.05, 0.05, 0.1};
  double P16[256], U9[9], Z9[9] = {0.5, 0, 0, 0, 0.5, 0, 0, 0, 0};
  for (int x = 0; x < 256; ++x) P16[x] = 1.0 / 256;
  for (int x = 0; x < 9; ++x) U9[x] = 1.0 / 9;
  struct { const double* P; int K, k; uint64_t bound; int mode; } kr[] = {
      {P3, 3, 17, 4096, 1}, {P3, 3, 12, 729, 0}, {P16, 16, 16, 300, 1}, {U9, 3, 12, 4000, 1},
      {Z9, 3, 12, 8000, 1}, {P3, 3, 40, 5000, 1}};
  for (size_t i = 0; i < sizeof(kr) / sizeof(kr[0]); ++i) {
    orc_table* t = orc_table_new();
    expect(orc_kron_build_table(kr[i].P, kr[i].K, kr[i].k, kr[i].bound, kr[i].mode, t), 0, "kron_build_table");
    edges(t, 11, 77, 4000, 8, 0, 2);
    orc_table_delete(t);
  }
  /* perturbed sets */
  double qs[8 * 4];
  expect(orc_perturbed_params(G[0], G[1], G[2], G[3], 8, 0.1, 2019, qs), 0, "perturbed_params");
  orc_table* set[8];
  for (int i = 0; i < 8; ++i) {
    set[i] = orc_table_new();
    expect(orc_build_table(qs[4 * i], qs[4 * i + 1], qs[4 * i + 2], qs[4 * i + 3], 26, 1024, 1, set[i]), 0,
           "perturbed member");
  }
  {
    void* s = malloc(6000 * 4);
    void* d = malloc(6000 * 4);
    expect(orc_generate_set((const orc_table* const*)set, 8, 3, 5, 6000, s, d, 4), 0, "generate_set");
    mix(s, 6000 * 4);
    mix(d, 6000 * 4);
    free(s);
    free(d);
  }
  for (int i = 0; i < 8; ++i) orc_table_delete(set[i]);
  printf("checksum %016llx, %d unexpected statuses\n", (unsigned long long)g_sum, g_bad);
  return g_bad ? 1 : 0;
}
