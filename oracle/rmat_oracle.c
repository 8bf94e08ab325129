/*
 * rmat_oracle.c -- plain, slow, CPU reference for the linear-work R-MAT sampler.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may use it.  It shares no code, header, table or
 * constant generator with the HIP implementation.
 *
 * What it computes follows Huebschle-Schneider & Sanders, "Linear Work
 * Generation of R-MAT Graphs" (arXiv 1905.03525):
 *
 *   - Sec. 1: the R-MAT process.  An edge of a graph with n = 2^k nodes is k
 *     independent quadrant choices a (row 0, col 0), b (row 0, col 1),
 *     c (row 1, col 0), d (row 1, col 1); one row bit and one column bit per
 *     level.
 *   - Sec. 2, the max-priority-queue fragment: a table of quadrant paths is
 *     grown by repeatedly expanding the most probable path into its four
 *     one-letter extensions; a path's probability is the product of its
 *     letters.  The fixed-length variant takes all paths of one length.
 *   - Sec. 2: the table is turned into a Walker alias structure [Walker 1977]
 *     for constant-time sampling.
 *   - Sec. 2, the sampling loop: sampled paths are appended to the row and
 *     column bit strings until k bits are known; the first k bits form the
 *     edge.
 *
 * Readings taken where the paper is silent (each is listed in the design
 * notes, with the reason):
 *   R1 letter -> bits: a=(0,0) b=(0,1) c=(1,0) d=(1,1); the row is the source.
 *   R2 variable table size: expand while |entries| + 3 < bound, so the table
 *      has 1 + 3t entries, t = ceil((bound - 4) / 3).  This reproduces every
 *      table size on the x-axis of Fig. 1 (253, 511, 1021, ...).
 *   R3 ties in deleteMax: order by probability descending, then depth
 *      ascending, then the path read as base-4 digits (a<b<c<d) ascending.
 *      A path's probability is the canonical product: 1.0 times a (n_a
 *      times), then b, then c, then d, each product rounded to nearest double.
 *   R4 depth cap min(15, k): a path of that length is never expanded.  With
 *      it the table's mean path length matches the "13.9 bits" (2^13 entries)
 *      and "15 bits" (2^21 entries) of Sec. 4 for a=.9, b=c=.025, d=.05.
 *   R5 fixed length: l = floor(log4 bound), 1 <= l <= depth cap.
 *   R6 items are the leaves sorted in tree order (left-aligned code); the
 *      alias table has 2^ceil(log2 |A|) buckets; padding items weigh 0.
 *   R7 weights w_j: p_j * 2^32 rounded by largest remainders (floors, then
 *      one more unit to each of the items with the largest fractional parts,
 *      ties to the lower index) so that they sum to exactly 2^32.
 *   R8 alias table: the deterministic sweep in build_alias() below; bucket i
 *      holds threshold T_i and alias A_i, bucket capacity C = 2^(32 - b).
 *   R9 randomness: Philox4x32-10 [Salmon, Moraes, Dror, Shaw, SC'11] with
 *      key (seed_lo, seed_hi) and counter (e_lo, e_hi, j, 0); sample s of
 *      edge e uses output word s mod 4 of counter j = s / 4.
 *  R10 a sample x picks bucket (x >> 4) mod 2^b, the b bits above the
 *      lowest four; the other 32 - b bits, in their order, form the uniform
 *      f = (x >> (b + 4)) * 16 + (x mod 16) in [0, C), and the item is the
 *      bucket's own item if f < T, else its alias.
 *  R11 the first (root-most) letter of the stream is the most significant
 *      bit of the k-bit row and column ids.
 *  R12 letters left over after the k-th are discarded (each edge has its own
 *      counter stream), instead of being carried over to the next edge.
 *  R19 Sec. 3 (Generalizations) epilogue, optional per call: an undirected
 *      graph mirrors each edge of the lower-left triangle (row > column) to
 *      the upper right, i.e. swaps its ids; the scramble relabels every id by
 *      one keyed bijection pi of [0, 2^k), applied after the mirror.  pi is
 *      three rounds of x = (x * M_r + C_r) mod 2^k, x = x XOR (x >> ceil(k/2)),
 *      with M_r (odd) and C_r the outputs of SplitMix64 [Steele, Lea, Flood,
 *      OOPSLA'14] seeded with the scramble key, drawn in the order M_0, C_0,
 *      M_1, C_1, M_2, C_2 (M_r with its lowest bit set).
 *  R22 Sec. 3 perturbed tables: P tables (P a power of two <= 64) built from
 *      (a, b, c, d) with each entry x multiplied by 1 + eps (2 u - 1) and then
 *      normalised, u the 53-bit uniforms of SplitMix64 seeded with the
 *      perturbation seed, drawn table by table, entries in the order a, b,
 *      c, d; edge e is drawn from table e mod P.
 *  R20 Sec. 3 partitioned generation: the adjacency matrix is cut into
 *      2^t x 2^t tiles; the m edges are split over them top-down, each node
 *      of the quadrant tree splitting its count n into (n_a, n_b, n_c, n_d)
 *      by n_a = Bin(n, a), n_b = Bin(n - n_a, b / (b + c + d)),
 *      n_c = Bin(n - n_a - n_b, c / (c + d)), n_d = the rest.  Bin(n, p) is
 *      inversion for n min(p, 1-p) < 30 and BTPE [Kachitvichyanukul &
 *      Schmeiser, CACM 1988] otherwise, with p > 1/2 drawn as n - Bin(n, 1-p).
 *      Node (level l, row prefix R, column prefix C) draws its uniforms from
 *      Philox4x32-10 under the seed with counter (R, C, i, 2^31 + l), two
 *      53-bit uniforms per block.  Edge j of tile (R, C) samples the
 *      remaining k - t letters with counter (j_lo, j_hi, s / 4,
 *      1 + R 2^t + C) and gets the tile's prefixes: src = R 2^(k-t) + row.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EINTERNAL (-3)
#define ORC_ERANGE (-4)

#define ORC_FIXED 0
#define ORC_VARIABLE 1
#define ORC_MAX_CAP 15

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon et al., SC'11, Sec. 3: the Philox S-box with
 * multipliers 0xD2511F53 / 0xCD9E8D57 and Weyl key increments 0x9E3779B9 /
 * 0xBB67AE85; ten rounds, the key bumped between rounds).
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------
 * Path probabilities (Sec. 2: a path's probability is the product of its
 * letters; reading R3 fixes the multiplication order).
 * ---------------------------------------------------------------------- */
double orc_canonical_product(const double q[4], const int counts[4]) {
  double p = 1.0;
  for (int letter = 0; letter < 4; ++letter)
    for (int i = 0; i < counts[letter]; ++i) p = p * q[letter];
  return p;
}

typedef struct {
  double p;
  uint64_t code; /* base-4 digits, root-most letter most significant */
  int depth;
  int counts[4];
} node_t;

/* Total order of reading R3: does u come before v? */
static int node_before(const node_t* u, const node_t* v) {
  if (u->p != v->p) return u->p > v->p;
  if (u->depth != v->depth) return u->depth < v->depth;
  return u->code < v->code;
}

/* Binary max-heap under node_before: the max-priority queue of Sec. 2. */
typedef struct {
  node_t* a;
  size_t n, cap;
} heap_t;

static int heap_push(heap_t* h, node_t v) {
  if (h->n == h->cap) {
    size_t nc = h->cap ? 2 * h->cap : 1024;
    node_t* na = (node_t*)realloc(h->a, nc * sizeof(node_t));
    if (!na) return ORC_ENOMEM;
    h->a = na;
    h->cap = nc;
  }
  size_t i = h->n++;
  h->a[i] = v;
  while (i > 0) {
    size_t parent = (i - 1) / 2;
    if (!node_before(&h->a[i], &h->a[parent])) break;
    node_t t = h->a[i]; h->a[i] = h->a[parent]; h->a[parent] = t;
    i = parent;
  }
  return ORC_OK;
}

static node_t heap_pop(heap_t* h) {
  node_t top = h->a[0];
  h->a[0] = h->a[--h->n];
  size_t i = 0;
  for (;;) {
    size_t l = 2 * i + 1, r = l + 1, best = i;
    if (l < h->n && node_before(&h->a[l], &h->a[best])) best = l;
    if (r < h->n && node_before(&h->a[r], &h->a[best])) best = r;
    if (best == i) break;
    node_t t = h->a[i]; h->a[i] = h->a[best]; h->a[best] = t;
    i = best;
  }
  return top;
}

/* ------------------------------------------------------------------------
 * The table.
 * ---------------------------------------------------------------------- */
typedef struct {
  int k, mode, cap, bucket_bits;
  uint64_t bound, n_items, n_buckets, capacity; /* capacity = C = 2^(32-b) */
  double q[4];
  int K;          /* initiator size: 2 for R-MAT, K x K for a Kronecker table (R21) */
  uint64_t powK[16];
  /* per item (n_buckets entries; items >= n_items are padding) */
  uint8_t* len;
  uint64_t* code;
  uint32_t* row;   /* row bits of the path, root-most letter is the MSB */
  uint32_t* col;
  double* p;
  int64_t* w;
  /* per bucket */
  uint32_t* thr;   /* T_i, equal to C for a full bucket */
  uint32_t* alias; /* A_i, equal to i for a full bucket */
} orc_table;

static int cmp_u64(const void* x, const void* y) {
  uint64_t a = *(const uint64_t*)x, b = *(const uint64_t*)y;
  return a < b ? -1 : (a > b ? 1 : 0);
}

void orc_free_table(orc_table* t) {
  if (!t) return;
  free(t->len); free(t->code); free(t->row); free(t->col);
  free(t->p); free(t->w); free(t->thr); free(t->alias);
  memset(t, 0, sizeof(*t));
}

/* Validation of the inputs (Sec. 1: a+b+c+d = 1; readings R2, R5). */
static int validate(const double q[4], int k, uint64_t bound, int mode) {
  double s = 0.0;
  for (int i = 0; i < 4; ++i) {
    if (!(q[i] >= 0.0) || isnan(q[i]) || isinf(q[i])) return ORC_EINVAL;
    s += q[i];
  }
  if (fabs(s - 1.0) > 1e-9) return ORC_EINVAL;
  if (k < 1 || k > 64) return ORC_EINVAL;
  if (bound > (1ull << 24)) return ORC_EINVAL;
  if (mode == ORC_VARIABLE) {
    if (bound < 5) return ORC_EINVAL;
  } else if (mode == ORC_FIXED) {
    if (bound < 4) return ORC_EINVAL;
  } else {
    return ORC_EINVAL;
  }
  return ORC_OK;
}

/* Enumerate the leaves.  Fixed: all 4^l paths (Sec. 2, first strategy).
 * Variable: the priority-queue expansion of Sec. 2 with readings R2-R4.
 * Output: codes and depths of the leaves in tree order. */
static int enumerate_leaves(orc_table* t, uint64_t** out_lac_sorted) {
  int cap = t->k < ORC_MAX_CAP ? t->k : ORC_MAX_CAP;
  t->cap = cap;
  size_t n = 0;
  node_t* leaves = NULL;
  if (t->mode == ORC_FIXED) {
    int ell = 0;
    while (ell < 30 && (1ull << (2 * (ell + 1))) <= t->bound) ++ell;
    if (ell < 1 || ell > cap) return ORC_EINVAL;
    n = (size_t)1 << (2 * ell);
    leaves = (node_t*)calloc(n, sizeof(node_t));
    if (!leaves) return ORC_ENOMEM;
    for (size_t code = 0; code < n; ++code) {
      node_t v;
      memset(&v, 0, sizeof(v));
      v.code = code;
      v.depth = ell;
      for (int pos = 0; pos < ell; ++pos) v.counts[(code >> (2 * pos)) & 3]++;
      v.p = orc_canonical_product(t->q, v.counts);
      leaves[code] = v;
    }
  } else {
    heap_t q = {0, 0, 0};
    size_t n_final = 0, cap_final = 0;
    node_t* final_leaves = NULL; /* entries at the depth cap: never expanded */
    node_t root;
    memset(&root, 0, sizeof(root));
    root.p = 1.0;
    if (heap_push(&q, root)) return ORC_ENOMEM;
    while (q.n > 0 && (uint64_t)(q.n + n_final) + 3 < t->bound) {
      node_t v = heap_pop(&q);
      for (int letter = 0; letter < 4; ++letter) {
        node_t c = v;
        c.code = v.code * 4 + (uint64_t)letter;
        c.depth = v.depth + 1;
        c.counts[letter]++;
        c.p = orc_canonical_product(t->q, c.counts);
        if (c.depth < cap) {
          if (heap_push(&q, c)) { free(q.a); free(final_leaves); return ORC_ENOMEM; }
        } else {
          if (n_final == cap_final) {
            cap_final = cap_final ? 2 * cap_final : 1024;
            node_t* nf = (node_t*)realloc(final_leaves, cap_final * sizeof(node_t));
            if (!nf) { free(q.a); free(final_leaves); return ORC_ENOMEM; }
            final_leaves = nf;
          }
          final_leaves[n_final++] = c;
        }
      }
    }
    n = q.n + n_final;
    leaves = (node_t*)malloc(n * sizeof(node_t));
    if (!leaves) { free(q.a); free(final_leaves); return ORC_ENOMEM; }
    if (q.n) memcpy(leaves, q.a, q.n * sizeof(node_t));
    if (n_final) memcpy(leaves + q.n, final_leaves, n_final * sizeof(node_t));
    free(q.a);
    free(final_leaves);
  }
  /* Tree order = order of left-aligned codes.  Key: lac << 32 | index. */
  uint64_t* key = (uint64_t*)malloc(n * sizeof(uint64_t));
  if (!key) { free(leaves); return ORC_ENOMEM; }
  for (size_t i = 0; i < n; ++i) {
    uint64_t lac = leaves[i].code << (2 * (ORC_MAX_CAP - leaves[i].depth));
    key[i] = (lac << 25) | (uint64_t)i; /* lac < 2^30, i < 2^25 */
  }
  qsort(key, n, sizeof(uint64_t), cmp_u64);
  uint64_t nb = 1;
  int b = 0;
  while (nb < n) { nb <<= 1; ++b; }
  t->n_items = n;
  t->n_buckets = nb;
  t->bucket_bits = b;
  t->capacity = 1ull << (32 - b);
  t->len = (uint8_t*)calloc(nb, 1);
  t->code = (uint64_t*)calloc(nb, sizeof(uint64_t));
  t->row = (uint32_t*)calloc(nb, sizeof(uint32_t));
  t->col = (uint32_t*)calloc(nb, sizeof(uint32_t));
  t->p = (double*)calloc(nb, sizeof(double));
  t->w = (int64_t*)calloc(nb, sizeof(int64_t));
  t->thr = (uint32_t*)calloc(nb, sizeof(uint32_t));
  t->alias = (uint32_t*)calloc(nb, sizeof(uint32_t));
  if (!t->len || !t->code || !t->row || !t->col || !t->p || !t->w || !t->thr ||
      !t->alias) {
    free(key); free(leaves);
    return ORC_ENOMEM;
  }
  for (size_t j = 0; j < n; ++j) {
    const node_t* v = &leaves[key[j] & ((1ull << 25) - 1)];
    t->len[j] = (uint8_t)v->depth;
    t->code[j] = v->code;
    t->p[j] = v->p;
    uint32_t r = 0, c = 0;
    for (int pos = v->depth - 1; pos >= 0; --pos) {
      unsigned digit = (unsigned)(v->code >> (2 * pos)) & 3u;
      r = (r << 1) | (digit >> 1);
      c = (c << 1) | (digit & 1u);
    }
    t->row[j] = r;
    t->col[j] = c;
  }
  free(key);
  free(leaves);
  (void)out_lac_sorted;
  return ORC_OK;
}

/* Reading R7: fixed-point weights summing to exactly 2^32, by largest
 * remainders.  x_j = p_j * 2^32 (exact scaling); every item gets floor(x_j);
 * the R = 2^32 - sum(floor(x_j)) units left over go one each to the R items
 * with the largest fractional parts x_j - floor(x_j), ties to the lower
 * index.  Every weight is within one unit of x_j. */
typedef struct {
  double frac;
  uint64_t index;
} frac_t;

static int cmp_frac(const void* x, const void* y) {
  const frac_t* a = (const frac_t*)x;
  const frac_t* b = (const frac_t*)y;
  if (a->frac != b->frac) return a->frac > b->frac ? -1 : 1;
  return a->index < b->index ? -1 : (a->index > b->index ? 1 : 0);
}

static int quantise(orc_table* t) {
  const double scale = 4294967296.0;
  const uint64_t n = t->n_items;
  frac_t* fr = (frac_t*)malloc(n * sizeof(frac_t));
  if (!fr) return ORC_ENOMEM;
  int64_t sum = 0;
  for (uint64_t j = 0; j < n; ++j) {
    double x = t->p[j] * scale;
    double fl = floor(x);
    t->w[j] = (int64_t)fl;
    sum += t->w[j];
    fr[j].frac = x - fl;
    fr[j].index = j;
  }
  int64_t residual = (int64_t)(1ull << 32) - sum;
  if (residual < 0 || (uint64_t)residual > n) { free(fr); return ORC_EINTERNAL; }
  qsort(fr, n, sizeof(frac_t), cmp_frac);
  for (int64_t r = 0; r < residual; ++r) t->w[fr[r].index] += 1;
  free(fr);
  return ORC_OK;
}

/* Reading R8: Walker's alias structure [Walker 1977] built by one sweep.
 * Lights (w < C) and heavies (w >= C) are each taken in ascending index
 * order.  The current heavy pays for each light's deficit; once the heavy's
 * remaining mass r drops below C, its own bucket gets threshold r and the
 * next heavy as alias, and the next heavy becomes current.  Every heavy left
 * at the end holds exactly C and aliases itself. */
static int build_alias(orc_table* t) {
  const uint64_t nb = t->n_buckets;
  const int64_t C = (int64_t)t->capacity;
  uint32_t* lights = (uint32_t*)malloc(nb * sizeof(uint32_t));
  uint32_t* heavies = (uint32_t*)malloc(nb * sizeof(uint32_t));
  if (!lights || !heavies) { free(lights); free(heavies); return ORC_ENOMEM; }
  uint64_t nl = 0, nh = 0;
  for (uint64_t i = 0; i < nb; ++i) {
    if (t->w[i] < C) lights[nl++] = (uint32_t)i;
    else heavies[nh++] = (uint32_t)i;
  }
  int rc = ORC_OK;
  if (nh == 0) { rc = ORC_EINTERNAL; goto done; }
  uint64_t h = 0;
  uint32_t j = heavies[0];
  int64_t r = t->w[j];
  for (uint64_t li = 0; li < nl; ++li) {
    uint32_t i = lights[li];
    t->thr[i] = (uint32_t)t->w[i];
    t->alias[i] = j;
    r -= C - t->w[i];
    while (r < C) {
      if (++h >= nh) { rc = ORC_EINTERNAL; goto done; }
      uint32_t jn = heavies[h];
      t->thr[j] = (uint32_t)r;
      t->alias[j] = jn;
      r = t->w[jn] - (C - r);
      j = jn;
    }
  }
  if (r != C) { rc = ORC_EINTERNAL; goto done; }
  t->thr[j] = (uint32_t)C;
  t->alias[j] = j;
  for (uint64_t hh = h + 1; hh < nh; ++hh) {
    uint32_t jj = heavies[hh];
    if (t->w[jj] != C) { rc = ORC_EINTERNAL; goto done; }
    t->thr[jj] = (uint32_t)C;
    t->alias[jj] = jj;
  }
done:
  free(lights);
  free(heavies);
  return rc;
}

int orc_build_table(double a, double b, double c, double d, int k,
                    uint64_t bound, int mode, orc_table* out) {
  memset(out, 0, sizeof(*out));
  double q[4] = {a, b, c, d};
  int rc = validate(q, k, bound, mode);
  if (rc) return rc;
  out->k = k;
  out->mode = mode;
  out->bound = bound;
  out->K = 2;
  memcpy(out->q, q, sizeof(q));
  if ((rc = enumerate_leaves(out, NULL)) != ORC_OK) { orc_free_table(out); return rc; }
  if ((rc = quantise(out)) != ORC_OK) { orc_free_table(out); return rc; }
  if ((rc = build_alias(out)) != ORC_OK) { orc_free_table(out); return rc; }
  return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Sampling (Sec. 2, the sampling loop, with readings R9-R12).
 * ---------------------------------------------------------------------- */
static void sample_letters(const orc_table* t, int k, uint32_t stream, uint64_t seed, uint64_t e,
                           uint64_t* src, uint64_t* dst, uint32_t* n_samples);

static void sample_edge(const orc_table* t, uint64_t seed, uint64_t e,
                        uint64_t* src, uint64_t* dst, uint32_t* n_samples) {
  sample_letters(t, t->k, 0u, seed, e, src, dst, n_samples);
}

/* k letters of one edge from counter stream (e_lo, e_hi, j, stream). */
static void sample_letters(const orc_table* t, int k, uint32_t stream, uint64_t seed, uint64_t e,
                           uint64_t* src, uint64_t* dst, uint32_t* n_samples) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const int b = t->bucket_bits;
  const uint32_t bmask = (uint32_t)(t->n_buckets - 1);
  uint64_t row = 0, col = 0;
  int filled = 0;
  uint32_t s = 0, words[4] = {0, 0, 0, 0};
  while (filled < k) {
    if ((s & 3u) == 0) {
      const uint32_t ctr[4] = {(uint32_t)e, (uint32_t)(e >> 32), s >> 2, stream};
      orc_philox4x32_10(ctr, key, words);
    }
    uint32_t x = words[s & 3u];
    ++s;
    uint32_t bucket = (x >> 4) & bmask;
    uint32_t f = (uint32_t)(((uint64_t)x >> (b + 4)) << 4) | (x & 15u);
    uint32_t item = (f < t->thr[bucket]) ? bucket : t->alias[bucket];
    int L = t->len[item];
    int take = (L < k - filled) ? L : (k - filled);
    if (t->K > 2) { /* base-K digits (R21): the leading `take` digits of the path */
      row = row * t->powK[take] + (uint64_t)t->row[item] / t->powK[L - take];
      col = col * t->powK[take] + (uint64_t)t->col[item] / t->powK[L - take];
    } else {
      row = (row << take) | (uint64_t)(t->row[item] >> (L - take));
      col = (col << take) | (uint64_t)(t->col[item] >> (L - take));
    }
    filled += take;
  }
  *src = row;
  *dst = col;
  if (n_samples) *n_samples = s;
}

/* ------------------------------------------------------------------------
 * Epilogue of Sec. 3 (reading R19): mirror to the upper triangle, scramble.
 * ---------------------------------------------------------------------- */
#define ORC_UNDIRECTED 1
#define ORC_SCRAMBLE 2

static int ids_fit_32(const orc_table* t);

/* SplitMix64: one step of the generator (state advanced in place). */
static uint64_t splitmix64_next(uint64_t* state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

typedef struct {
  uint64_t mul[3], add[3];
} scramble_t;

static scramble_t scramble_keys(uint64_t key) {
  scramble_t p;
  uint64_t st = key;
  for (int r = 0; r < 3; ++r) {
    p.mul[r] = splitmix64_next(&st) | 1ull;
    p.add[r] = splitmix64_next(&st);
  }
  return p;
}

static uint64_t scramble_id(const scramble_t* p, int k, uint64_t x) {
  const uint64_t mask = k >= 64 ? ~0ull : ((1ull << k) - 1);
  const int h = (k + 1) / 2;
  for (int r = 0; r < 3; ++r) {
    x = (x * p->mul[r] + p->add[r]) & mask;
    x ^= x >> h;
  }
  return x;
}

/* pi(x) for one id, for tests. */
uint64_t orc_scramble(int k, uint64_t key, uint64_t x) {
  scramble_t p = scramble_keys(key);
  return scramble_id(&p, k, x);
}

static void epilogue(int flags, const scramble_t* p, int k, uint64_t* s, uint64_t* d) {
  if ((flags & ORC_UNDIRECTED) && *s > *d) {
    uint64_t t = *s;
    *s = *d;
    *d = t;
  }
  if (flags & ORC_SCRAMBLE) {
    *s = scramble_id(p, k, *s);
    *d = scramble_id(p, k, *d);
  }
}

/* MurmurHash3's 64-bit finaliser (A. Appleby, public domain). */
static uint64_t fmix64(uint64_t z) {
  z ^= z >> 33;
  z *= 0xFF51AFD7ED558CCDull;
  z ^= z >> 33;
  z *= 0xC4CEB9FE1A85EC53ull;
  z ^= z >> 33;
  return z;
}

/* Per-edge checksum term of the chunk reduction. */
uint64_t orc_edge_mix(uint64_t e, uint64_t src, uint64_t dst) {
  uint64_t rot = (dst << 32) | (dst >> 32);
  return fmix64(e ^ fmix64(src ^ rot));
}

typedef struct {
  const orc_table* t;
  uint64_t seed, edge_begin, lo, hi;
  void* src;
  void* dst;
  int width; /* bytes per id: 4 or 8 */
  uint32_t* n_samples;
  int flags; /* ORC_UNDIRECTED | ORC_SCRAMBLE */
  scramble_t scr;
  /* reduction outputs */
  int hist_bits;
  uint64_t* hist;
  uint64_t xor_acc;
} work_t;

static void* gen_worker(void* arg) {
  work_t* w = (work_t*)arg;
  for (uint64_t slot = w->lo; slot < w->hi; ++slot) {
    uint64_t s, d;
    uint32_t ns;
    sample_edge(w->t, w->seed, w->edge_begin + slot, &s, &d, &ns);
    epilogue(w->flags, &w->scr, w->t->k, &s, &d);
    if (w->width == 4) {
      ((uint32_t*)w->src)[slot] = (uint32_t)s;
      ((uint32_t*)w->dst)[slot] = (uint32_t)d;
    } else {
      ((uint64_t*)w->src)[slot] = s;
      ((uint64_t*)w->dst)[slot] = d;
    }
    if (w->n_samples) w->n_samples[slot] = ns;
  }
  return NULL;
}

static void* reduce_worker(void* arg) {
  work_t* w = (work_t*)arg;
  int shift = w->t->k - w->hist_bits;
  for (uint64_t slot = w->lo; slot < w->hi; ++slot) {
    uint64_t e = w->edge_begin + slot, s, d;
    sample_edge(w->t, w->seed, e, &s, &d, NULL);
    w->hist[s >> shift] += 1;
    w->xor_acc ^= orc_edge_mix(e, s, d);
  }
  return NULL;
}

static int run_threads(work_t* proto, uint64_t m, int threads,
                       void* (*fn)(void*), work_t** out_items) {
  if (threads < 1) threads = 1;
  if ((uint64_t)threads > m && m > 0) threads = (int)m;
  if (m == 0) threads = 1;
  work_t* items = (work_t*)calloc((size_t)threads, sizeof(work_t));
  pthread_t* tid = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
  if (!items || !tid) { free(items); free(tid); return ORC_ENOMEM; }
  for (int i = 0; i < threads; ++i) {
    items[i] = *proto;
    items[i].lo = m * (uint64_t)i / (uint64_t)threads;
    items[i].hi = m * (uint64_t)(i + 1) / (uint64_t)threads;
  }
  for (int i = 1; i < threads; ++i) pthread_create(&tid[i], NULL, fn, &items[i]);
  fn(&items[0]);
  for (int i = 1; i < threads; ++i) pthread_join(tid[i], NULL);
  free(tid);
  *out_items = items;
  return threads;
}

/* Edges e in [edge_begin, edge_begin + m) go to slot e - edge_begin.
 * width is 4 (k <= 32) or 8 bytes per id.  flags: ORC_UNDIRECTED and/or
 * ORC_SCRAMBLE (with scramble_key), reading R19. */
int orc_generate_ex(const orc_table* t, uint64_t seed, uint64_t edge_begin,
                    uint64_t m, void* src, void* dst, int width,
                    uint32_t* n_samples, int threads, int flags, uint64_t scramble_key) {
  /* the last edge of the stream is 2^64 - 1 */
  if (m > 0 && edge_begin + (m - 1) < edge_begin) return ORC_ERANGE;
  if (width != 4 && width != 8) return ORC_EINVAL;
  if (width == 4 && !ids_fit_32(t)) return ORC_EINVAL;
  if (flags & ~(ORC_UNDIRECTED | ORC_SCRAMBLE)) return ORC_EINVAL;
  if ((flags & ORC_SCRAMBLE) && t->K > 2) return ORC_EINVAL; /* pi is defined on [0, 2^k) */
  if (m == 0) return ORC_OK;
  work_t proto;
  memset(&proto, 0, sizeof(proto));
  proto.t = t; proto.seed = seed; proto.edge_begin = edge_begin;
  proto.src = src; proto.dst = dst; proto.width = width;
  proto.n_samples = n_samples;
  proto.flags = flags;
  proto.scr = scramble_keys(scramble_key);
  work_t* items = NULL;
  int nt = run_threads(&proto, m, threads, gen_worker, &items);
  if (nt < 0) return nt;
  free(items);
  return ORC_OK;
}

int orc_generate(const orc_table* t, uint64_t seed, uint64_t edge_begin,
                 uint64_t m, void* src, void* dst, int width,
                 uint32_t* n_samples, int threads) {
  return orc_generate_ex(t, seed, edge_begin, m, src, dst, width, n_samples, threads, 0, 0);
}

/* Chunk reduction: histogram of the top hist_bits bits of each source id and
 * the XOR over edges of orc_edge_mix(e, src, dst). */
int orc_generate_reduce(const orc_table* t, uint64_t seed, uint64_t edge_begin,
                        uint64_t m, int hist_bits, uint64_t* hist,
                        uint64_t* xor_out, int threads) {
  if (m > 0 && edge_begin + (m - 1) < edge_begin) return ORC_ERANGE;
  if (hist_bits < 0 || hist_bits > t->k || hist_bits > 24 || t->K > 2) return ORC_EINVAL;
  uint64_t nbins = 1ull << hist_bits;
  memset(hist, 0, nbins * sizeof(uint64_t));
  *xor_out = 0;
  if (m == 0) return ORC_OK;
  work_t proto;
  memset(&proto, 0, sizeof(proto));
  proto.t = t; proto.seed = seed; proto.edge_begin = edge_begin;
  proto.hist_bits = hist_bits;
  if (threads < 1) threads = 1;
  /* each worker gets its own histogram */
  uint64_t* hists = (uint64_t*)calloc((size_t)threads * nbins, sizeof(uint64_t));
  if (!hists) return ORC_ENOMEM;
  if ((uint64_t)threads > m) threads = (int)m;
  work_t* items = (work_t*)calloc((size_t)threads, sizeof(work_t));
  pthread_t* tid = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
  if (!items || !tid) { free(hists); free(items); free(tid); return ORC_ENOMEM; }
  for (int i = 0; i < threads; ++i) {
    items[i] = proto;
    items[i].lo = m * (uint64_t)i / (uint64_t)threads;
    items[i].hi = m * (uint64_t)(i + 1) / (uint64_t)threads;
    items[i].hist = hists + (size_t)i * nbins;
  }
  for (int i = 1; i < threads; ++i) pthread_create(&tid[i], NULL, reduce_worker, &items[i]);
  reduce_worker(&items[0]);
  for (int i = 1; i < threads; ++i) pthread_join(tid[i], NULL);
  for (int i = 0; i < threads; ++i) {
    for (uint64_t bin = 0; bin < nbins; ++bin) hist[bin] += items[i].hist[bin];
    *xor_out ^= items[i].xor_acc;
  }
  free(hists); free(items); free(tid);
  return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Flat accessors for the ctypes wrapper.
 * ---------------------------------------------------------------------- */
/* ------------------------------------------------------------------------
 * Partitioned generation (Sec. 3, reading R20).
 * ---------------------------------------------------------------------- */
typedef struct {
  uint32_t key[2], ctr[4];
  uint32_t words[4];
  int used; /* uniforms taken from `words` (0, 1 or 2) */
} ustream_t;

static void ustream_init(ustream_t* u, uint64_t seed, uint32_t r, uint32_t c, int level) {
  u->key[0] = (uint32_t)seed;
  u->key[1] = (uint32_t)(seed >> 32);
  u->ctr[0] = r;
  u->ctr[1] = c;
  u->ctr[2] = 0;
  u->ctr[3] = 0x80000000u | (uint32_t)level;
  u->used = 2;
}

/* A uniform in [0, 1) with 53 random bits: two Philox words per uniform. */
static double uniform53(ustream_t* u) {
  if (u->used == 2) {
    orc_philox4x32_10(u->ctr, u->key, u->words);
    u->ctr[2] += 1;
    u->used = 0;
  }
  const uint64_t hi = u->words[2 * u->used], lo = u->words[2 * u->used + 1];
  u->used += 1;
  return (double)(((hi << 32) | lo) >> 11) * (1.0 / 9007199254740992.0);
}

/* Bin(n, p), 0 < p <= 1/2, by inversion (n p < 30): walk the pmf upwards
 * from f(0) = (1-p)^n with f(x)/f(x-1) = ((n+1) p/(1-p)) / x - p/(1-p). */
static uint64_t binomial_inversion(ustream_t* us, uint64_t n, double p) {
  const double q = 1.0 - p, s = p / q, a = ((double)n + 1.0) * s;
  const double f0 = pow(q, (double)n);
  for (;;) {
    double u = uniform53(us), f = f0;
    uint64_t x = 0;
    int restart = 0;
    while (u > f) {
      u -= f;
      x += 1;
      if (x > n || x > 110) { restart = 1; break; }
      f *= a / (double)x - s;
    }
    if (!restart) return x;
  }
}

/* Stirling-series remainder of ln(x!) at x + 1 = a: 1/(12a) - 1/(360a^3) + ... */
static double stirling_tail(double a) {
  const double a2 = a * a;
  return (13860.0 - (462.0 - (132.0 - (99.0 - 140.0 / a2) / a2) / a2) / a2) / a / 166320.0;
}

/* Bin(n, p), 0 < p <= 1/2, n p >= 30: BTPE (triangle, parallelogram and two
 * exponential tails over the pmf, squeeze, then the exact ratio). */
static uint64_t binomial_btpe(ustream_t* us, uint64_t n, double p) {
  const double dn = (double)n, r = p, q = 1.0 - p;
  const double nrq = dn * r * q;
  const double fm = dn * r + r;
  const double M = floor(fm);
  const double p1 = floor(2.195 * sqrt(nrq) - 4.6 * q) + 0.5;
  const double xm = M + 0.5, xl = xm - p1, xr = xm + p1;
  const double c = 0.134 + 20.5 / (15.3 + M);
  double a = (fm - xl) / (fm - xl * r);
  const double laml = a * (1.0 + a / 2.0);
  a = (xr - fm) / (xr * q);
  const double lamr = a * (1.0 + a / 2.0);
  const double p2 = p1 * (1.0 + 2.0 * c), p3 = p2 + c / laml, p4 = p3 + c / lamr;
  for (;;) {
    const double u = uniform53(us) * p4;
    double v = uniform53(us), y;
    if (u <= p1) { /* triangle: accept at once */
      return (uint64_t)floor(xm - p1 * v + u);
    }
    if (u <= p2) { /* parallelogram */
      const double x = xl + (u - p1) / c;
      v = v * c + 1.0 - fabs(M - x + 0.5) / p1;
      if (v > 1.0) continue;
      y = floor(x);
    } else if (u <= p3) { /* left exponential tail */
      y = floor(xl + log(v) / laml);
      if (y < 0.0) continue;
      v = v * (u - p2) * laml;
    } else { /* right exponential tail */
      y = floor(xr - log(v) / lamr);
      if (y > dn) continue;
      v = v * (u - p3) * lamr;
    }
    const double k = fabs(y - M);
    if (k <= 20.0 || k >= nrq / 2.0 - 1.0) {
      /* f(y) / f(M) by the pmf recurrence */
      const double s = r / q, aa = s * (dn + 1.0);
      double F = 1.0;
      if (M < y) {
        for (double i = M + 1.0; i <= y; i += 1.0) F *= aa / i - s;
      } else if (M > y) {
        for (double i = y + 1.0; i <= M; i += 1.0) F /= aa / i - s;
      }
      if (v <= F) return (uint64_t)y;
      continue;
    }
    /* squeeze on ln f(y) / f(M) */
    const double rho = (k / nrq) * ((k * (k / 3.0 + 0.625) + 0.1666666666666) / nrq + 0.5);
    const double tt = -k * k / (2.0 * nrq);
    const double A = log(v);
    if (A < tt - rho) return (uint64_t)y;
    if (A > tt + rho) continue;
    /* the exact bound with Stirling's series for the four factorials */
    const double x1 = y + 1.0, f1 = M + 1.0, z = dn + 1.0 - M, w = dn - y + 1.0;
    const double bound = xm * log(f1 / x1) + (dn - M + 0.5) * log(z / w) + (y - M) * log(w * r / (x1 * q)) +
                         stirling_tail(f1) + stirling_tail(z) - stirling_tail(x1) - stirling_tail(w);
    if (A <= bound) return (uint64_t)y;
  }
}

static uint64_t binomial(ustream_t* us, uint64_t n, double p) {
  if (n == 0 || p <= 0.0) return 0;
  if (p >= 1.0) return n;
  const int flip = p > 0.5;
  const double pp = flip ? 1.0 - p : p;
  const uint64_t x = ((double)n * pp < 30.0) ? binomial_inversion(us, n, pp) : binomial_btpe(us, n, pp);
  return flip ? n - x : x;
}

/* Bin(n, p) from the stream of node (level, r, c), for tests. */
uint64_t orc_binomial(uint64_t seed, uint32_t r, uint32_t c, int level, uint64_t n, double p) {
  ustream_t us;
  ustream_init(&us, seed, r, c, level);
  return binomial(&us, n, p);
}

/* Counts of the quadrant children of node (level, r, c) holding n edges. */
static void split4(const double q[4], uint64_t seed, int level, uint32_t r, uint32_t c, uint64_t n,
                   uint64_t out[4]) {
  ustream_t us;
  ustream_init(&us, seed, r, c, level);
  const double bcd = q[1] + q[2] + q[3], cd = q[2] + q[3];
  out[0] = binomial(&us, n, q[0]);
  uint64_t rest = n - out[0];
  out[1] = binomial(&us, rest, bcd > 0.0 ? q[1] / bcd : 0.0);
  rest -= out[1];
  out[2] = binomial(&us, rest, cd > 0.0 ? q[2] / cd : 0.0);
  out[3] = rest - out[2];
}

static void partition_rec(const double q[4], uint64_t seed, int t, int level, uint32_t r, uint32_t c,
                          uint64_t n, uint32_t row_begin, uint32_t row_end, uint64_t* counts) {
  if (level == t) {
    counts[(uint64_t)(r - row_begin) << t | c] = n;
    return;
  }
  if (n == 0) return; /* counts start at zero */
  uint64_t ch[4];
  split4(q, seed, level, r, c, n, ch);
  for (int quad = 0; quad < 4; ++quad) {
    const uint32_t cr = 2 * r + (uint32_t)(quad >> 1), cc = 2 * c + (uint32_t)(quad & 1);
    /* tile rows under the child: [cr, cr + 1) << (t - level - 1) */
    const int sh = t - level - 1;
    const uint64_t lo = (uint64_t)cr << sh, hi = (uint64_t)(cr + 1) << sh;
    if (hi <= row_begin || lo >= row_end) continue;
    partition_rec(q, seed, t, level + 1, cr, cc, ch[quad], row_begin, row_end, counts);
  }
}

/* Edge counts of the tiles in tile rows [row_begin, row_end): row-major,
 * (row_end - row_begin) x 2^t entries.  1 <= t <= min(k - 1, 15). */
int orc_partition_counts(const orc_table* t, uint64_t seed, uint64_t m, int tbits,
                         uint32_t row_begin, uint32_t row_end, uint64_t* counts) {
  if (tbits < 1 || tbits > 15 || tbits >= t->k || t->K > 2) return ORC_EINVAL;
  if (row_begin >= row_end || row_end > (1u << tbits)) return ORC_EINVAL;
  if (m > (1ull << 53)) return ORC_EINVAL;
  memset(counts, 0, sizeof(uint64_t) * ((uint64_t)(row_end - row_begin) << tbits));
  partition_rec(t->q, seed, tbits, 0, 0, 0, m, row_begin, row_end, counts);
  return ORC_OK;
}

/* All edges of the tiles in tile rows [row_begin, row_end), tile by tile in
 * row-major order, edge j of a tile in slot offset(tile) + j. */
int orc_generate_partition(const orc_table* t, uint64_t seed, uint64_t m, int tbits,
                           uint32_t row_begin, uint32_t row_end, void* src, void* dst, int width,
                           const uint64_t* counts) {
  if (tbits < 1 || tbits > 15 || tbits >= t->k) return ORC_EINVAL;
  if (width != 4 && width != 8) return ORC_EINVAL;
  if (width == 4 && t->k > 32) return ORC_EINVAL;
  const int kk = t->k - tbits;
  uint64_t slot = 0;
  for (uint32_t r = row_begin; r < row_end; ++r) {
    for (uint32_t c = 0; c < (1u << tbits); ++c) {
      const uint64_t n = counts[(uint64_t)(r - row_begin) << tbits | c];
      const uint32_t stream = 1u + ((r << tbits) | c);
      for (uint64_t j = 0; j < n; ++j, ++slot) {
        uint64_t s, d;
        sample_letters(t, kk, stream, seed, j, &s, &d, NULL);
        s |= (uint64_t)r << kk;
        d |= (uint64_t)c << kk;
        if (width == 4) {
          ((uint32_t*)src)[slot] = (uint32_t)s;
          ((uint32_t*)dst)[slot] = (uint32_t)d;
        } else {
          ((uint64_t*)src)[slot] = s;
          ((uint64_t*)dst)[slot] = d;
        }
      }
    }
  }
  (void)m;
  return ORC_OK;
}

/* ------------------------------------------------------------------------
 * K x K stochastic Kronecker initiators (Sec. 3, reading R21): the same
 * table over the K^2 cells of the initiator.  Letter x = K i + j is cell
 * (i, j): row digit i, column digit j; ids are base-K numbers of k digits.
 * ---------------------------------------------------------------------- */
#define KRON_MAX_LETTERS 256

typedef struct {
  double p;
  uint64_t code; /* base-K^2 digits, root-most letter most significant */
  int depth;
  uint8_t counts[KRON_MAX_LETTERS];
} knode_t;

static int knode_before(const knode_t* u, const knode_t* v) {
  if (u->p != v->p) return u->p > v->p;
  if (u->depth != v->depth) return u->depth < v->depth;
  return u->code < v->code;
}

typedef struct {
  knode_t* a;
  size_t n, cap;
} kheap_t;

static int kheap_push(kheap_t* h, const knode_t* v) {
  if (h->n == h->cap) {
    size_t nc = h->cap ? 2 * h->cap : 256;
    knode_t* na = (knode_t*)realloc(h->a, nc * sizeof(knode_t));
    if (!na) return ORC_ENOMEM;
    h->a = na;
    h->cap = nc;
  }
  size_t i = h->n++;
  h->a[i] = *v;
  while (i > 0) {
    size_t parent = (i - 1) / 2;
    if (!knode_before(&h->a[i], &h->a[parent])) break;
    knode_t tmp = h->a[i]; h->a[i] = h->a[parent]; h->a[parent] = tmp;
    i = parent;
  }
  return ORC_OK;
}

static void kheap_pop(kheap_t* h, knode_t* top) {
  *top = h->a[0];
  h->a[0] = h->a[--h->n];
  size_t i = 0;
  for (;;) {
    size_t l = 2 * i + 1, r = l + 1, best = i;
    if (l < h->n && knode_before(&h->a[l], &h->a[best])) best = l;
    if (r < h->n && knode_before(&h->a[r], &h->a[best])) best = r;
    if (best == i) break;
    knode_t tmp = h->a[i]; h->a[i] = h->a[best]; h->a[best] = tmp;
    i = best;
  }
}

/* 1.0 times each letter's probability n_x times, letters in order x = 0, 1, ... */
static double kron_product(const double* P, int letters, const uint8_t* counts) {
  double p = 1.0;
  for (int x = 0; x < letters; ++x)
    for (int i = 0; i < counts[x]; ++i) p = p * P[x];
  return p;
}

/* The largest L with K^L <= 2^15: a path's row (column) value fits 15 bits. */
static int kron_cap(int K) {
  int L = 0;
  uint64_t v = 1;
  while (v * (uint64_t)K <= 32768u) { v *= (uint64_t)K; ++L; }
  return L;
}

int orc_kron_build_table(const double* P, int K, int k, uint64_t bound, int mode, orc_table* out) {
  memset(out, 0, sizeof(*out));
  if (K < 2 || K > 16) return ORC_EINVAL;
  const int letters = K * K;
  double s = 0.0;
  for (int x = 0; x < letters; ++x) {
    if (!(P[x] >= 0.0) || isnan(P[x]) || isinf(P[x])) return ORC_EINVAL;
    s += P[x];
  }
  if (fabs(s - 1.0) > 1e-9) return ORC_EINVAL;
  /* n = K^k node ids must fit 64 bits */
  if (k < 1) return ORC_EINVAL;
  {
    unsigned __int128 n = 1;
    for (int i = 0; i < k; ++i) { n *= (unsigned)K; if (n > ((unsigned __int128)1 << 64)) return ORC_EINVAL; }
  }
  if (bound > (1ull << 24)) return ORC_EINVAL;
  if (mode == ORC_VARIABLE) {
    if (bound < (uint64_t)letters + 1) return ORC_EINVAL;
  } else if (mode == ORC_FIXED) {
    if (bound < (uint64_t)letters) return ORC_EINVAL;
  } else {
    return ORC_EINVAL;
  }
  out->k = k;
  out->mode = mode;
  out->bound = bound;
  out->K = K;
  out->powK[0] = 1;
  for (int i = 1; i < 16; ++i) out->powK[i] = out->powK[i - 1] * (uint64_t)K;
  const int cap = kron_cap(K) < k ? kron_cap(K) : k;
  out->cap = cap;
  size_t n = 0;
  knode_t* leaves = NULL;
  if (mode == ORC_FIXED) {
    int ell = 0;
    uint64_t sz = 1;
    while (sz * (uint64_t)letters <= bound) { sz *= (uint64_t)letters; ++ell; }
    if (ell < 1 || ell > cap) { orc_free_table(out); return ORC_EINVAL; }
    n = (size_t)sz;
    leaves = (knode_t*)calloc(n, sizeof(knode_t));
    if (!leaves) return ORC_ENOMEM;
    for (size_t code = 0; code < n; ++code) {
      knode_t* v = &leaves[code];
      v->code = code;
      v->depth = ell;
      uint64_t c = code;
      for (int pos = 0; pos < ell; ++pos) { v->counts[c % (uint64_t)letters]++; c /= (uint64_t)letters; }
      v->p = kron_product(P, letters, v->counts);
    }
  } else {
    kheap_t q = {0, 0, 0};
    size_t n_final = 0, cap_final = 0;
    knode_t* final_leaves = NULL;
    knode_t root;
    memset(&root, 0, sizeof(root));
    root.p = 1.0;
    if (kheap_push(&q, &root)) return ORC_ENOMEM;
    while (q.n > 0 && (uint64_t)(q.n + n_final) + (uint64_t)(letters - 1) < bound) {
      knode_t v;
      kheap_pop(&q, &v);
      for (int x = 0; x < letters; ++x) {
        knode_t c = v;
        c.code = v.code * (uint64_t)letters + (uint64_t)x;
        c.depth = v.depth + 1;
        c.counts[x]++;
        c.p = kron_product(P, letters, c.counts);
        if (c.depth < cap) {
          if (kheap_push(&q, &c)) { free(q.a); free(final_leaves); return ORC_ENOMEM; }
        } else {
          if (n_final == cap_final) {
            cap_final = cap_final ? 2 * cap_final : 256;
            knode_t* nf = (knode_t*)realloc(final_leaves, cap_final * sizeof(knode_t));
            if (!nf) { free(q.a); free(final_leaves); return ORC_ENOMEM; }
            final_leaves = nf;
          }
          final_leaves[n_final++] = c;
        }
      }
    }
    n = q.n + n_final;
    leaves = (knode_t*)malloc(n * sizeof(knode_t));
    if (!leaves) { free(q.a); free(final_leaves); return ORC_ENOMEM; }
    if (q.n) memcpy(leaves, q.a, q.n * sizeof(knode_t));
    if (n_final) memcpy(leaves + q.n, final_leaves, n_final * sizeof(knode_t));
    free(q.a);
    free(final_leaves);
  }
  if (n > (1u << 25)) { free(leaves); return ORC_EINVAL; }
  /* tree order: left-aligned codes, code * letters^(cap - depth) */
  uint64_t* lac = (uint64_t*)malloc(n * sizeof(uint64_t));
  uint64_t* key = (uint64_t*)malloc(n * sizeof(uint64_t));
  if (!lac || !key) { free(lac); free(key); free(leaves); return ORC_ENOMEM; }
  for (size_t i = 0; i < n; ++i) {
    uint64_t v = leaves[i].code;
    for (int d = leaves[i].depth; d < cap; ++d) v *= (uint64_t)letters;
    lac[i] = v;
  }
  /* sort indices by lac (insertion into a key of lac rank: lac < letters^cap <= 2^30) */
  for (size_t i = 0; i < n; ++i) key[i] = (lac[i] << 25) | (uint64_t)i;
  qsort(key, n, sizeof(uint64_t), cmp_u64);
  free(lac);
  uint64_t nb = 1;
  int b = 0;
  while (nb < n) { nb <<= 1; ++b; }
  out->n_items = n;
  out->n_buckets = nb;
  out->bucket_bits = b;
  out->capacity = 1ull << (32 - b);
  out->len = (uint8_t*)calloc(nb, 1);
  out->code = (uint64_t*)calloc(nb, sizeof(uint64_t));
  out->row = (uint32_t*)calloc(nb, sizeof(uint32_t));
  out->col = (uint32_t*)calloc(nb, sizeof(uint32_t));
  out->p = (double*)calloc(nb, sizeof(double));
  out->w = (int64_t*)calloc(nb, sizeof(int64_t));
  out->thr = (uint32_t*)calloc(nb, sizeof(uint32_t));
  out->alias = (uint32_t*)calloc(nb, sizeof(uint32_t));
  if (!out->len || !out->code || !out->row || !out->col || !out->p || !out->w || !out->thr || !out->alias) {
    free(key); free(leaves); orc_free_table(out);
    return ORC_ENOMEM;
  }
  for (size_t j = 0; j < n; ++j) {
    const knode_t* v = &leaves[key[j] & ((1ull << 25) - 1)];
    out->len[j] = (uint8_t)v->depth;
    out->code[j] = v->code;
    out->p[j] = v->p;
    /* row / column values: the path's digits, root-most most significant */
    uint64_t r = 0, c = 0, digits[16];
    uint64_t code = v->code;
    for (int pos = 0; pos < v->depth; ++pos) { digits[pos] = code % (uint64_t)letters; code /= (uint64_t)letters; }
    for (int pos = v->depth - 1; pos >= 0; --pos) {
      r = r * (uint64_t)K + digits[pos] / (uint64_t)K;
      c = c * (uint64_t)K + digits[pos] % (uint64_t)K;
    }
    out->row[j] = (uint32_t)r;
    out->col[j] = (uint32_t)c;
  }
  free(key);
  free(leaves);
  int rc;
  if ((rc = quantise(out)) != ORC_OK) { orc_free_table(out); return rc; }
  if ((rc = build_alias(out)) != ORC_OK) { orc_free_table(out); return rc; }
  return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Perturbed tables (Sec. 3, reading R22).
 * ---------------------------------------------------------------------- */
int orc_perturbed_params(double a, double b, double c, double d, int n_tables, double eps,
                         uint64_t seed, double* out /* n_tables x 4 */) {
  if (n_tables < 1 || n_tables > 64 || (n_tables & (n_tables - 1))) return ORC_EINVAL;
  if (!(eps >= 0.0 && eps < 1.0)) return ORC_EINVAL;
  const double q[4] = {a, b, c, d};
  uint64_t st = seed;
  for (int i = 0; i < n_tables; ++i) {
    double v[4];
    for (int x = 0; x < 4; ++x) {
      const double u = (double)(splitmix64_next(&st) >> 11) * (1.0 / 9007199254740992.0);
      v[x] = q[x] * (1.0 + eps * (2.0 * u - 1.0));
    }
    const double s = v[0] + v[1] + v[2] + v[3];
    for (int x = 0; x < 4; ++x) out[4 * i + x] = v[x] / s;
  }
  return ORC_OK;
}

/* Edges of a set of tables: edge e from tables[e mod n_tables]. */
int orc_generate_set(const orc_table* const* tables, int n_tables, uint64_t seed, uint64_t edge_begin,
                     uint64_t m, void* src, void* dst, int width) {
  if (m > 0 && edge_begin + (m - 1) < edge_begin) return ORC_ERANGE;
  if (n_tables < 1 || (n_tables & (n_tables - 1))) return ORC_EINVAL;
  for (uint64_t slot = 0; slot < m; ++slot) {
    const uint64_t e = edge_begin + slot;
    const orc_table* t = tables[e & (uint64_t)(n_tables - 1)];
    uint64_t s, d;
    sample_edge(t, seed, e, &s, &d, NULL);
    if (width == 4) {
      ((uint32_t*)src)[slot] = (uint32_t)s;
      ((uint32_t*)dst)[slot] = (uint32_t)d;
    } else {
      ((uint64_t*)src)[slot] = s;
      ((uint64_t*)dst)[slot] = d;
    }
  }
  return ORC_OK;
}

orc_table* orc_table_new(void) { return (orc_table*)calloc(1, sizeof(orc_table)); }
void orc_table_delete(orc_table* t) { orc_free_table(t); free(t); }

/* info[0..7] = k, mode, cap, bucket_bits, n_items, n_buckets, capacity, K */
void orc_table_info(const orc_table* t, uint64_t info[8]) {
  info[0] = (uint64_t)t->k; info[1] = (uint64_t)t->mode;
  info[2] = (uint64_t)t->cap; info[3] = (uint64_t)t->bucket_bits;
  info[4] = t->n_items; info[5] = t->n_buckets; info[6] = t->capacity;
  info[7] = (uint64_t)t->K;
}

/* Do the ids of this table fit 32 bits (2^k, or K^k, at most 2^32)? */
static int ids_fit_32(const orc_table* t) {
  if (t->K <= 2) return t->k <= 32;
  uint64_t n = 1;
  for (int i = 0; i < t->k; ++i) {
    n *= (uint64_t)t->K;
    if (n > (1ull << 32)) return 0;
  }
  return 1;
}

/* Copies the per-item and per-bucket arrays (n_buckets entries each). */
void orc_table_arrays(const orc_table* t, uint8_t* len, uint64_t* code,
                      uint32_t* row, uint32_t* col, double* p, int64_t* w,
                      uint32_t* thr, uint32_t* alias) {
  size_t nb = (size_t)t->n_buckets;
  if (len) memcpy(len, t->len, nb);
  if (code) memcpy(code, t->code, nb * sizeof(uint64_t));
  if (row) memcpy(row, t->row, nb * sizeof(uint32_t));
  if (col) memcpy(col, t->col, nb * sizeof(uint32_t));
  if (p) memcpy(p, t->p, nb * sizeof(double));
  if (w) memcpy(w, t->w, nb * sizeof(int64_t));
  if (thr) memcpy(thr, t->thr, nb * sizeof(uint32_t));
  if (alias) memcpy(alias, t->alias, nb * sizeof(uint32_t));
}
