// table_build.hip -- builds the path table and its alias structure on the GPU.
//
// One 1024-thread workgroup builds one table, so a batch of tables is a
// single launch.  The result is bit-identical to the sequential definition
// (Sec. 2: the max-priority queue that always expands the most probable path,
// then a Walker alias table), reached by a data-parallel route:
//
//  0. All nodes with the same letter counts share one probability, so every
//     probability the build needs is one of 3876 classes (depth <= 15),
//     tabulated once in LDS with the sequential rounding of the definition.
//  1. The queue expands nodes in a fixed total order (probability descending,
//     then depth, then base-4 code), and a node never precedes its parent in
//     that order, so the expanded set is exactly the first t nodes of the
//     order.  The t-th node is found by a radix select over the classes'
//     probability bits weighted by their node counts (stopping once the group
//     left holds one probability), then a walk over the digits of the codes
//     inside the last, partly expanded class group.  Expansion is then a test
//     against that boundary node.  (Sec. 3, Parallelization, notes the same
//     idea: expand every entry above a probability threshold.)
//  2. The tree is expanded level by level with block-wide prefix sums;
//     subtree leaf counts (bottom-up) and leaf offsets (top-down) place every
//     leaf at its tree-order index without sorting.
//  3. Weights p * 2^32 are rounded by largest remainders: floors, then a
//     radix select of the residual's worth of largest fractional parts (the
//     keys in LDS for tables of up to 10240 items).
//  4. The alias sweep (lights and heavies in index order, the current heavy
//     paying for each light) is evaluated in closed form from two prefix
//     sums: light i aliases the first heavy whose cumulative excess reaches
//     the lights' cumulative deficit before i, and a heavy whose cumulative
//     excess E falls short of the total deficit keeps C + E - D(i) where
//     D(i) is the first cumulative deficit above E, aliasing the next heavy.
//     The binary searches run over LDS for tables of up to 10240 buckets.
//     Sec. 3 cites a parallel construction of the same kind [HubSan19].
#include "rmat_internal.h"

namespace rmat {
namespace {

constexpr int kWaves = kBuildThreads / 64;

// ---------------------------------------------------------------- helpers --
__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int d) {
  uint32_t lo = __shfl_up(static_cast<uint32_t>(v), d, 64);
  uint32_t hi = __shfl_up(static_cast<uint32_t>(v >> 32), d, 64);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int d) {
  uint32_t lo = __shfl_xor(static_cast<uint32_t>(v), d, 64);
  uint32_t hi = __shfl_xor(static_cast<uint32_t>(v >> 32), d, 64);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Exclusive prefix sum over the workgroup; *total gets the sum of all v.
__device__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* s_warp, uint64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t y = shfl_up_u64(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_warp[wave] = x;
  __syncthreads();
  if (wave == 0) {
    uint64_t y = lane < kWaves ? s_warp[lane] : 0;
#pragma unroll
    for (int d = 1; d < kWaves; d <<= 1) {
      uint64_t z = shfl_up_u64(y, d);
      if (lane >= d) y += z;
    }
    if (lane < kWaves) s_warp[lane] = y;
  }
  __syncthreads();
  uint64_t base = wave > 0 ? s_warp[wave - 1] : 0;
  *total = s_warp[kWaves - 1];
  __syncthreads();
  return base + x - v;
}

__device__ uint64_t block_sum(uint64_t v, uint64_t* s_warp) {
  uint64_t total;
  block_exclusive_scan(v, s_warp, &total);
  return total;
}

// Exclusive prefix sum over the workgroup of values below 2^kBits: a wave
// counts the values' bit planes with ballots (no shuffles), the waves' totals
// pass through LDS (two barriers).  *total gets the sum of all values.
template <int kBits>
__device__ __forceinline__ uint32_t block_scan_small(uint32_t v, uint32_t* total) {
  __shared__ uint32_t s_tot[kWaves];
  const int wave = threadIdx.x >> 6;
  uint32_t below = 0, wave_sum = 0;
#pragma unroll
  for (int b = 0; b < kBits; ++b) {
    const uint64_t m = __ballot((v >> b) & 1u);
    below += __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                       __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u)) << b;
    wave_sum += static_cast<uint32_t>(__popcll(m)) << b;
  }
  const int lane = threadIdx.x & 63;
  if (lane == 0) s_tot[wave] = wave_sum;
  __syncthreads();
  // lane w < kWaves: the inclusive sum of the totals of waves 0..w
  uint32_t incl = lane < kWaves ? s_tot[lane] : 0u;
#pragma unroll
  for (int d = 1; d < kWaves; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  __syncthreads();
  *total = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(incl), kWaves - 1));
  const uint32_t base = wave > 0 ? static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(incl), wave - 1)) : 0u;
  return base + below;
}

// Whether the keys of a radix select's current group are all one value,
// without atomics: each lane tracks the first group key it saw (rep) and
// whether another differed; a wave writes one verdict (0: no keys, 1: all its
// keys equal its rep, 2: mixed) and, after a barrier, every thread combines
// the waves' verdicts.
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  return static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), l))) |
         (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v >> 32), l))) << 32);
}

__device__ __forceinline__ void vote_uniform(uint64_t rep, bool has, bool differ, uint64_t* s_rep,
                                             uint32_t* s_state) {
  const uint64_t hb = __ballot(has);
  uint32_t state = 0;
  uint64_t wrep = 0;
  if (hb != 0) {
    wrep = readlane_u64(rep, __builtin_ctzll(hb));
    state = __ballot(differ || (has && rep != wrep)) != 0 ? 2u : 1u;
  }
  if ((threadIdx.x & 63) == 0) {
    s_state[threadIdx.x >> 6] = state;
    s_rep[threadIdx.x >> 6] = wrep;
  }
}

__device__ __forceinline__ bool group_uniform(const uint64_t* s_rep, const uint32_t* s_state, uint64_t* only) {
  const int lane = threadIdx.x & 63;
  const uint32_t st = lane < kWaves ? s_state[lane] : 0u;
  const uint64_t r = lane < kWaves ? s_rep[lane] : 0;
  const uint64_t with = __ballot(st != 0);
  if (with == 0) return false;
  const uint64_t r0 = readlane_u64(r, __builtin_ctzll(with));
  *only = r0;
  return __ballot(st == 2 || (st == 1 && r != r0)) == 0;
}

// Two exclusive 64-bit prefix sums over the workgroup in one pass (two
// barriers for both); *ta and *tb get the sums of all a and all b.
__device__ void block_exclusive_scan2(uint64_t a, uint64_t b, uint64_t* pa, uint64_t* pb, uint64_t* ta,
                                      uint64_t* tb) {
  __shared__ uint64_t s_w2[2 * kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t x = a, y = b;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t xu = shfl_up_u64(x, d), yu = shfl_up_u64(y, d);
    if (lane >= d) {
      x += xu;
      y += yu;
    }
  }
  if (lane == 63) {
    s_w2[wave] = x;
    s_w2[kWaves + wave] = y;
  }
  __syncthreads();
  // lane w < kWaves: the inclusive sums of the totals of waves 0..w
  uint64_t wx = lane < kWaves ? s_w2[lane] : 0, wy = lane < kWaves ? s_w2[kWaves + lane] : 0;
#pragma unroll
  for (int d = 1; d < kWaves; d <<= 1) {
    const uint64_t xu = shfl_up_u64(wx, d), yu = shfl_up_u64(wy, d);
    if (lane >= d) {
      wx += xu;
      wy += yu;
    }
  }
  __syncthreads();
  auto lane_u64 = [](uint64_t v, int l) {
    return static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), l))) |
           (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v >> 32), l)))
            << 32);
  };
  *ta = lane_u64(wx, kWaves - 1);
  *tb = lane_u64(wy, kWaves - 1);
  *pa = (wave > 0 ? lane_u64(wx, wave - 1) : 0) + x - a;
  *pb = (wave > 0 ? lane_u64(wy, wave - 1) : 0) + y - b;
}

__device__ uint32_t block_min_max(uint32_t vmin, uint32_t vmax, uint32_t* s_u32, uint32_t* out_max) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    vmin = min(vmin, static_cast<uint32_t>(__shfl_xor(vmin, d, 64)));
    vmax = max(vmax, static_cast<uint32_t>(__shfl_xor(vmax, d, 64)));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { s_u32[wave] = vmin; s_u32[kWaves + wave] = vmax; }
  __syncthreads();
  uint32_t mn = 0xFFFFFFFFu, mx = 0;
  for (int w = 0; w < kWaves; ++w) { mn = min(mn, s_u32[w]); mx = max(mx, s_u32[kWaves + w]); }
  __syncthreads();
  *out_max = mx;
  return mn;
}

// Radix-select step, run by one wave: walks 256 histogram bins from bin 255
// down to bin 0 and returns the bin in which the running count reaches
// `need` (bin 0 if it never does), with `need` reduced by the counts of the
// bins passed.  Lane L owns bins 255 - 4L .. 252 - 4L.
template <typename Count>
__device__ uint32_t wave_select_desc(const Count* hist, uint64_t* need) {
  const int lane = threadIdx.x & 63;
  uint64_t c[4], own = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    c[i] = hist[255 - 4 * lane - i];
    own += c[i];
  }
  uint64_t incl = own;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = shfl_up_u64(incl, d);
    if (lane >= d) incl += y;
  }
  const uint64_t want = *need;
  const uint64_t hit = __ballot(incl >= want);
  // the first lane whose range reaches `want`; none: every bin is passed
  // down to bin 0, which takes the remainder
  const int f = hit ? __builtin_ctzll(hit) : 63;
  const uint64_t before = __shfl(static_cast<uint32_t>(incl - own), f, 64) |
                          (static_cast<uint64_t>(__shfl(static_cast<uint32_t>((incl - own) >> 32), f, 64)) << 32);
  uint64_t rest = want - before;
  uint32_t bin = 0;
  if (lane == f) {
    int i = 0;
    for (; i < 3; ++i) {
      if (rest <= c[i]) break;
      rest -= c[i];
    }
    bin = 255 - 4 * f - i;
  }
  bin = __shfl(bin, f, 64);
  const uint32_t rlo = __shfl(static_cast<uint32_t>(rest), f, 64);
  const uint32_t rhi = __shfl(static_cast<uint32_t>(rest >> 32), f, 64);
  *need = (static_cast<uint64_t>(rhi) << 32) | rlo;
  return bin;
}

// Path probabilities by letter-count class.  A path's probability is 1.0
// times a (na times), then b, c, d, rounding after every product, so it
// depends only on the class (na, nb, nc, nd); the build tabulates every class
// of depth <= kMaxDepthCap once, in LDS.  Classes sit in rows, one row per
// (na, nb, nc) with na + nb + nc <= 15 in lexicographic order, holding
// nd = 0 .. 15 - na - nb - nc; rows[(na * 16 + nb) * 16 + nc] is the row's
// first slot.  Along a row each entry is the previous one times d, which is
// the same rounded product as the chain from 1.0.
constexpr int kClassRows = 816;     // triples with na + nb + nc <= 15: C(18, 3)
constexpr int kClassSlots = 3876;   // classes of depth <= 15: C(19, 4)
static_assert(kClassSlots <= kMaxClasses, "class slots exceed the class arrays");
static_assert(kMaxDepthCap == 15, "the class rows cover depths up to 15");

__device__ __forceinline__ uint32_t class_slot(const uint16_t* rows, int na, int nb, int nc, int nd) {
  return rows[(na * 16 + nb) * 16 + nc] + static_cast<uint32_t>(nd);
}

// Row bits (digit bit 1) and column bits (digit bit 0) of a code, root-most
// digit most significant: the odd and the even bits of the code, each
// compacted to consecutive positions.
__device__ __forceinline__ uint32_t compact_even_bits(uint32_t x) {
  x &= 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0F0F0F0Fu;
  x = (x | (x >> 4)) & 0x00FF00FFu;
  x = (x | (x >> 8)) & 0x0000FFFFu;
  return x;
}

// Letter counts of a base-4 code of `depth` digits (a=0, b=1, c=2, d=3).
__device__ __forceinline__ void letter_counts(uint32_t code, int depth, int n[4]) {
  const uint32_t mask = ((depth >= 16) ? 0xFFFFFFFFu : ((1u << (2 * depth)) - 1u)) & 0x55555555u;
  const uint32_t lo = code & mask, hi = (code >> 1) & mask;
  n[3] = __popc(hi & lo);
  n[2] = __popc(hi & ~lo & mask);
  n[1] = __popc(~hi & lo & mask);
  n[0] = depth - n[1] - n[2] - n[3];
}

__device__ __forceinline__ void split_code(uint32_t code, uint32_t* row, uint32_t* col) {
  *row = compact_even_bits(code >> 1);
  *col = compact_even_bits(code);
}

// Binomial coefficient C(n, r), 0 <= n <= 17, computed directly (used once
// per entry to fill the LDS table of the build kernel).
__device__ __forceinline__ uint32_t binom_direct(int n, int r) {
  if (r < 0 || r > n) return 0;
  uint32_t c = 1;
  for (int i = 1; i <= r; ++i) c = c * static_cast<uint32_t>(n - r + i) / static_cast<uint32_t>(i);
  return c;
}

// expanded nodes whose per-node arrays (17 bytes each) fit the LDS work area
constexpr uint32_t kLdsNodes = 2880;
static_assert(kLdsNodes * 17 <= kMaxClasses * 12, "per-node arrays exceed the LDS work area");
constexpr int kBinomN = 18;  // rows 0..17: enough for C(D + 3, 3) with D <= 14

// Number of distinct paths with the given letter counts (a multinomial
// coefficient), as a product of binomials from the LDS table.
__device__ __forceinline__ uint64_t multinomial(const uint32_t* bt, int na, int nb, int nc, int nd) {
  const int D = na + nb + nc + nd;
  return static_cast<uint64_t>(bt[D * kBinomN + na]) * bt[(D - na) * kBinomN + nb] * bt[(nc + nd) * kBinomN + nc];
}

// Packed class key: counts of a, b, c, d (4 bits each) and depth.
__device__ __forceinline__ uint32_t pack_class(int na, int nb, int nc, int nd) {
  return na | (nb << 4) | (nc << 8) | (nd << 12) | ((na + nb + nc + nd) << 16);
}
__device__ __forceinline__ int class_n(uint32_t key, int x) { return (key >> (4 * x)) & 15; }
__device__ __forceinline__ int class_depth(uint32_t key) { return key >> 16; }
constexpr uint32_t kNoClass = 0xFFFF0000u;  // an unused class slot

// Order of the priority queue: does (p1, D1) come strictly before (p2, D2)?
__device__ __forceinline__ bool class_before(double p1, int d1, double p2, int d2) {
  return p1 > p2 || (p1 == p2 && d1 < d2);
}

struct Boundary {
  double p;
  int depth;
  uint32_t code;
  int all;  // every expandable node is expanded
};

__device__ __forceinline__ bool node_expanded(const Boundary& B, int mode, int cap, int fixed_len, double p,
                                              int depth, uint32_t code) {
  if (depth >= cap) return false;
  if (mode == 0) return depth < fixed_len;
  if (B.all) return true;
  if (p != B.p) return p > B.p;
  if (depth != B.depth) return depth < B.depth;
  return code <= B.code;
}

// The len low bits of v in reverse order (the first letter of a path, its
// most significant bit, goes to bit 0).
__device__ __forceinline__ uint32_t reversed_bits(uint32_t len, uint32_t v) {
  return len == 0 ? 0u : (__brev(v) >> (32u - len));
}

__device__ __forceinline__ uint64_t frac_key(double p, uint64_t* floor_out) {
  double x = __dmul_rn(p, 4294967296.0);
  double fl = floor(x);
  *floor_out = static_cast<uint64_t>(fl);
  return static_cast<uint64_t>(__double_as_longlong(x - fl));
}

// VARIABLE leaves in tree order: level-by-level expansion of the nodes the
// boundary admits, bottom-up leaf counts, top-down leaf placement.  The
// per-node arrays are LDS for trees of up to kLdsNodes expanded nodes and the
// job's global scratch beyond (one body, inlined for either address space).
// Returns false on an internal error (*s_error set).
__device__ __forceinline__ bool variable_leaves(const BuildJob& J, const Boundary& B, const double* prod,
                                                const uint16_t* rows, int cap,
                                                uint32_t n, uint32_t* lvl_code, uint8_t* lvl_mask,
                                                uint32_t* lvl_first, uint32_t* lvl_size, uint32_t* lvl_off,
                                                uint64_t* s_warp, uint32_t* s_lvl_start, int* s_error) {
  const int tid = threadIdx.x;
  // level-by-level expansion
  if (tid == 0) {
    lvl_code[0] = 0;
    s_lvl_start[0] = 0;
    s_lvl_start[1] = 1;
  }
  __syncthreads();
  int D = 0;
  for (; D < cap; ++D) {
    const uint32_t start = s_lvl_start[D], end = s_lvl_start[D + 1];
    if (start == end) break;
    uint32_t next = end;
    for (uint32_t base = start; base < end; base += kBuildThreads) {
      const uint32_t i = base + tid;
      uint32_t mask = 0, code = 0;
      if (i < end) {
        code = lvl_code[i];
        int cnt[4];
        letter_counts(code, D, cnt);
        for (int x = 0; x < 4; ++x) {
          cnt[x]++;
          const double p = prod[class_slot(rows, cnt[0], cnt[1], cnt[2], cnt[3])];
          cnt[x]--;
          if (node_expanded(B, 1, cap, 0, p, D + 1, code * 4 + x)) mask |= 1u << x;
        }
      }
      uint32_t total;
      uint32_t pos = next + block_scan_small<3>(__popc(mask), &total);
      if (i < end) {
        lvl_mask[i] = static_cast<uint8_t>(mask);
        lvl_first[i] = pos;
        for (int x = 0; x < 4; ++x)
          if (mask & (1u << x)) {
            if (pos < J.n_expand) lvl_code[pos] = code * 4 + x;
            else *s_error = kBuildItemCount;
            ++pos;
          }
      }
      next += total;
    }
    if (tid == 0) s_lvl_start[D + 2] = next;
    __syncthreads();
    if (*s_error) return false;
  }
  const int levels = D;  // levels 0..levels-1 are non-empty
  if (tid == 0 && s_lvl_start[levels] != J.n_expand) *s_error = kBuildItemCount;
  __syncthreads();
  if (*s_error) return false;
  // bottom-up leaf counts
  for (int L = levels - 1; L >= 0; --L) {
    for (uint32_t i = s_lvl_start[L] + tid; i < s_lvl_start[L + 1]; i += kBuildThreads) {
      uint32_t mask = lvl_mask[i], f = lvl_first[i], size = 0;
      for (int x = 0; x < 4; ++x) size += (mask & (1u << x)) ? lvl_size[f++] : 1u;
      lvl_size[i] = size;
    }
    __syncthreads();
  }
  if (tid == 0 && lvl_size[0] != n) *s_error = kBuildItemCount;
  __syncthreads();
  if (*s_error) return false;
  // top-down leaf placement
  if (tid == 0) lvl_off[0] = 0;
  __syncthreads();
  for (int L = 0; L < levels; ++L) {
    for (uint32_t i = s_lvl_start[L] + tid; i < s_lvl_start[L + 1]; i += kBuildThreads) {
      uint32_t mask = lvl_mask[i], f = lvl_first[i], cur = lvl_off[i], code = lvl_code[i];
      int cnt[4];
      letter_counts(code, L, cnt);
      for (int x = 0; x < 4; ++x) {
        if (mask & (1u << x)) {
          lvl_off[f] = cur;
          cur += lvl_size[f];
          ++f;
        } else {
          uint32_t cc = code * 4 + x, r, c;
          split_code(cc, &r, &c);
          cnt[x]++;
          J.item_len[cur] = L + 1;
          J.item_row[cur] = r;
          J.item_col[cur] = c;
          J.item_p[cur] = prod[class_slot(rows, cnt[0], cnt[1], cnt[2], cnt[3])];
          cnt[x]--;
          ++cur;
        }
      }
    }
    __syncthreads();
  }
  return true;
}

// Phases 3 to 5, the same for every table: fixed-point weights by largest
// remainders, the alias table in closed form, the hot-path records and the
// statistics.  Returns false on an internal error (*S.error set).
struct BuildShared {
  uint64_t* warp;
  uint32_t* u32;
  uint32_t* hist;
  uint64_t* sel_prefix;
  uint64_t* sel_need;
  unsigned long long* len_mass;
  int* error;
  uint64_t* area;       // LDS free from phase 3 on (or null): the items' keys, then the alias sums
  uint32_t area_words;  // its size in 8-byte words
  uint64_t* vote_rep;    // per wave: a key of the select's current group
  uint32_t* vote_state;  // per wave: none, all equal to it, or mixed
};

__device__ __forceinline__ bool weights_alias_records(const BuildJob& J, uint32_t n, uint32_t nb, uint64_t C,
                                                      const BuildShared& S) {
  const int tid = threadIdx.x;
  // digit values of K x K paths are stored as they are; R-MAT bit strings
  // reversed (the root-most letter in bit 0), for the shift-or append
  const bool reverse = J.kron_K <= 2;
  // ---- 3. weights by largest remainders -------------------------------------
  {
    // the radix passes read every key once per pass: from LDS when the
    // items fit the area, else recomputed from the items
    uint64_t* const keys = n <= S.area_words ? S.area : nullptr;
    uint64_t part = 0;
    for (uint32_t j = tid; j < n; j += kBuildThreads) {
      uint64_t fl;
      const uint64_t key = frac_key(J.item_p[j], &fl);
      if (keys) keys[j] = key;
      part += fl;
    }
    const uint64_t sum = block_sum(part, S.warp);
    const int64_t R = static_cast<int64_t>(1ull << 32) - static_cast<int64_t>(sum);
    if (R < 0 || R > static_cast<int64_t>(n)) {
      if (tid == 0) *S.error = kBuildResidual;
      __syncthreads();
      return false;
    }
    // radix select of the R-th largest fractional part (its bit pattern)
    if (tid == 0) { *S.sel_prefix = 0; *S.sel_need = static_cast<uint64_t>(R); }
    __syncthreads();
    if (R > 0) {
      uint64_t pmask = 0;
      for (int shift = 56; shift >= 0; shift -= 8) {
        for (int i = tid; i < 256; i += kBuildThreads) S.hist[i] = 0;
        __syncthreads();
        const uint64_t prefix = *S.sel_prefix;
        uint64_t rep = 0;
        bool has = false, differ = false;
        for (uint32_t j = tid; j < n; j += kBuildThreads) {
          uint64_t fl;
          const uint64_t key = keys ? keys[j] : frac_key(J.item_p[j], &fl);
          if ((key & pmask) == prefix) {
            atomicAdd(&S.hist[(key >> shift) & 255u], 1u);
            differ = differ || (has && key != rep);
            if (!has) rep = key;
            has = true;
          }
        }
        vote_uniform(rep, has, differ, S.vote_rep, S.vote_state);
        __syncthreads();
        // every key left in the group is the same: it is the threshold, and
        // *S.sel_need the number of its ties that round up
        uint64_t only;
        if (group_uniform(S.vote_rep, S.vote_state, &only)) {
          __syncthreads();
          if (tid == 0) *S.sel_prefix = only;
          __syncthreads();
          break;
        }
        if (tid < 64) {
          uint64_t need = *S.sel_need;
          const uint32_t bin = wave_select_desc(S.hist, &need);
          if (tid == 0) {
            *S.sel_need = need;
            *S.sel_prefix = prefix | (static_cast<uint64_t>(bin) << shift);
          }
        }
        pmask |= 255ull << shift;
        __syncthreads();
      }
    }
    const uint64_t tau = *S.sel_prefix, take_ties = (R > 0) ? *S.sel_need : 0;
    // items above tau round up; ties at tau round up in index order
    uint64_t tie_base = 0;
    for (uint32_t base = 0; base < n; base += kBuildThreads) {
      const uint32_t j = base + tid;
      uint64_t fl = 0, key = 0;
      bool tie = false;
      if (j < n) {
        key = frac_key(J.item_p[j], &fl);
        tie = (R > 0) && key == tau;
      }
      uint32_t total;
      const uint64_t rank = tie_base + block_scan_small<1>(tie ? 1u : 0u, &total);
      if (j < n) {
        bool up = (R > 0) && (key > tau || (tie && rank < take_ties));
        J.item_w[j] = fl + (up ? 1u : 0u);
      }
      tie_base += total;
    }
    for (uint32_t j = n + tid; j < nb; j += kBuildThreads) J.item_w[j] = 0;
    if (tid == 0) J.stats->residual = static_cast<uint64_t>(R);
    __syncthreads();
  }

  // ---- 4. alias table ----------------------------------------------------------
  {
    // the lights' cumulative deficits by light rank and the heavies'
    // cumulative excesses by heavy rank: in LDS when the table fits the area
    // (lights from the bottom, heavies from the top), else in the job's arrays
    uint64_t* const cum = nb <= S.area_words ? S.area : nullptr;
    auto light_cum = [&](uint32_t li) { return cum ? cum[li] : J.light_cum[li]; };
    auto heavy_cum = [&](uint32_t hi) { return cum ? cum[nb - 1 - hi] : J.heavy_cum[hi]; };
    uint64_t nl = 0, dsum = 0, esum = 0;
    for (uint32_t base = 0; base < nb; base += kBuildThreads) {
      const uint32_t j = base + tid;
      uint64_t w = 0;
      bool light = false, valid = j < nb;
      if (valid) { w = J.item_w[j]; light = w < C; }
      uint32_t t_l;
      uint64_t t_d, t_e, dpre, epre;
      const uint64_t lrank = nl + block_scan_small<1>(valid && light ? 1u : 0u, &t_l);
      block_exclusive_scan2(valid && light ? C - w : 0u, valid && !light ? w - C : 0u, &dpre, &epre, &t_d, &t_e);
      dpre += dsum;
      epre += esum;
      if (valid) {
        if (light) {
          J.light_idx[lrank] = j;
          if (cum) cum[lrank] = dpre + (C - w);
          else J.light_cum[lrank] = dpre + (C - w);
        } else {
          uint64_t hrank = j - lrank;
          J.heavy_idx[hrank] = j;
          if (cum) cum[nb - 1 - hrank] = epre + (w - C);
          else J.heavy_cum[hrank] = epre + (w - C);
        }
      }
      nl += t_l; dsum += t_d; esum += t_e;
    }
    __syncthreads();
    const uint32_t n_light = static_cast<uint32_t>(nl), n_heavy = nb - n_light;
    if (dsum != esum || n_heavy == 0) {
      if (tid == 0) *S.error = kBuildAlias;
      __syncthreads();
      return false;
    }
    for (uint32_t li = tid; li < n_light; li += kBuildThreads) {
      const uint32_t j = J.light_idx[li];
      const uint64_t prev = li > 0 ? light_cum(li - 1) : 0;
      // the first heavy whose cumulative excess reaches prev
      uint32_t lo = 0, up = n_heavy;
      while (lo < up) {
        const uint32_t mid = (lo + up) >> 1;
        if (heavy_cum(mid) < prev) lo = mid + 1; else up = mid;
      }
      J.thr[j] = static_cast<uint32_t>(J.item_w[j]);
      J.alias[j] = J.heavy_idx[lo < n_heavy ? lo : n_heavy - 1];
    }
    for (uint32_t hi = tid; hi < n_heavy; hi += kBuildThreads) {
      const uint32_t j = J.heavy_idx[hi];
      const uint64_t E = heavy_cum(hi);
      if (E < dsum && hi + 1 < n_heavy) {
        // the first light whose cumulative deficit exceeds E
        uint32_t lo = 0, up = n_light;
        while (lo < up) {
          const uint32_t mid = (lo + up) >> 1;
          if (light_cum(mid) <= E) lo = mid + 1; else up = mid;
        }
        J.thr[j] = static_cast<uint32_t>(C + E - light_cum(lo < n_light ? lo : n_light - 1));
        J.alias[j] = J.heavy_idx[hi + 1];
      } else {
        J.thr[j] = static_cast<uint32_t>(C);
        J.alias[j] = j;
      }
    }
    __syncthreads();
  }

  // ---- 5. hot-path records and statistics --------------------------------------
  {
    uint64_t wl = 0;
    uint32_t mn = 0xFFFFFFFFu, mx = 0;
    for (uint32_t i = tid; i < nb; i += kBuildThreads) {
      const uint32_t a = J.alias[i];
      const uint32_t ls = J.item_len[i], la = J.item_len[a];
      BucketRecord r;
      // T < C = 2^32 / nb when the alias differs, so (T & ~15) * nb < 2^32
      const uint32_t T = J.thr[i];
      r.thr_abs = a == i ? i << 4 : ((T & ~15u) * nb) | (i << 4) | (T & 15u);
      if (reverse) {
        r.rows = reversed_bits(ls, J.item_row[i]) | (reversed_bits(la, J.item_row[a]) << 16);
        r.cols = reversed_bits(ls, J.item_col[i]) | (reversed_bits(la, J.item_col[a]) << 16);
      } else {
        r.rows = J.item_row[i] | (J.item_row[a] << 16);
        r.cols = J.item_col[i] | (J.item_col[a] << 16);
      }
      r.lens = ls | (la << 16);
      J.records[i] = r;
      if (i < n) {
        wl += J.item_w[i] * ls;
        mn = min(mn, ls);
        mx = max(mx, ls);
        atomicAdd(&S.len_mass[ls & 15u], static_cast<unsigned long long>(J.item_w[i]));
      }
    }
    const uint64_t sum_wl = block_sum(wl, S.warp);
    uint32_t vmax;
    const uint32_t vmin = block_min_max(mn, mx, S.u32, &vmax);
    if (tid == 0) {
      J.stats->sum_wl = sum_wl;
      J.stats->min_len = vmin;
      J.stats->max_len = vmax;
    }
    if (tid < 16) J.stats->len_mass[tid] = S.len_mass[tid];
  }
  return true;
}

// End of a build: on failure every bucket gets a record that still ends each
// edge (see below); then the status and the item count.
__device__ __forceinline__ void finish_build(const BuildJob& J, uint32_t n, uint32_t nb, int error) {
  const int tid = threadIdx.x;
  if (error != 0 && J.records) {
    // A failed build still leaves a table a generation can run on: every
    // bucket holds two empty paths of the longest length, so each sample
    // adds kMaxDepthCap letters and every edge ends within five samples.  A
    // batch or a served round that launches generation right after the
    // build (before the host sees the status) therefore terminates; its
    // output is meaningless and the status reports the failure.
    const uint32_t len2 = static_cast<uint32_t>(kMaxDepthCap) * 0x10001u;
    for (uint32_t i = tid; i < nb; i += kBuildThreads) J.records[i] = BucketRecord{0xFFFFFFFFu, 0u, 0u, len2};
  }
  if (tid == 0) {
    J.stats->error = error;
    J.stats->n_items = n;
  }
}


// ------------------------------------------------------ K x K initiators --
// The table of a K x K initiator is the R-MAT table over K^2 letters (letter
// K i + j is cell (i, j)): the same queue order and canonical products, with
// paths capped at the largest L with K^L <= 2^15, so that each path's row
// and column digits fit 15 bits as base-K values.  Phases 3 to 5 are shared
// with R-MAT tables; phases 1 and 2 work on packed codes (digit_bits bits
// per letter, the root-most letter most significant).  Letter-count classes
// do not scale to K^2 letters (C(D + K^2 - 1, D) of them), so the boundary
// node is found by bisection over its probability instead: the expandable
// nodes of probability >= tau form a subtree (a child is never more
// probable than its parent), counted level by level up to t; the largest
// tau with at least t of them is the boundary's probability, and the
// boundary is the r-th node of that probability in (depth, code) order,
// which a level-order walk meets in exactly that order.

constexpr int kKronMaxDigits = 9;  // K >= 3: K^L <= 2^15 gives L <= 9

struct KronCtx {
  const double* q;  // the K^2 letter probabilities (LDS)
  uint32_t L;       // letters
  uint32_t dbits;   // bits per letter in a packed code
  uint32_t K;
  int cap;
};

struct KronBoundary {
  double p;
  int depth;
  int all;  // every expandable node is expanded
  uint64_t code;
};

// Canonical probability of a path: its letters sorted ascending, multiplied
// into 1.0 one at a time with rounding after each product (the same as
// multiplying P_x n_x times for x = 0, 1, ...).
__device__ __forceinline__ double kron_prob(const KronCtx& X, uint64_t code, int depth) {
  const uint32_t mask = (1u << X.dbits) - 1u;
  uint32_t d[kKronMaxDigits];
#pragma unroll
  for (int i = 0; i < kKronMaxDigits; ++i)
    d[i] = i < depth ? static_cast<uint32_t>(code >> (X.dbits * i)) & mask : 0xFFFFFFFFu;
  // odd-even transposition sort: n rounds sort n values
#pragma unroll
  for (int r = 0; r < kKronMaxDigits; ++r)
#pragma unroll
    for (int i = r & 1; i + 1 < kKronMaxDigits; i += 2) {
      const uint32_t lo = min(d[i], d[i + 1]), hi = max(d[i], d[i + 1]);
      d[i] = lo;
      d[i + 1] = hi;
    }
  double p = 1.0;
#pragma unroll
  for (int i = 0; i < kKronMaxDigits; ++i)
    if (i < depth) p = __dmul_rn(p, X.q[d[i]]);
  return p;
}

__device__ __forceinline__ uint64_t prob_bits(double p) { return static_cast<uint64_t>(__double_as_longlong(p)); }

// Row and column digit values of a path (root-most digit most significant).
__device__ __forceinline__ void kron_rowcol(const KronCtx& X, uint64_t code, int depth, uint32_t* row, uint32_t* col) {
  const uint32_t mask = (1u << X.dbits) - 1u;
  uint32_t r = 0, c = 0;
  for (int pos = depth - 1; pos >= 0; --pos) {
    const uint32_t x = static_cast<uint32_t>(code >> (X.dbits * pos)) & mask;
    r = r * X.K + x / X.K;
    c = c * X.K + x % X.K;
  }
  *row = r;
  *col = c;
}

__device__ __forceinline__ bool kron_expanded(const KronBoundary& B, int cap, double p, int depth, uint64_t code) {
  if (depth >= cap) return false;
  if (B.all) return true;
  if (p != B.p) return p > B.p;
  if (depth != B.depth) return depth < B.depth;
  return code <= B.code;
}

// Number of expandable nodes (depth < cap) of probability >= tau (bit
// pattern), counted level by level and stopped once it reaches `limit`:
// returns min(count, limit).  Each level's nodes are kept (in code order) in
// one of two buffers of cap_buf codes.
__device__ uint64_t kron_count_ge(const KronCtx& X, uint64_t tau, uint64_t limit, uint64_t* buf0, uint64_t* buf1,
                                  uint64_t cap_buf, uint64_t* s_warp) {
  const int tid = threadIdx.x;
  uint64_t count = 1;  // the root, probability 1 >= tau
  if (count >= limit) return limit;
  uint64_t* cur = buf0;
  uint64_t* nxt = buf1;
  __syncthreads();  // a previous walk's last stores into the buffers are done
  if (tid == 0) cur[0] = 0;
  __syncthreads();
  uint32_t len = 1;
  for (int D = 0; D + 1 < X.cap && len > 0; ++D) {
    const uint32_t pairs = len * X.L;
    uint64_t next = 0;
    for (uint32_t base = 0; base < pairs; base += kBuildThreads) {
      const uint32_t pr = base + tid;
      bool pass = false;
      uint64_t child = 0;
      if (pr < pairs) {
        const uint32_t i = pr / X.L, x = pr - i * X.L;
        child = (cur[i] << X.dbits) | x;
        pass = prob_bits(kron_prob(X, child, D + 1)) >= tau;
      }
      uint64_t total;
      const uint64_t pos = next + block_exclusive_scan(pass ? 1u : 0u, s_warp, &total);
      if (pass && pos < cap_buf) nxt[pos] = child;
      next += total;
      if (count + next >= limit) return limit;  // uniform
    }
    __syncthreads();
    count += next;
    uint64_t* t = cur;
    cur = nxt;
    nxt = t;
    len = static_cast<uint32_t>(next);
  }
  return count;
}

// Boundary of a VARIABLE table: the n_expand-th expandable node in the queue
// order (probability descending, depth ascending, code ascending).  Written
// to *s_bnd by the thread that meets it; error kBuildItemCount if the walk
// ends without it.
__device__ void kron_boundary(const BuildJob& J, const KronCtx& X, KronBoundary* s_bnd, uint64_t* s_warp,
                              int* s_error) {
  const int tid = threadIdx.x;
  const uint64_t t = J.n_expand;
  uint64_t all_nodes = 0, lp = 1;
  for (int D = 0; D < X.cap; ++D, lp *= X.L) all_nodes += lp;
  if (tid == 0) {
    s_bnd->p = 0.0;
    s_bnd->depth = 0;
    s_bnd->code = 0;
    s_bnd->all = t >= all_nodes ? 1 : 0;
  }
  __syncthreads();
  if (t >= all_nodes) return;
  uint64_t* buf0 = J.bfs[0];
  uint64_t* buf1 = J.bfs[1];
  const uint64_t one = prob_bits(1.0);
  // the largest tau with at least t nodes of probability >= tau: such a
  // node exists (the count drops past it), and it is the t-th node's
  uint64_t lo = 0, hi = one + 1, c_hi = 0;
  while (hi - lo > 1) {
    const uint64_t mid = lo + (hi - lo) / 2;
    const uint64_t c = kron_count_ge(X, mid, t, buf0, buf1, J.bfs_cap, s_warp);
    if (c >= t) {
      lo = mid;
    } else {
      hi = mid;
      c_hi = c;  // exact: below the limit
    }
  }
  const uint64_t tau = lo;
  const uint64_t r = t - c_hi;  // rank of the boundary among the nodes of probability tau
  // level-order walk over the nodes of probability >= tau, counting those of
  // probability exactly tau; children are generated in code order
  uint64_t ties = (one == tau) ? 1 : 0;
  if (ties >= r) {
    if (tid == 0) {
      s_bnd->p = 1.0;
      s_bnd->depth = 0;
      s_bnd->code = 0;
    }
    __syncthreads();
    return;
  }
  uint64_t* cur = buf0;
  uint64_t* nxt = buf1;
  __syncthreads();
  if (tid == 0) cur[0] = 0;
  __syncthreads();
  uint32_t len = 1;
  for (int D = 0; D + 1 < X.cap && len > 0; ++D) {
    const uint32_t pairs = len * X.L;
    uint64_t next = 0;
    for (uint32_t base = 0; base < pairs; base += kBuildThreads) {
      const uint32_t pr = base + tid;
      bool pass = false, tie = false;
      uint64_t child = 0;
      double p = 0.0;
      if (pr < pairs) {
        const uint32_t i = pr / X.L, x = pr - i * X.L;
        child = (cur[i] << X.dbits) | x;
        p = kron_prob(X, child, D + 1);
        pass = prob_bits(p) >= tau;
        tie = prob_bits(p) == tau;
      }
      // one scan for both counts: passes in the low word, ties in the high
      uint64_t total;
      const uint64_t both = block_exclusive_scan((pass ? 1ull : 0ull) | (tie ? 1ull << 32 : 0ull), s_warp, &total);
      const uint64_t pos = next + (both & 0xFFFFFFFFull);
      if (pass && pos < J.bfs_cap) nxt[pos] = child;
      next += total & 0xFFFFFFFFull;
      const uint64_t tie_total = total >> 32;
      if (ties + tie_total >= r) {
        if (tie && ties + (both >> 32) + 1 == r) {
          s_bnd->p = p;
          s_bnd->depth = D + 1;
          s_bnd->code = child;
        }
        __syncthreads();
        return;
      }
      ties += tie_total;
    }
    __syncthreads();
    uint64_t* tmp = cur;
    cur = nxt;
    nxt = tmp;
    len = static_cast<uint32_t>(next);
  }
  if (tid == 0) *s_error = kBuildItemCount;
  __syncthreads();
}

// VARIABLE leaves of a K x K table in tree order: the nodes the boundary
// admits, level by level (one thread per (node, letter) pair), subtree leaf
// counts bottom-up, leaf placement top-down.  A node's expanded children are
// stored from lvl_first[node] in letter order, so the number of them is the
// distance to the next node's first child.  Returns false on an internal
// error (*s_error set).
__device__ bool kron_variable_leaves(const BuildJob& J, const KronCtx& X, const KronBoundary& B, uint32_t n,
                                     uint64_t* s_warp, uint32_t* s_lvl_start, int* s_error) {
  const int tid = threadIdx.x;
  uint64_t* code = J.kcode;
  uint32_t* first = J.lvl_first;
  uint32_t* size = J.lvl_size;
  uint32_t* off = J.lvl_off;
  if (tid == 0) {
    code[0] = 0;
    s_lvl_start[0] = 0;
    s_lvl_start[1] = 1;
  }
  __syncthreads();
  int D = 0;
  for (; D < X.cap; ++D) {
    const uint32_t start = s_lvl_start[D], end = s_lvl_start[D + 1];
    if (start == end) break;
    const uint32_t pairs = (end - start) * X.L;
    uint32_t next = end;
    for (uint32_t base = 0; base < pairs; base += kBuildThreads) {
      const uint32_t pr = base + tid;
      bool pass = false;
      uint64_t child = 0;
      uint32_t i = 0, x = 0;
      if (pr < pairs) {
        i = start + pr / X.L;
        x = pr % X.L;
        child = (code[i] << X.dbits) | x;
        if (D + 1 < X.cap) pass = kron_expanded(B, X.cap, kron_prob(X, child, D + 1), D + 1, child);
      }
      uint32_t total;
      const uint32_t pos = next + block_scan_small<1>(pass ? 1u : 0u, &total);
      if (pr < pairs && x == 0) first[i] = pos;
      if (pass) {
        if (pos < J.n_expand) code[pos] = child;
        else *s_error = kBuildItemCount;
      }
      next += total;
    }
    if (tid == 0) s_lvl_start[D + 2] = next;
    __syncthreads();
    if (*s_error) return false;
  }
  const int levels = D;
  if (tid == 0 && s_lvl_start[levels] != J.n_expand) *s_error = kBuildItemCount;
  __syncthreads();
  if (*s_error) return false;
  // bottom-up leaf counts
  for (int Lv = levels - 1; Lv >= 0; --Lv) {
    const uint32_t end = s_lvl_start[Lv + 1];
    for (uint32_t i = s_lvl_start[Lv] + tid; i < end; i += kBuildThreads) {
      const uint32_t f = first[i], e = i + 1 < end ? first[i + 1] : s_lvl_start[Lv + 2];
      uint32_t sz = X.L - (e - f);
      for (uint32_t j = f; j < e; ++j) sz += size[j];
      size[i] = sz;
    }
    __syncthreads();
  }
  if (tid == 0 && size[0] != n) *s_error = kBuildItemCount;
  __syncthreads();
  if (*s_error) return false;
  // top-down placement
  if (tid == 0) off[0] = 0;
  __syncthreads();
  for (int Lv = 0; Lv < levels; ++Lv) {
    for (uint32_t i = s_lvl_start[Lv] + tid; i < s_lvl_start[Lv + 1]; i += kBuildThreads) {
      const uint64_t c0 = code[i];
      uint32_t f = first[i], cur = off[i];
      for (uint32_t x = 0; x < X.L; ++x) {
        const uint64_t child = (c0 << X.dbits) | x;
        const double p = kron_prob(X, child, Lv + 1);
        if (kron_expanded(B, X.cap, p, Lv + 1, child)) {
          off[f] = cur;
          cur += size[f];
          ++f;
        } else {
          uint32_t r, c;
          kron_rowcol(X, child, Lv + 1, &r, &c);
          J.item_len[cur] = Lv + 1;
          J.item_row[cur] = r;
          J.item_col[cur] = c;
          J.item_p[cur] = p;
          ++cur;
        }
      }
    }
    __syncthreads();
  }
  return true;
}

__global__ __launch_bounds__(kBuildThreads) void kron_table_build_kernel(BuildJob J) {
  const int tid = threadIdx.x;
  __shared__ double s_q[256];
  __shared__ uint64_t s_warp[kWaves];
  __shared__ uint32_t s_u32[2 * kWaves];
  __shared__ uint32_t s_hist[256];
  __shared__ int s_error;
  __shared__ uint64_t s_sel_prefix, s_sel_need;
  __shared__ unsigned long long s_len_mass[16];
  __shared__ uint32_t s_lvl_start[kKronMaxDigits + 2];
  __shared__ KronBoundary s_kb;
  __shared__ uint64_t s_vote_rep[kWaves];
  __shared__ uint32_t s_vote_state[kWaves];

  const uint32_t n = J.n_items;
  const uint32_t nb = static_cast<uint32_t>(J.n_buckets);
  const uint64_t C = J.capacity;
  if (tid == 0) s_error = 0;
  if (tid < 16) s_len_mass[tid] = 0ull;
  for (int x = tid; x < J.letters; x += kBuildThreads) s_q[x] = J.qk[x];
  __syncthreads();
  const KronCtx X{s_q, static_cast<uint32_t>(J.letters), static_cast<uint32_t>(J.digit_bits),
                  static_cast<uint32_t>(J.kron_K), J.cap};

  if (J.mode == 0) {  // FIXED: all paths of length l, in code order
    const int ell = J.fixed_len;
    for (uint32_t j = tid; j < n; j += kBuildThreads) {
      uint64_t code = 0;
      uint32_t v = j;
      for (int pos = 0; pos < ell; ++pos) {
        code |= static_cast<uint64_t>(v % X.L) << (X.dbits * pos);
        v /= X.L;
      }
      uint32_t r, c;
      kron_rowcol(X, code, ell, &r, &c);
      J.item_len[j] = ell;
      J.item_row[j] = r;
      J.item_col[j] = c;
      J.item_p[j] = kron_prob(X, code, ell);
    }
  } else {
    kron_boundary(J, X, &s_kb, s_warp, &s_error);
    __syncthreads();
    if (s_error) goto finish;
    {
      const KronBoundary B = s_kb;
      if (!kron_variable_leaves(J, X, B, n, s_warp, s_lvl_start, &s_error)) goto finish;
    }
  }
  for (uint32_t j = n + tid; j < nb; j += kBuildThreads) {
    J.item_len[j] = 0; J.item_row[j] = 0; J.item_col[j] = 0; J.item_p[j] = 0.0;
  }
  __syncthreads();
  {
    const BuildShared S{s_warp,    s_u32,      s_hist,  &s_sel_prefix, &s_sel_need, s_len_mass,
                        &s_error,  nullptr,    0u,      s_vote_rep,    s_vote_state};
    weights_alias_records(J, n, nb, C, S);
  }

finish:
  __syncthreads();
  finish_build(J, n, nb, s_error);
}

// ------------------------------------------------------------------ kernel --
__device__ __forceinline__ void build_table(const BuildJob& J) {
  const int tid = threadIdx.x;

  // one area: phase 1's class keys, then phase 2's per-node arrays (small
  // trees) in its first part, the class probabilities by slot behind them;
  // from phase 3 on the whole area holds the items' keys, then alias sums
  constexpr size_t kWorkBytes = kMaxClasses * (sizeof(double) + sizeof(uint32_t));
  constexpr size_t kAreaBytes = kWorkBytes + kMaxClasses * sizeof(double);
  __shared__ __align__(16) unsigned char s_area[kAreaBytes];
  unsigned char* const s_work = s_area;
  uint32_t* const s_cls_key = reinterpret_cast<uint32_t*>(s_work);
  double* const s_cls_p = reinterpret_cast<double*>(s_area + kWorkBytes);
  // the class slots' rows (phases 1 and 2)
  __shared__ uint16_t s_rows[16 * 16 * 16];
  __shared__ uint64_t s_warp[kWaves];
  __shared__ uint32_t s_u32[2 * kWaves];
  __shared__ uint32_t s_hist[256];
  __shared__ unsigned long long s_hist64[256];
  __shared__ uint16_t s_group[kMaxClasses];
  __shared__ uint32_t s_lvl_start[kMaxDepthCap + 2];
  __shared__ Boundary s_bnd;
  __shared__ int s_error;
  __shared__ uint64_t s_sel_prefix, s_sel_need;
  __shared__ uint32_t s_binom[kBinomN * kBinomN];
  __shared__ unsigned long long s_len_mass[16];
  __shared__ uint64_t s_vote_rep[kWaves];
  __shared__ uint32_t s_vote_state[kWaves];

  const double q[4] = {J.q[0], J.q[1], J.q[2], J.q[3]};
  const int cap = J.cap;
  const uint32_t n = J.n_items;
  const uint32_t nb = static_cast<uint32_t>(J.n_buckets);
  const uint64_t C = J.capacity;

  if (tid == 0) {
    s_error = 0;
    s_bnd.p = 0.0; s_bnd.depth = 0; s_bnd.code = 0; s_bnd.all = 0;
    if (J.reset_counter) *J.reset_counter = 0u;
  }
  if (tid < 16) s_len_mass[tid] = 0ull;
  for (int i = tid; i < kBinomN * kBinomN; i += kBuildThreads) s_binom[i] = binom_direct(i / kBinomN, i % kBinomN);
  __syncthreads();
  const uint32_t* bt = s_binom;

  // ---- class probabilities ----------------------------------------------------
  {
    // thread t < kClassRows owns row t: (na, nb, nc) from t, the row's first
    // slot from a scan of the row lengths
    int na = 0, nb_ = 0, nc = 0, len = 0;
    if (tid < kClassRows) {
      int r = tid;
      while (r >= (16 - na) * (17 - na) / 2) { r -= (16 - na) * (17 - na) / 2; ++na; }
      while (r >= 16 - na - nb_) { r -= 16 - na - nb_; ++nb_; }
      nc = r;
      len = 16 - na - nb_ - nc;
    }
    uint64_t total;
    const uint32_t first = static_cast<uint32_t>(block_exclusive_scan(static_cast<uint64_t>(len), s_warp, &total));
    if (tid < kClassRows) {
      s_rows[(na * 16 + nb_) * 16 + nc] = static_cast<uint16_t>(first);
      double p = 1.0;
      for (int i = 0; i < na; ++i) p = __dmul_rn(p, q[0]);
      for (int i = 0; i < nb_; ++i) p = __dmul_rn(p, q[1]);
      for (int i = 0; i < nc; ++i) p = __dmul_rn(p, q[2]);
      for (int nd = 0; nd < len; ++nd) {
        if (nd > 0) p = __dmul_rn(p, q[3]);
        s_cls_p[first + nd] = p;
        // phase 1 takes the classes of depth < cap
        s_cls_key[first + nd] = na + nb_ + nc + nd < cap ? pack_class(na, nb_, nc, nd) : kNoClass;
      }
    }
    for (int i = kClassSlots + tid; i < kMaxClasses; i += kBuildThreads) {
      s_cls_p[i] = -1.0;
      s_cls_key[i] = kNoClass;
    }
    __syncthreads();
  }

  // ---- 1. boundary node (VARIABLE) ------------------------------------------
  if (J.mode == 1) {
    // The boundary is node n_expand of the order (p descending, depth
    // ascending, code ascending).  Classes hold whole (p, depth) runs, so a
    // radix select over the bits of p (descending; a non-negative double's
    // bit pattern orders like its value), weighted by the classes' node
    // counts, then over depth, finds the run holding it and its rank there.
    constexpr int kPer = kMaxClasses / kBuildThreads;
    uint64_t cnt_local[kPer], pb_local[kPer], sum_local = 0;
    for (int u = 0; u < kPer; ++u) {
      const int i = tid * kPer + u;
      const uint32_t key = s_cls_key[i];
      cnt_local[u] = key != kNoClass ? multinomial(bt, class_n(key, 0), class_n(key, 1), class_n(key, 2), class_n(key, 3)) : 0;
      pb_local[u] = static_cast<uint64_t>(__double_as_longlong(s_cls_p[i]));
      sum_local += cnt_local[u];
    }
    const uint64_t total_nodes = block_sum(sum_local, s_warp);
    const bool all = J.n_expand == 0 || J.n_expand > total_nodes;
    if (tid == 0) { s_sel_prefix = 0; s_sel_need = J.n_expand; s_u32[0] = 0; }
    uint64_t prefix = 0, pmask = 0;
    if (!all) {
      for (int shift = 56; shift >= 0; shift -= 8) {
        for (int i = tid; i < 256; i += kBuildThreads) s_hist64[i] = 0;
        __syncthreads();
        uint64_t rep = 0;
        bool has = false, differ = false;
        for (int u = 0; u < kPer; ++u)
          if (cnt_local[u] != 0 && (pb_local[u] & pmask) == prefix) {
            atomicAdd(&s_hist64[(pb_local[u] >> shift) & 255u], static_cast<unsigned long long>(cnt_local[u]));
            differ = differ || (has && pb_local[u] != rep);
            if (!has) rep = pb_local[u];
            has = true;
          }
        vote_uniform(rep, has, differ, s_vote_rep, s_vote_state);
        __syncthreads();
        // every class left in the group has the same probability: that is
        // the boundary's, and s_sel_need its rank among the group's nodes
        uint64_t only;
        if (group_uniform(s_vote_rep, s_vote_state, &only)) {
          prefix = only;
          break;
        }
        if (tid < 64) {
          uint64_t need = s_sel_need;
          const uint32_t bin = wave_select_desc(s_hist64, &need);
          if (tid == 0) {
            s_sel_need = need;
            s_sel_prefix = prefix | (static_cast<uint64_t>(bin) << shift);
          }
        }
        __syncthreads();
        prefix = s_sel_prefix;
        pmask |= 255ull << shift;
      }
      // depth, ascending, among the classes of probability bits `prefix`
      if (tid < 16) s_hist64[tid] = 0;
      __syncthreads();
      for (int u = 0; u < kPer; ++u)
        if (cnt_local[u] != 0 && pb_local[u] == prefix)
          atomicAdd(&s_hist64[class_depth(s_cls_key[tid * kPer + u])], static_cast<unsigned long long>(cnt_local[u]));
      __syncthreads();
      if (tid == 0) {
        uint64_t need = s_sel_need;
        int d = 0;
        for (; d < 15; ++d) {
          if (need <= s_hist64[d]) break;
          need -= s_hist64[d];
        }
        s_sel_need = need;
        s_u32[1] = static_cast<uint32_t>(d);
      }
      __syncthreads();
      // the run's classes, in any order (the rank below only sums over them)
      const int run_depth = static_cast<int>(s_u32[1]);
      for (int u = 0; u < kPer; ++u) {
        const int i = tid * kPer + u;
        if (cnt_local[u] != 0 && pb_local[u] == prefix && class_depth(s_cls_key[i]) == run_depth)
          s_group[atomicAdd(&s_u32[0], 1u)] = static_cast<uint16_t>(i);
      }
      __syncthreads();
    }
    if (tid < 64 && s_error == 0) {
      if (all) {
        if (tid == 0) s_bnd.all = 1;
      } else {
        // digit by digit, the letter whose completions (summed over the
        // run's classes) hold the rank: lane L counts letter L & 3 over the
        // classes g = L >> 2, L >> 2 + 16, ...
        uint64_t r = s_sel_need - 1;  // rank of the last expanded node in its run
        const int n_group = static_cast<int>(s_u32[0]);
        const int D = static_cast<int>(s_u32[1]);
        const int x = tid & 3;
        int used[4] = {0, 0, 0, 0};
        uint32_t code = 0;
        for (int pos = 0; pos < D; ++pos) {
          uint64_t cnt = 0;
          for (int g = tid >> 2; g < n_group; g += 16) {
            const uint32_t key = s_cls_key[s_group[g]];
            int rem[4];
            bool ok = true;
            for (int y = 0; y < 4; ++y) {
              rem[y] = class_n(key, y) - used[y] - (y == x ? 1 : 0);
              ok = ok && rem[y] >= 0;
            }
            if (ok) cnt += multinomial(bt, rem[0], rem[1], rem[2], rem[3]);
          }
          for (int d = 4; d < 64; d <<= 1) cnt += shfl_xor_u64(cnt, d);  // lanes of one letter
          int chosen = 3;
          for (int y = 0; y < 4; ++y) {
            const uint64_t c = static_cast<uint64_t>(static_cast<uint32_t>(__shfl(static_cast<uint32_t>(cnt), y, 64))) |
                               (static_cast<uint64_t>(static_cast<uint32_t>(__shfl(static_cast<uint32_t>(cnt >> 32), y, 64)))
                                << 32);
            if (r < c) {
              chosen = y;
              break;
            }
            r -= c;
          }
          used[chosen]++;
          code = code * 4 + chosen;
        }
        if (tid == 0) {
          s_bnd.p = __longlong_as_double(static_cast<long long>(prefix));
          s_bnd.depth = D;
          s_bnd.code = code;
        }
      }
    }
    __syncthreads();
  }
  const Boundary B = s_bnd;
  if (s_error) goto finish;

  // ---- 2. leaves in tree order ----------------------------------------------
  if (J.mode == 0) {
    const int ell = J.fixed_len;
    for (uint32_t j = tid; j < n; j += kBuildThreads) {
      int cnt[4];
      letter_counts(j, ell, cnt);
      uint32_t r, c;
      split_code(j, &r, &c);
      J.item_len[j] = ell;
      J.item_row[j] = r;
      J.item_col[j] = c;
      J.item_p[j] = s_cls_p[class_slot(s_rows, cnt[0], cnt[1], cnt[2], cnt[3])];
    }
  } else {
    bool ok;
    if (J.n_expand <= kLdsNodes) {
      uint32_t* code = reinterpret_cast<uint32_t*>(s_work);
      uint32_t* first = code + kLdsNodes;
      uint32_t* size = first + kLdsNodes;
      uint32_t* off = size + kLdsNodes;
      uint8_t* mask = reinterpret_cast<uint8_t*>(off + kLdsNodes);
      ok = variable_leaves(J, B, s_cls_p, s_rows, cap, n, code, mask, first, size, off, s_warp, s_lvl_start, &s_error);
    } else {
      ok = variable_leaves(J, B, s_cls_p, s_rows, cap, n, J.lvl_code, J.lvl_mask, J.lvl_first, J.lvl_size, J.lvl_off, s_warp,
                           s_lvl_start, &s_error);
    }
    if (!ok) goto finish;
  }
  for (uint32_t j = n + tid; j < nb; j += kBuildThreads) {
    J.item_len[j] = 0; J.item_row[j] = 0; J.item_col[j] = 0; J.item_p[j] = 0.0;
  }
  __syncthreads();

  {
    const BuildShared S{s_warp,  s_u32,       s_hist,   &s_sel_prefix,
                        &s_sel_need, s_len_mass, &s_error, reinterpret_cast<uint64_t*>(s_area),
                        static_cast<uint32_t>(kAreaBytes / sizeof(uint64_t)), s_vote_rep, s_vote_state};
    weights_alias_records(J, n, nb, C, S);
  }

finish:
  __syncthreads();
  finish_build(J, n, nb, s_error);
}

// One workgroup per job, jobs in device memory (batches, table sets).
__global__ __launch_bounds__(kBuildThreads) void table_build_kernel(const BuildJob* __restrict__ jobs) {
  const BuildJob J = jobs[blockIdx.x];
  build_table(J);
}

// A single job passed by value (no upload before the launch).
__global__ __launch_bounds__(kBuildThreads) void table_build_one_kernel(BuildJob J) { build_table(J); }

}  // namespace

hipError_t launch_table_build(const BuildJob* d_jobs, int n_jobs, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(table_build_kernel, dim3(n_jobs), dim3(kBuildThreads), 0, s, d_jobs);
  return hipGetLastError();
}

hipError_t launch_kron_table_build(const BuildJob& job, hipStream_t s) {
  hipLaunchKernelGGL(kron_table_build_kernel, dim3(1), dim3(kBuildThreads), 0, s, job);
  return hipGetLastError();
}

hipError_t launch_table_build_one(const BuildJob& job, hipStream_t s) {
  hipLaunchKernelGGL(table_build_one_kernel, dim3(1), dim3(kBuildThreads), 0, s, job);
  return hipGetLastError();
}

}  // namespace rmat
