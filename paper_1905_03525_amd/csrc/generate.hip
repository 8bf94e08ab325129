// generate.hip -- the hot path: per-edge Philox draws, alias lookups in an
// LDS-resident (or L2-resident) bucket table, and bit concatenation (Sec. 2,
// the sampling loop), plus the variants that reduce edges on the device
// instead of storing them (a source-prefix histogram with a checksum, or an
// out-degree counter per node), the persistent kernel of batches, partitioned
// tiles and served requests, and the base-K accumulators of K x K initiators.
//
// Work split.  The absolute edge index space is cut into 64-edge blocks
// aligned to multiples of 64, so the high counter word e >> 32 is uniform
// across a wave and every store instruction covers 64 consecutive slots.  A
// wave takes its blocks in tiles of 8 (wave, wave + W, wave + 2W, ... for W
// waves in the grid).  Every edge of a tile draws its first Philox block (4
// samples; two blocks when the table's edges mostly need more); an edge
// with k letters is stored at once from registers, 64 consecutive ids per
// store, and the others (11% at k = 26 with the 4093-path table) join a
// small per-wave LDS queue, which continues them 64 at a time with counter
// blocks 1, 2, ... as soon as it holds a full wave's worth, so a further
// Philox block is only paid for edges that need it.  The queue's 128
// entries leave the LDS to the table: two 12-wave workgroups share a CU
// where one 64 KiB table copy each fits.  The kernel is bound by
// instruction issue under the chip's power limit, so a full tile of whole
// blocks -- all but a few tiles at the ends of a range -- takes an unrolled,
// software-pipelined copy with no per-block lane masks or loop control,
// whose ids go out through one buffer descriptor per output array.
#include <mutex>
#include <type_traits>
#include <vector>

#include "rmat_internal.h"

namespace rmat {
namespace {

constexpr int kGenThreads = 1024;  // the largest workgroup: 16 waves share one LDS copy of the table
constexpr int kWaves = kGenThreads / 64;
constexpr uint32_t kMaxTile = 8;
// Every path of a built table has at least one letter and ids have at most
// 64, so an edge uses at most 64 samples: 16 Philox blocks.  The
// continuation loop stops there whatever the table holds.
constexpr uint32_t kMaxBlocksPerEdge = 16;
constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products (one v_mad_u64_u32 each) and three-input XORs (v_bitop3_b32,
// truth table 0x96), the key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox10(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3, uint32_t k0,
                                         uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = static_cast<uint64_t>(x0) * kPhiloxM0;
    const uint64_t p1 = static_cast<uint64_t>(x2) * kPhiloxM1;
    const uint32_t y0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p1 >> 32), x1, k0, 0x96);
    const uint32_t y2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p0 >> 32), x3, k1, 0x96);
    x0 = y0;
    x1 = static_cast<uint32_t>(p1);
    x2 = y2;
    x3 = static_cast<uint32_t>(p0);
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
}

// The first counter block of an edge, (e_lo, e_hi, 0, ctr3) with e_hi and
// ctr3 the same across the wave: rounds 1 and 2 are specialised (a zero word's product is
// zero; what depends only on e_hi and the key stays on the scalar unit); the
// output equals philox10 on that counter.
__device__ __forceinline__ void philox10_first(uint32_t e_lo, uint32_t e_hi, uint32_t ctr3, uint32_t k0, uint32_t k1,
                                               uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3) {
  const uint64_t p0 = static_cast<uint64_t>(e_lo) * kPhiloxM0;
  const uint32_t a0 = e_hi ^ k0;  // hi(0 * M1) ^ e_hi ^ k0
  const uint32_t a2 = static_cast<uint32_t>(p0 >> 32) ^ (ctr3 ^ k1);
  const uint32_t a3 = static_cast<uint32_t>(p0);  // and a1 = lo(0 * M1) = 0
  k0 += kPhiloxW0;
  k1 += kPhiloxW1;
  const uint64_t q0 = static_cast<uint64_t>(a0) * kPhiloxM0;
  const uint64_t q1 = static_cast<uint64_t>(a2) * kPhiloxM1;
  const uint32_t b0 = static_cast<uint32_t>(q1 >> 32) ^ k0;  // ^ a1 = 0
  const uint32_t b1 = static_cast<uint32_t>(q1);
  const uint32_t b2 = (static_cast<uint32_t>(q0 >> 32) ^ k1) ^ a3;
  const uint32_t b3 = static_cast<uint32_t>(q0);  // uniform
  k0 += kPhiloxW0;
  k1 += kPhiloxW1;
  const uint64_t r0 = static_cast<uint64_t>(b0) * kPhiloxM0;
  const uint64_t r1 = static_cast<uint64_t>(b2) * kPhiloxM1;
  x0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(r1 >> 32), b1, k0, 0x96);
  x1 = static_cast<uint32_t>(r1);
  x2 = static_cast<uint32_t>(r0 >> 32) ^ (b3 ^ k1);
  x3 = static_cast<uint32_t>(r0);
  k0 += kPhiloxW0;
  k1 += kPhiloxW1;
#pragma unroll
  for (int r = 3; r < 10; ++r) {
    const uint64_t m0 = static_cast<uint64_t>(x0) * kPhiloxM0;
    const uint64_t m1 = static_cast<uint64_t>(x2) * kPhiloxM1;
    const uint32_t y0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(m1 >> 32), x1, k0, 0x96);
    const uint32_t y2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(m0 >> 32), x3, k1, 0x96);
    x0 = y0;
    x1 = static_cast<uint32_t>(m1);
    x2 = y2;
    x3 = static_cast<uint32_t>(m0);
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
}

// (x * m + a) mod 2^64 with 32-bit x, m: one v_mad_u64_u32, which runs at
// the full vector rate on gfx950 where v_mul_lo_u32 does not.
__device__ __forceinline__ uint64_t mad_u64_u32(uint32_t x, uint32_t m, uint64_t a) {
  uint64_t r, carry;
  __asm__("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "=s"(carry) : "v"(x), "v"(m), "v"(a));
  return r;
}

// Powers of a K x K initiator's K for the base-K accumulators: pow[i] = K^i
// (i <= 15) and magic[i] = floor(2^32 / K^i) + 1, with which the high word of
// x * magic[i] is floor(x / K^i) for every x < 2^16 when 2 <= K^i <= 2^16
// (the error x * (magic[i] - 2^32 / K^i) / 2^32 < 2^-16 <= 1 / K^i cannot
// carry the quotient past the next integer).  rcp[i] is the double one unit
// in the last place above the rounded 1 / K^i, so 1 / K^i <= rcp[i] <=
// (1 / K^i)(1 + 2^-51).
struct KronPow {
  uint64_t pow[16];
  uint32_t magic[16];
  double rcp[16];
};

// Row/column accumulators, filled from bit 0 up: a path of L letters,
// stored bit-reversed, is shifted to the current fill level and OR-ed in
// (one v_lshl_or_b32 per half); letters past the register's width fall off
// the top.  The id is the first k letters, the first one most significant:
// the bit reversal of the accumulator, shifted down to k bits.
struct Acc32 {
  static constexpr bool kKron = false;
  using Id = uint32_t;
  using Packed = uint2;
  uint32_t row, col;
  __device__ __forceinline__ void clear() { row = 0; col = 0; }
  __device__ __forceinline__ void first(uint32_t rowv, uint32_t colv) { row = rowv; col = colv; }
  __device__ __forceinline__ void append(uint32_t rowv, uint32_t colv, uint32_t, uint32_t filled, uint32_t,
                                         const KronPow*) {
    row |= rowv << filled;
    col |= colv << filled;
  }
  __device__ __forceinline__ void trim(uint32_t, uint32_t, const KronPow*) {}
  __device__ __forceinline__ uint32_t src(uint32_t k) const { return __builtin_bitreverse32(row) >> (32 - k); }
  __device__ __forceinline__ uint32_t dst(uint32_t k) const { return __builtin_bitreverse32(col) >> (32 - k); }
  // the ids' letters first-most-significant, before the shift down to k bits
  __device__ __forceinline__ uint32_t src_fill() const { return __builtin_bitreverse32(row); }
  __device__ __forceinline__ uint32_t dst_fill() const { return __builtin_bitreverse32(col); }
  __device__ __forceinline__ Packed pack() const { return make_uint2(row, col); }
  __device__ __forceinline__ void unpack(const Packed& p) { row = p.x; col = p.y; }
};

struct Acc64 {
  static constexpr bool kKron = false;
  using Id = uint64_t;
  using Packed = ulonglong2;
  uint64_t row, col;
  __device__ __forceinline__ void clear() { row = 0; col = 0; }
  __device__ __forceinline__ void first(uint32_t rowv, uint32_t colv) { row = rowv; col = colv; }
  __device__ __forceinline__ void append(uint32_t rowv, uint32_t colv, uint32_t, uint32_t filled, uint32_t,
                                         const KronPow*) {
    row |= static_cast<uint64_t>(rowv) << filled;
    col |= static_cast<uint64_t>(colv) << filled;
  }
  __device__ __forceinline__ void trim(uint32_t, uint32_t, const KronPow*) {}
  __device__ __forceinline__ uint64_t src(uint32_t k) const { return __builtin_bitreverse64(row) >> (64 - k); }
  __device__ __forceinline__ uint64_t dst(uint32_t k) const { return __builtin_bitreverse64(col) >> (64 - k); }
  __device__ __forceinline__ Packed pack() const { return make_ulonglong2(row, col); }
  __device__ __forceinline__ void unpack(const Packed& p) { row = p.x; col = p.y; }
};

// Base-K accumulators for K x K initiators: a path of L digit pairs holds
// its row and column digits as base-K numbers (root-most digit most
// significant), and the id is the first k digits of the edge's paths.
// 64-bit ids append the first min(L, k - filled) digits of each path by
// id = id * K^take + value / K^(L - take); path values are below 2^15 and
// the divisor K^(L - take) is at least K, so the quotient is a multiply-high
// by KronPow::magic.  32-bit ids (K^k <= 2^32) append every path whole, with
// one 32 x 32 + 32 multiply-add whose 64-bit result is exact: the value
// before the last path is below K^(k-1) < 2^32, so the last one ends below
// 2^32 * K^L <= 2^47, and trim() divides it once by K^(filled - k).  The
// quotient q < 2^32 is the truncated double product value * rcp[filled - k]:
// with value = q K^d + r, 0 <= r < K^d <= 2^15, the exact product lies in
// [value / K^d, value / K^d + 2^-19), rounding moves it by at most 2^-22 and
// not below an integer it is at or above, and value / K^d is an integer or
// at least 2^-15 from both neighbours, so the truncation is q.
template <typename IdT>
struct KronAcc {
  static constexpr bool kKron = true;
  static constexpr bool kNarrow = sizeof(IdT) == 4;
  using Id = IdT;
  using Packed = typename std::conditional<kNarrow, uint2, ulonglong2>::type;
  Id row, col;
  uint32_t row_hi, col_hi;  // 32-bit ids: bits 32 and up of the last path's product
  __device__ __forceinline__ void clear() {
    row = 0;
    col = 0;
    if constexpr (kNarrow) row_hi = col_hi = 0;
  }
  // an edge's first path when it is taken whole (k is above the longest path)
  __device__ __forceinline__ void first(uint32_t rowv, uint32_t colv) {
    row = rowv;
    col = colv;
    if constexpr (kNarrow) row_hi = col_hi = 0;
  }
  __device__ __forceinline__ void append(uint32_t rowv, uint32_t colv, uint32_t len, uint32_t filled, uint32_t k,
                                         const KronPow* kpow) {
    if constexpr (kNarrow) {
      const uint32_t mul = static_cast<uint32_t>(kpow->pow[len]);
      const uint64_t r = mad_u64_u32(row, mul, rowv), c = mad_u64_u32(col, mul, colv);
      row = static_cast<uint32_t>(r);
      row_hi = static_cast<uint32_t>(r >> 32);
      col = static_cast<uint32_t>(c);
      col_hi = static_cast<uint32_t>(c >> 32);
    } else {
      const uint32_t take = len < k - filled ? len : k - filled;
      if (take < len) {  // the edge's last path, cut to the digits still needed
        const uint32_t mg = kpow->magic[len - take];
        rowv = static_cast<uint32_t>(mad_u64_u32(rowv, mg, 0) >> 32);
        colv = static_cast<uint32_t>(mad_u64_u32(colv, mg, 0) >> 32);
      }
      const Id mul = static_cast<Id>(kpow->pow[take]);
      row = row * mul + rowv;
      col = col * mul + colv;
    }
  }
  // 32-bit ids: the first k of `filled` digits (filled >= k; the index is
  // masked only to keep the read inside the table)
  __device__ __forceinline__ void trim(uint32_t filled, uint32_t k, const KronPow* kpow) {
    if constexpr (kNarrow) {
      const double r = kpow->rcp[(filled - k) & 15u];
      row = static_cast<uint32_t>(fma(static_cast<double>(row_hi), 4294967296.0, static_cast<double>(row)) * r);
      col = static_cast<uint32_t>(fma(static_cast<double>(col_hi), 4294967296.0, static_cast<double>(col)) * r);
    }
  }
  __device__ __forceinline__ Id src(uint32_t) const { return row; }
  __device__ __forceinline__ Id dst(uint32_t) const { return col; }
  __device__ __forceinline__ Packed pack() const { return Packed{row, col}; }
  // a queued edge is short of k digits, so its value is all in row and col
  __device__ __forceinline__ void unpack(const Packed& p) {
    row = p.x;
    col = p.y;
    if constexpr (kNarrow) row_hi = col_hi = 0;
  }
};

// A record's own (low) or alias (high) half-words of its three fields.  For
// 32-bit base-K ids, whose path values go straight into 64-bit addends, one
// byte permute per field from a shared selector: there the compiler would
// otherwise mask and shift each half before selecting.
template <typename Acc>
__device__ __forceinline__ void pick(bool own, const BucketRecord& q, uint32_t& len, uint32_t& rowv, uint32_t& colv) {
  if constexpr (Acc::kKron && sizeof(typename Acc::Id) == 4) {
    const uint32_t sel = own ? 0x0C0C0100u : 0x0C0C0302u;  // bytes 1:0 or 3:2, zero above
    len = __builtin_amdgcn_perm(q.lens, q.lens, sel);
    rowv = __builtin_amdgcn_perm(q.rows, q.rows, sel);
    colv = __builtin_amdgcn_perm(q.cols, q.cols, sel);
  } else {
    len = own ? (q.lens & 0xFFFFu) : (q.lens >> 16);
    rowv = own ? (q.rows & 0xFFFFu) : (q.rows >> 16);
    colv = own ? (q.cols & 0xFFFFu) : (q.cols >> 16);
  }
}

// Up to four samples of one Philox block, stopping at k letters, on bucket
// records already loaded.  A sample x keeps its bucket's own path when
// x < thr_abs (its bits other than the bucket's, read in order, are below
// the threshold T), else takes the alias; each field is the low half-word
// for the own item, else the high one.  kSure1: an edge's first block
// (filled = 0) with k > kMaxDepthCap, so the first path is taken whole and
// the second sample is always used (k letters cannot come from one path).
template <typename Acc, bool kSure1 = false>
__device__ __forceinline__ void consume4(uint32_t k, const uint32_t (&x)[4], const BucketRecord (&r)[4], Acc& acc,
                                         uint32_t& filled, const KronPow* kpow) {
  auto half = [](bool own, uint32_t v) { return own ? (v & 0xFFFFu) : (v >> 16); };
  const bool o0 = x[0] < r[0].thr_abs, o1 = x[1] < r[1].thr_abs, o2 = x[2] < r[2].thr_abs, o3 = x[3] < r[3].thr_abs;
  auto take = [&](bool o, const BucketRecord& q) {
    uint32_t len, rowv, colv;
    pick<Acc>(o, q, len, rowv, colv);
    acc.append(rowv, colv, len, filled, k, kpow);
    filled += len;
  };
  if constexpr (kSure1) {  // the edge's first path: whole, no power of K or cut
    acc.first(half(o0, r[0].rows), half(o0, r[0].cols));
    filled = half(o0, r[0].lens);
  } else {
    take(o0, r[0]);
  }
  if (kSure1 || filled < k) {
    take(o1, r[1]);
    if (filled < k) {
      take(o2, r[2]);
      if (filled < k) take(o3, r[3]);
    }
  }
}

// The four samples of a first block with no branches, for the
// bit-concatenating accumulators of the pipelined passes: every path is
// appended whatever the fill level, since letters past k are dropped when the
// id is read.  The first three start at most 2 * kMaxDepthCap < 32
// positions up.  The fourth may start past the register's width: 64-bit ids
// still hold it; for 32-bit ids its shift is clamped to 31, which lands at
// or above bit k only while k < 32 (the callers take this path for k < 32).
// filled ends as the sum of the four lengths, so filled < k exactly when
// consume4 would also have used all four.
template <typename Acc>
__device__ __forceinline__ void consume4_flat(uint32_t k, const uint32_t (&x)[4], const BucketRecord (&r)[4], Acc& acc,
                                              uint32_t& filled) {
  static_assert(!Acc::kKron, "base-K accumulators cut their last path to the digits needed");
  static_assert(2 * kMaxDepthCap < 32, "the first three paths must start inside a 32-bit register");
  auto half = [](bool own, uint32_t v) { return own ? (v & 0xFFFFu) : (v >> 16); };
  const bool o0 = x[0] < r[0].thr_abs, o1 = x[1] < r[1].thr_abs, o2 = x[2] < r[2].thr_abs, o3 = x[3] < r[3].thr_abs;
  auto take = [&](bool o, const BucketRecord& q) {
    const uint32_t len = half(o, q.lens);
    acc.append(half(o, q.rows), half(o, q.cols), len, filled, k, nullptr);
    filled += len;
  };
  take(o0, r[0]);
  take(o1, r[1]);
  take(o2, r[2]);
  if constexpr (sizeof(typename Acc::Id) == 8) {
    take(o3, r[3]);
  } else {
    const uint32_t sh = filled < 31u ? filled : 31u;
    acc.row |= half(o3, r[3].rows) << sh;
    acc.col |= half(o3, r[3].cols) << sh;
    filled += half(o3, r[3].lens);
  }
}

typedef __attribute__((address_space(3))) const BucketRecord* LdsRecordPtr;

// A wave-uniform record of a list that no launch writes (instances, work
// items, running costs), read through the constant address space: the
// compiler may then load it with scalar loads into scalar registers, where a
// plain load, which a store of the same kernel might alias, goes through the
// vector unit and holds the whole record in vector registers.
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "whole words");
  typedef __attribute__((address_space(4))) const uint32_t* ConstWordPtr;
  const ConstWordPtr w = (ConstWordPtr)reinterpret_cast<uintptr_t>(p);
  uint32_t words[sizeof(T) / 4];
#pragma unroll
  for (unsigned i = 0; i < sizeof(T) / 4; ++i) words[i] = w[i];
  T r;
  __builtin_memcpy(&r, words, sizeof(T));
  return r;
}

// The record sample x selects in the table at byte offset toff of a set:
// bucket (x >> 4) mod nb, whose offset within the table is x & bmask with
// bmask = (nb - 1) << 4 (one AND-OR: toff is a multiple of nb * 16).  A set
// staged in LDS starts at LDS address 0 (the generation kernels declare no
// static LDS), so that offset is the read's whole address.
template <bool kLds>
__device__ __forceinline__ BucketRecord record_of(const BucketRecord* __restrict__ set, uint32_t toff, uint32_t bmask,
                                                  uint32_t x) {
  const uint32_t off = toff | (x & bmask);
  if constexpr (kLds)  // an LDS pointer, read through the generic type (the loads stay LDS reads)
    return *(const BucketRecord*)(LdsRecordPtr)static_cast<uintptr_t>(off);
  else
    return *reinterpret_cast<const BucketRecord*>(reinterpret_cast<const char*>(set) + off);
}

// Loads the four bucket records of one Philox block, then samples them.  All
// four reads are issued before any is used, so they are in flight together.
template <typename Acc, bool kLds, bool kSure1 = false>
__device__ __forceinline__ void sample4(const BucketRecord* __restrict__ set, uint32_t toff, uint32_t bmask, uint32_t k,
                                        uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, Acc& acc,
                                        uint32_t& filled, const KronPow* kpow) {
  const uint32_t x[4] = {x0, x1, x2, x3};
  const BucketRecord r[4] = {record_of<kLds>(set, toff, bmask, x0), record_of<kLds>(set, toff, bmask, x1),
                             record_of<kLds>(set, toff, bmask, x2), record_of<kLds>(set, toff, bmask, x3)};
  // keep the reads ahead of the branches below (an operand-only asm, no code)
  __asm__ volatile("" ::"v"(r[1].thr_abs), "v"(r[1].rows), "v"(r[1].cols), "v"(r[1].lens), "v"(r[2].thr_abs),
                   "v"(r[2].rows), "v"(r[2].cols), "v"(r[2].lens), "v"(r[3].thr_abs), "v"(r[3].rows), "v"(r[3].cols),
                   "v"(r[3].lens));
  consume4<Acc, kSure1>(k, x, r, acc, filled, kpow);
}

// The samples of one Philox block with each bucket record loaded only when
// the edge still needs letters (same samples, same order as sample4).  The
// continuation of an edge usually needs one or two of a block's four
// samples, so this saves the unused random reads: line fetches from L2 for a
// table in global memory, LDS reads (and their energy) for one in LDS.
template <typename Acc, bool kLds>
__device__ __forceinline__ void sample_lazy(const BucketRecord* __restrict__ set, uint32_t toff, uint32_t bmask,
                                            uint32_t k, uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, Acc& acc,
                                            uint32_t& filled, const KronPow* kpow) {
  const uint32_t x[4] = {x0, x1, x2, x3};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (filled >= k) break;
    const BucketRecord q = record_of<kLds>(set, toff, bmask, x[i]);
    uint32_t len, rowv, colv;
    pick<Acc>(x[i] < q.thr_abs, q, len, rowv, colv);
    acc.append(rowv, colv, len, filled, k, kpow);
    filled += len;
  }
}

using Inst = GenInst;

// LDS layout shared by both kernels: [table | per-wave queues].
struct TileLayout {
  uint32_t tile;        // blocks per tile
  uint32_t lds_table;   // LDS bytes holding the table (0: read from global memory)
  uint32_t wave_bytes;  // LDS bytes of one wave's queue
  uint32_t waves;       // waves per workgroup
};

struct Launch {
  Inst I;
  TileLayout L;
  uint32_t hist_shift;
  uint16_t* bins;  // reduction: source prefix of edge e at bins[e - I.edge_begin]
  unsigned long long* xor_out;
  uint32_t* degree;  // out-degree counters, one per node (degree launches)
};

struct BatchLaunch {
  const Inst* insts;
  const GenWorkItem* items;
  uint32_t n_items;
  unsigned int* counter;  // reset to 0 by the batch's table-build launch
  TileLayout L;
};

struct TilesLaunch {
  const Inst* insts;
  const uint64_t* cum;  // cum[i]: cost of the instances before i (blocks + inst_cost each)
  uint32_t n_inst;
  uint32_t inst_cost;   // an instance's fixed cost, in blocks
  TileLayout L;
};

// A wave-uniform value held in a vector register: the epilogue's parameters
// stay out of the scalar registers, which the tile loop needs.
__device__ __forceinline__ uint32_t in_vgpr(uint32_t x) {
  uint32_t r;
  __asm__("v_mov_b32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

__device__ __forceinline__ uint64_t in_vgpr(uint64_t x) {
  return (static_cast<uint64_t>(in_vgpr(static_cast<uint32_t>(x >> 32))) << 32) | in_vgpr(static_cast<uint32_t>(x));
}

// The Sec. 3 epilogue of a launch: flags and the scramble's round constants.
template <typename Id>
struct Epilogue {
  uint32_t flags;  // kEpiUndirected | kEpiScramble, wave-uniform
  Id mul[3], add[3], mask;
  uint32_t shift;
  uint32_t width;  // k - shift: the bits a round's xor-shift brings down
};

template <typename Id>
__device__ __forceinline__ Epilogue<Id> make_epilogue(const Inst& I) {
  Epilogue<Id> E;
  E.flags = I.epi;
  for (int r = 0; r < 3; ++r) {
    E.mul[r] = in_vgpr(static_cast<Id>(I.scr_mul[r]));
    E.add[r] = in_vgpr(static_cast<Id>(I.scr_add[r]));
  }
  E.mask = in_vgpr(static_cast<Id>(I.scr_mask));
  E.shift = in_vgpr(I.scr_shift);
  E.width = in_vgpr(I.k - I.scr_shift);
  return E;
}

// The scramble bijection of [0, 2^k): three rounds of an affine map with an
// odd multiplier followed by an xor-shift, each a bijection mod 2^k.  In
// 32-bit arithmetic when the ids are (k <= 32: the low k bits agree).  With
// t the affine map's 32-bit result, the round's value y = t mod 2^k and
// y >> shift is the bit field of t at [shift, k), so a round is the
// multiply-add, one field extract and one three-input and/xor.
__device__ __forceinline__ uint32_t scramble_id(uint32_t x, const Epilogue<uint32_t>& E) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const uint32_t t = static_cast<uint32_t>(mad_u64_u32(x, E.mul[r], E.add[r]));
    x = (t & E.mask) ^ __builtin_amdgcn_ubfe(t, E.shift, E.width);
  }
  return x;
}

__device__ __forceinline__ uint64_t scramble_id(uint64_t x, const Epilogue<uint64_t>& E) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    // low 64 bits of x * mul + add from 32-bit halves
    const uint32_t xl = static_cast<uint32_t>(x), xh = static_cast<uint32_t>(x >> 32);
    const uint32_t ml = static_cast<uint32_t>(E.mul[r]), mh = static_cast<uint32_t>(E.mul[r] >> 32);
    const uint64_t t = mad_u64_u32(xl, ml, E.add[r]);
    uint32_t hi = static_cast<uint32_t>(mad_u64_u32(xl, mh, t >> 32));
    hi = static_cast<uint32_t>(mad_u64_u32(xh, ml, hi));
    x = ((static_cast<uint64_t>(hi) << 32) | static_cast<uint32_t>(t)) & E.mask;
    x ^= x >> E.shift;
  }
  return x;
}

// The Sec. 3 epilogue on one edge, when the launch asks for it (uniform):
// mirror to row <= column, then relabel both ids.
template <bool kGeneral, typename Id>
__device__ __forceinline__ void epilogue(const Epilogue<Id>& E, Id& s, Id& d) {
  if (kGeneral && E.flags != 0) {
    if (E.flags & kEpiUndirected) {
      const Id lo = s < d ? s : d;
      d = s < d ? d : s;
      s = lo;
    }
    if (E.flags & kEpiScramble) {
      s = scramble_id(s, E);
      d = scramble_id(d, E);
    }
  }
}

// One id per lane of a 64-edge block to out[first_slot + lane].  The block's
// address goes into a buffer descriptor (scalar work: dword 3 = 32-bit data
// format, the gfx9 untyped-access value) so the lane's byte offset is the
// store's only vector operand.  In an instance's first block first_slot
// wraps below the buffer; the lanes before edge_begin are inactive there.
constexpr int kBufferDword3 = 0x00020000;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void store_ids(void* out, uint64_t first_slot, uint32_t lane, uint32_t v) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc(static_cast<uint32_t*>(out) + first_slot, 0, 64 * 4, kBufferDword3);
  __builtin_amdgcn_raw_buffer_store_b32(v, r, static_cast<int>(lane * 4), 0, 0);
}

__device__ __forceinline__ void store_ids(void* out, uint64_t first_slot, uint32_t lane, uint64_t v) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc(static_cast<uint64_t*>(out) + first_slot, 0, 64 * 8, kBufferDword3);
  u32x2 w;
  w.x = static_cast<uint32_t>(v);
  w.y = static_cast<uint32_t>(v >> 32);
  __builtin_amdgcn_raw_buffer_store_b64(w, r, static_cast<int>(lane * 8), 0, 0);
}

// A lane's id at byte offset soff (wave-uniform) + lane * size of a buffer.
__device__ __forceinline__ void store_at(__amdgpu_buffer_rsrc_t r, uint32_t lane, uint32_t soff, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, static_cast<int>(lane * 4), static_cast<int>(soff), 0);
}

__device__ __forceinline__ void store_at(__amdgpu_buffer_rsrc_t r, uint32_t lane, uint32_t soff, uint64_t v) {
  u32x2 w;
  w.x = static_cast<uint32_t>(v);
  w.y = static_cast<uint32_t>(v >> 32);
  __builtin_amdgcn_raw_buffer_store_b64(w, r, static_cast<int>(lane * 8), static_cast<int>(soff), 0);
}

// MurmurHash3's 64-bit finaliser.
__device__ __forceinline__ uint64_t fmix64(uint64_t z) {
  z ^= z >> 33;
  z *= 0xFF51AFD7ED558CCDull;
  z ^= z >> 33;
  z *= 0xC4CEB9FE1A85EC53ull;
  z ^= z >> 33;
  return z;
}

// XOR over the 64 lanes of a wave, in every lane.
__device__ __forceinline__ uint64_t wave_xor(uint64_t x) {
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t lo = __shfl_xor(static_cast<uint32_t>(x), o, 64);
    const uint32_t hi = __shfl_xor(static_cast<uint32_t>(x >> 32), o, 64);
    x ^= (static_cast<uint64_t>(hi) << 32) | lo;
  }
  return x;
}

// Orders this wave's LDS accesses across the passes of a tile.
__device__ __forceinline__ void wave_lds_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Lanes of block `rel` (within the instance) whose edge lies in
// [edge_begin, last]: every lane except in the first and the last block.
__device__ __forceinline__ uint64_t block_mask(const GenInst& I, uint64_t rel, uint64_t last) {
  uint64_t mask = ~0ull;
  if (rel == 0) mask <<= (I.edge_begin & 63u);
  if (rel == I.n_blocks - 1) mask &= ~0ull >> (63u - (last & 63u));
  return mask;
}

// Per-wave LDS queue of the edges still short of k letters after their
// first counter block: entry i holds (slot << 6 | filled), slot = j * 64 +
// lane within the tile, and the partial accumulator.  A full wave's worth
// (64 entries) is finished as soon as it is there, so the queue holds at
// most 63 + 64 entries.
constexpr uint32_t kQueueCap = 128;

template <typename Acc>
constexpr uint32_t queue_bytes() {
  return kQueueCap * static_cast<uint32_t>(sizeof(typename Acc::Packed) + sizeof(uint16_t));
}

// Blocks t0 + j*stride of one instance for one wave, t0 = wave_blk,
// wave_blk + stride*tile, ... below blk_end, in tiles of L.tile blocks.
// Each edge's first counter block is drawn in block order; an edge with k
// letters is stored (or reduced) at once, from registers, and the others
// join the wave's queue, which is finished 64 edges at a time (counter
// blocks 1, 2, ...) and emptied at the end of the tile.  kLazy: the table
// set is read from global memory (L2); otherwise it sits at LDS address 0.
// Every block after an edge's first (the first pass's second block, the
// continuations) loads a record only for a sample the edge uses.
template <typename Acc, bool kReduce, bool kDigest = false, bool kGeneral = true, bool kDegree = false,
          bool kLazy = false, bool kTwo = false, bool kPrefix = false, bool kFunnelIds = false>
__device__ __forceinline__ void run_blocks(const Inst& I, const BucketRecord* __restrict__ tab, const TileLayout& L,
                                           uint64_t wave_blk, uint64_t blk_end, uint64_t stride,
                                           typename Acc::Packed* qacc, uint16_t* qent, uint32_t hist_shift,
                                           uint16_t* bins, uint64_t& xsum, const KronPow* kpow = nullptr,
                                           uint32_t* degree = nullptr) {
  using Id = typename Acc::Id;
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t last = I.edge_begin + (I.m - 1);  // last edge, no overflow
  // edge e reads table e mod P; blocks start at multiples of 64 and P divides
  // 64, so in the first pass that is the lane's table for the whole run (at
  // byte offset toff_lane of the set)
  const uint32_t tbytes = I.n_buckets * static_cast<uint32_t>(sizeof(BucketRecord));
  const uint32_t toff_lane = (lane & I.table_mask) * tbytes;
  Epilogue<Id> E;
  if (kGeneral) E = make_epilogue<Id>(I);
  // kPrefix: id prefixes without the epilogue (the tiles of a partitioned graph)
  const Id src_prefix = static_cast<Id>(kGeneral || kPrefix ? I.src_prefix : 0);
  const Id dst_prefix = static_cast<Id>(kGeneral || kPrefix ? I.dst_prefix : 0);
  // kFunnelIds, 32-bit bit-string ids: a prefix (zero below bit k) shifted
  // down by k, so that one funnel shift of (prefix >> k : reversed fill) by
  // 32 - k gives the prefixed id (one vector register more: the batch kernel,
  // at the edge of a register step, keeps the shift and the OR)
  constexpr bool kFunnel = kFunnelIds && (kGeneral || kPrefix) && std::is_same<Acc, Acc32>::value;
  const uint32_t src_hi = kFunnel && I.k < 32 ? static_cast<uint32_t>(src_prefix) >> I.k : 0u;
  const uint32_t dst_hi = kFunnel && I.k < 32 ? static_cast<uint32_t>(dst_prefix) >> I.k : 0u;
  const uint32_t fshift = kFunnel ? in_vgpr(32u - I.k) : 0u;  // a vector operand: the funnel takes one scalar

  // the ids of a finished edge e: reduced, counted, or handed to put(s, d)
  auto finish_edge = [&](Acc acc, uint32_t filled, uint64_t e, auto put) {
    acc.trim(filled, I.k, kpow);
    if (kReduce) {
      const uint64_t s = acc.src(I.k), d = acc.dst(I.k);
      bins[e - I.edge_begin] = static_cast<uint16_t>(hist_shift >= 64 ? 0 : (s >> hist_shift));
      xsum ^= fmix64(e ^ fmix64(s ^ ((d << 32) | (d >> 32))));
    } else if (kDegree) {  // one more edge out of its source
      atomicAdd(degree + acc.src(I.k), 1u);
    } else {
      Id s, d;
      if constexpr (kFunnel) {  // tiles of a partitioned graph carry id prefixes
        s = __builtin_amdgcn_alignbit(src_hi, acc.src_fill(), fshift);
        d = __builtin_amdgcn_alignbit(dst_hi, acc.dst_fill(), fshift);
      } else {
        s = static_cast<Id>(acc.src(I.k));
        d = static_cast<Id>(acc.dst(I.k));
        if (kGeneral || kPrefix) {
          s |= src_prefix;
          d |= dst_prefix;
        }
      }
      epilogue<kGeneral>(E, s, d);
      put(s, d);
      if (kDigest) {
        const uint64_t s64 = s, d64 = d;
        xsum ^= fmix64(e ^ fmix64(s64 ^ ((d64 << 32) | (d64 >> 32))));
      }
    }
  };

  for (uint64_t t0 = wave_blk; t0 < blk_end; t0 += stride * L.tile) {
    // blocks t0 + j * stride below blk_end, at most L.tile (counted without
    // a 64-bit division: only a wave's last tile is short)
    uint32_t nb_tile = L.tile;
    if (blk_end - t0 <= (L.tile - 1) * stride) {
      nb_tile = 1;
      while (t0 + nb_tile * stride < blk_end) ++nb_tile;
    }
    // a full tile of whole blocks (every tile but a few at the ends of the
    // range) runs without per-block lane masks and stores through one buffer
    // descriptor per output array, block j at a scalar offset
    const bool whole_tile = nb_tile == L.tile && stride < (1u << 16) && (t0 != 0 || (I.edge_begin & 63u) == 0) &&
                            (t0 + (nb_tile - 1) * stride != I.n_blocks - 1 || (last & 63u) == 63u);
    const uint64_t slot0 = ((I.first_block + t0) << 6) - I.edge_begin;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(static_cast<Id*>(I.out_src) + slot0, 0, 0x7FFFFFFF, kBufferDword3);
    const __amdgpu_buffer_rsrc_t rd =
        __builtin_amdgcn_make_buffer_rsrc(static_cast<Id*>(I.out_dst) + slot0, 0, 0x7FFFFFFF, kBufferDword3);
    const uint32_t step = static_cast<uint32_t>(stride) * 64u * static_cast<uint32_t>(sizeof(Id));

    // the queued edges [q0, q0 + cnt), one per lane, finished from counter
    // block 1 (2 when the first pass drew two) and stored.  A queued edge is
    // the tile's first edge plus j * stride * 64 + lane: every launch keeps
    // stride (its waves) below 2^16, so that offset is one 24-bit
    // multiply-add, and the stores go through the tile's buffer descriptors
    // at it.
    const uint64_t tile_e0 = (I.first_block + t0) << 6;
    const uint32_t stride64 = static_cast<uint32_t>(stride) << 6;
    auto drain = [&](uint32_t q0, uint32_t cnt) {
      wave_lds_fence();
      if (lane < cnt) {
        const uint32_t entry = qent[q0 + lane];
        Acc acc;
        acc.unpack(qacc[q0 + lane]);
        const uint32_t slot = entry >> 6;
        uint32_t filled = entry & 63u;
        const uint32_t lane_e = slot & 63u;
        const uint32_t off = __umul24(slot >> 6, stride64) + lane_e;
        const uint64_t e = tile_e0 + off;
        const uint32_t e_lo = static_cast<uint32_t>(e), e_hi = static_cast<uint32_t>(e >> 32);
        const uint32_t toff_e = __umul24(lane_e & I.table_mask, tbytes);  // a set member: tbytes < 2^24
        for (uint32_t jj = I.first_blocks == 2 ? 2u : 1u; filled < I.k && jj < kMaxBlocksPerEdge; ++jj) {
          uint32_t x0 = e_lo, x1 = e_hi, x2 = jj, x3 = I.ctr3;
          philox10(x0, x1, x2, x3, I.key0, I.key1);
          sample_lazy<Acc, !kLazy>(tab, toff_e, I.bmask, I.k, x0, x1, x2, x3, acc, filled, kpow);
        }
        finish_edge(acc, filled, e, [&](Id s, Id d) {
          store_at(rs, off, 0u, s);
          store_at(rd, off, 0u, d);
        });
      }
      wave_lds_fence();
    };

    // block j of the tile after its first counter block: finished lanes are
    // emitted, the others queued; a full wave of queued edges is drained
    uint32_t n_q = 0;
    // soff: block j's byte offset from the tile's first block (whole tiles)
    auto settle = [&](uint32_t j, uint64_t base, const Acc& acc, uint32_t filled, bool active, uint32_t soff,
                      auto desc) {
      const bool need = active && filled < I.k;
      const uint64_t qmask = __ballot(need);
      if (active && !need) {
        finish_edge(acc, filled, base + lane, [&](Id s, Id d) {
          if constexpr (decltype(desc)::value) {
            store_at(rs, lane, soff, s);
            store_at(rd, lane, soff, d);
          } else {
            store_ids(I.out_src, base - I.edge_begin, lane, s);
            store_ids(I.out_dst, base - I.edge_begin, lane, d);
          }
        });
      }
      if (qmask != 0) {
        if (need) {
          const uint32_t rank = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(qmask >> 32),
                                                          __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(qmask), 0u));
          qent[n_q + rank] = static_cast<uint16_t>(((j * 64 + lane) << 6) | filled);
          qacc[n_q + rank] = acc.pack();
        }
        n_q += __popcll(qmask);
        if (n_q >= 64) {
          n_q -= 64;
          drain(n_q, 64);
        }
      }
    };

    // counter block 1 of the lanes still short of k letters, in the first
    // pass when the table's edges mostly need it (the same samples, in the
    // same order, as the queue's drain would draw)
    auto second_block = [&](uint64_t base, Acc& acc, uint32_t& filled) {
      if (I.first_blocks == 2 && filled < I.k) {
        uint32_t y0 = static_cast<uint32_t>(base) + lane, y1 = static_cast<uint32_t>(base >> 32), y2 = 1u,
                 y3 = I.ctr3;
        philox10(y0, y1, y2, y3, I.key0, I.key1);
        sample_lazy<Acc, !kLazy>(tab, toff_lane, I.bmask, I.k, y0, y1, y2, y3, acc, filled, kpow);
      }
    };
    auto first_block = [&](uint32_t j, uint64_t base, uint64_t amask, auto whole, auto sure, auto desc) {
      Acc acc;
      acc.clear();
      uint32_t filled = 0;
      uint32_t x0, x1, x2, x3;
      philox10_first(static_cast<uint32_t>(base) + lane, static_cast<uint32_t>(base >> 32), I.ctr3, I.key0, I.key1, x0, x1,
                     x2, x3);
      sample4<Acc, !kLazy, decltype(sure)::value>(tab, toff_lane, I.bmask, I.k, x0, x1, x2, x3, acc, filled, kpow);
      second_block(base, acc, filled);
      settle(j, base, acc, filled, decltype(whole)::value || ((amask >> lane) & 1ull), j * step, desc);
    };
    const bool sure1 = I.k > static_cast<uint32_t>(kMaxDepthCap);  // a path has at most kMaxDepthCap letters
    // the pipelined passes consume a block without branches (consume4_flat):
    // exact for 64-bit ids and base-K accumulators, for 32-bit ids when k < 32
    const bool pipe_ok = sure1 && (Acc::kKron || sizeof(typename Acc::Id) == 8 || I.k < 32u);
    // block j's Philox draws and table reads, issued before block j - 1 is
    // consumed so that the reads overlap work
    auto draw = [&](uint32_t j, uint32_t (&x)[4], BucketRecord (&r)[4]) {
      const uint64_t base = (I.first_block + t0 + j * stride) << 6;
      philox10_first(static_cast<uint32_t>(base) + lane, static_cast<uint32_t>(base >> 32), I.ctr3, I.key0, I.key1,
                     x[0], x[1], x[2], x[3]);
#pragma unroll
      for (int i = 0; i < 4; ++i) r[i] = record_of<!kLazy>(tab, toff_lane, I.bmask, x[i]);
    };
    auto consume = [&](const uint32_t (&x)[4], const BucketRecord (&r)[4], Acc& acc, uint32_t& filled) {
      if constexpr (Acc::kKron)
        consume4<Acc, true>(I.k, x, r, acc, filled, kpow);
      else
        consume4_flat<Acc>(I.k, x, r, acc, filled);
    };
    if (whole_tile && pipe_ok && nb_tile == kMaxTile && (kTwo || I.first_blocks != 2)) {
      // software-pipelined, unrolled; the copy with kTwo also draws counter
      // block 1 in this pass for the lanes that need it (a separate copy:
      // its presence slows the one-block code)
      // a running store offset (the products j * step, kept for all blocks,
      // would crowd the scalar registers)
      uint32_t soff = 0;
      auto finish = [&](uint32_t j, const uint32_t (&x)[4], const BucketRecord (&r)[4]) {
        Acc acc;
        acc.clear();
        uint32_t filled = 0;
        consume(x, r, acc, filled);
        const uint64_t base = (I.first_block + t0 + j * stride) << 6;
        if constexpr (kTwo) second_block(base, acc, filled);
        settle(j, base, acc, filled, true, soff, std::true_type{});
        soff += step;
      };
      uint32_t xa[4];
      BucketRecord ra[4];
      draw(0, xa, ra);
#pragma unroll
      for (uint32_t j = 1; j < kMaxTile; ++j) {
        uint32_t xb[4];
        BucketRecord rb[4];
        draw(j, xb, rb);
        finish(j - 1, xa, ra);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          xa[i] = xb[i];
          ra[i] = rb[i];
        }
      }
      finish(kMaxTile - 1, xa, ra);
    } else if (whole_tile) {
      // other full tiles of whole blocks, rolled
      for (uint32_t j = 0; j < nb_tile; ++j) {
        const uint64_t base = (I.first_block + t0 + j * stride) << 6;
        if (sure1)
          first_block(j, base, ~0ull, std::true_type{}, std::true_type{}, std::true_type{});
        else
          first_block(j, base, ~0ull, std::true_type{}, std::false_type{}, std::true_type{});
      }
    } else {
      for (uint32_t j = 0; j < nb_tile; ++j) {
        const uint64_t rel = t0 + j * stride;              // block index within the instance
        const uint64_t base = (I.first_block + rel) << 6;  // wave-uniform
        const uint64_t amask = block_mask(I, rel, last);
        if (amask == ~0ull)
          first_block(j, base, amask, std::true_type{}, std::false_type{}, std::false_type{});
        else
          first_block(j, base, amask, std::false_type{}, std::false_type{}, std::false_type{});
      }
    }
    if (n_q != 0) drain(0, n_q);
  }
}

__device__ __forceinline__ void stage_table(const BucketRecord* src_rec, uint32_t n_buckets, unsigned char* s_mem) {
  const uint4* src = reinterpret_cast<const uint4*>(src_rec);
  uint4* dst = reinterpret_cast<uint4*>(s_mem);
  for (uint32_t i = threadIdx.x; i < n_buckets; i += blockDim.x) dst[i] = src[i];
}

// kGeneral: the store may carry id prefixes and the epilogue; without it the
// launch stores the plain ids and keeps none of their parameters live.
template <typename Acc, bool kLds, bool kReduce, bool kGeneral, bool kDegree = false, bool kTwo = false>
__global__ __launch_bounds__(kGenThreads) void generate_kernel(Launch P) {
  // all LDS is dynamic: [table set | queues | misc], the set at address 0
  extern __shared__ __align__(16) unsigned char s_mem[];
  unsigned char* misc = s_mem + P.L.lds_table + P.L.waves * P.L.wave_bytes;
  unsigned long long* s_xor = reinterpret_cast<unsigned long long*>(misc);  // kWaves words
  using Packed = typename Acc::Packed;
  const KronPow* kpow = nullptr;
  if constexpr (Acc::kKron) {
    KronPow* s_kpow = reinterpret_cast<KronPow*>(misc + kWaves * sizeof(unsigned long long));
    if (threadIdx.x == 0) {
      uint64_t x = 1;
      for (int i = 0; i < 16; ++i, x *= P.I.kron_k) {
        s_kpow->pow[i] = x;
        s_kpow->magic[i] = static_cast<uint32_t>((1ull << 32) / x + 1);  // used for 2 <= x < 2^15 only
        s_kpow->rcp[i] = __longlong_as_double(__double_as_longlong(1.0 / static_cast<double>(x)) + 1);
      }
    }
    __syncthreads();
    kpow = s_kpow;
  }
  const BucketRecord* tab = P.I.records;
  if (kLds) {
    stage_table(P.I.records, P.I.n_buckets * (P.I.table_mask + 1), s_mem);
    __syncthreads();
    tab = reinterpret_cast<const BucketRecord*>(s_mem);
  }
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave_in_wg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t wave = static_cast<uint64_t>(blockIdx.x) * P.L.waves + wave_in_wg;
  const uint64_t n_waves = static_cast<uint64_t>(gridDim.x) * P.L.waves;
  Packed* qacc = reinterpret_cast<Packed*>(s_mem + P.L.lds_table + wave_in_wg * P.L.wave_bytes);
  uint16_t* qent = reinterpret_cast<uint16_t*>(qacc + kQueueCap);
  uint64_t xsum = 0;
  run_blocks<Acc, kReduce, false, kGeneral, kDegree, !kLds, kTwo, false, true>(
      P.I, tab, P.L, wave, P.I.n_blocks, n_waves, qacc, qent, P.hist_shift, P.bins, xsum, kpow, P.degree);
  if (kReduce) {
    const uint64_t x = wave_xor(xsum);
    if (lane == 0) s_xor[wave_in_wg] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long t = 0;
      for (uint32_t w = 0; w < P.L.waves; ++w) t ^= s_xor[w];
      atomicXor(P.xor_out, t);
    }
  }
}

// Persistent kernel over the work items of a batch.  A workgroup claims an
// item, restages the table only when the item's table differs from the one
// in LDS (items are in instance order; the tiles of a partitioned graph and
// requests served from one cached table share it), and its waves share the
// item's blocks.
template <typename Acc, bool kLds, bool kDigest, bool kGeneral>
__global__ __launch_bounds__(kGenThreads) void generate_batch_kernel(BatchLaunch B) {
  // all LDS is dynamic: [table | queues | misc], the table at address 0
  extern __shared__ __align__(16) unsigned char s_mem[];
  uint32_t& s_item = *reinterpret_cast<uint32_t*>(s_mem + B.L.lds_table + B.L.waves * B.L.wave_bytes);
  using Packed = typename Acc::Packed;
  const uint32_t wave_in_wg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  Packed* qacc = reinterpret_cast<Packed*>(s_mem + B.L.lds_table + wave_in_wg * B.L.wave_bytes);
  uint16_t* qent = reinterpret_cast<uint16_t*>(qacc + kQueueCap);
  const BucketRecord* cur = nullptr;  // table in LDS and its buckets
  uint32_t cur_buckets = 0;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(B.counter, 1u);
    __syncthreads();
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();  // everyone has read s_item (and finished the previous item)
    if (item >= B.n_items) break;
    const GenWorkItem W = load_uniform(B.items + item);
    const Inst I = load_uniform(B.insts + W.inst);
    const uint32_t buckets = I.n_buckets * (I.table_mask + 1);
    if (kLds && (I.records != cur || buckets != cur_buckets)) {
      stage_table(I.records, buckets, s_mem);
      __syncthreads();
      cur = I.records;
      cur_buckets = buckets;
    }
    if (W.n_inst > 1) {
      // a run of small instances on this table: each wave takes whole
      // instances (no workgroup step between them)
      for (uint32_t j = wave_in_wg; j < W.n_inst; j += B.L.waves) {
        const Inst Ij = load_uniform(B.insts + W.inst + j);
        const BucketRecord* tab = kLds ? reinterpret_cast<const BucketRecord*>(s_mem) : Ij.records;
        uint64_t xsum = 0;
        run_blocks<Acc, false, kDigest, kGeneral, false, !kLds>(Ij, tab, B.L, 0, Ij.n_blocks, 1, qacc, qent, 0,
                                                               nullptr, xsum);
        if (kDigest && Ij.digest != nullptr) {
          const uint64_t x = wave_xor(xsum);
          if ((threadIdx.x & 63) == 0 && x != 0) atomicXor(Ij.digest, x);
        }
      }
      continue;
    }
    const BucketRecord* tab = kLds ? reinterpret_cast<const BucketRecord*>(s_mem) : I.records;
    uint64_t xsum = 0;
    run_blocks<Acc, false, kDigest, kGeneral, false, !kLds>(I, tab, B.L, W.first + wave_in_wg, W.first + W.n_blocks,
                                                           B.L.waves, qacc, qent, 0, nullptr, xsum);
    if (kDigest && I.digest != nullptr) {
      const uint64_t x = wave_xor(xsum);
      if ((threadIdx.x & 63) == 0 && x != 0) atomicXor(I.digest, x);
    }
  }
}

// The tiles of a partitioned graph: instances on one table (staged once per
// workgroup) laid out in list order on one line of cost, each instance a
// fixed cost (its setup, its partial tiles and drains, in blocks) followed by
// its blocks; the grid's waves share the line in equal contiguous parts.  A
// wave finds the instance holding the start of its part with a 64-way search
// (three rounds for 2^18 instances) and runs every instance whose blocks meet
// its part over those blocks; no work is claimed and no workgroup waits
// after the staging, and a run of tiny tiles weighs as much as its cost.
template <typename Acc, bool kLds>
__global__ __launch_bounds__(kGenThreads) void generate_tiles_kernel(TilesLaunch P) {
  extern __shared__ __align__(16) unsigned char s_mem[];
  using Packed = typename Acc::Packed;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave_in_wg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  Packed* qacc = reinterpret_cast<Packed*>(s_mem + P.L.lds_table + wave_in_wg * P.L.wave_bytes);
  uint16_t* qent = reinterpret_cast<uint16_t*>(qacc + kQueueCap);
  if (kLds) {
    stage_table(P.insts[0].records, P.insts[0].n_buckets, s_mem);
    __syncthreads();
  }
  // this wave's part [lo, hi) of the line
  const uint64_t total = P.cum[P.n_inst];
  const uint64_t n_waves = static_cast<uint64_t>(gridDim.x) * P.L.waves;
  const uint64_t w = static_cast<uint64_t>(blockIdx.x) * P.L.waves + wave_in_wg;
  const uint64_t q = total / n_waves, r = total % n_waves;
  const uint64_t lo = q * w + (w < r ? w : r), hi = lo + q + (w < r ? 1 : 0);
  if (lo >= hi) return;
  // the instance holding position lo: cum[a] <= lo < cum[b] narrows to b = a + 1
  uint32_t a = 0, b = P.n_inst;
  while (b - a > 1) {
    const uint32_t step = (b - a + 63) / 64;
    const uint32_t idx = a + lane * step;
    const uint64_t below = __ballot(idx < b && P.cum[idx] <= lo);  // a prefix of the lanes, lane 0 in it
    const uint32_t last = 63u - static_cast<uint32_t>(__builtin_clzll(below));
    a += last * step;
    b = a + step < b ? a + step : b;
  }
  // the same in every lane: instances load through the scalar unit
  a = __builtin_amdgcn_readfirstlane(a);
  uint64_t xsum = 0;
  for (uint32_t i = a; i < P.n_inst; ++i) {
    const uint64_t ci = load_uniform(P.cum + i);
    if (ci >= hi) break;
    // the instance's blocks sit at [c0, c1) on the line, after its fixed cost
    const uint64_t c0 = ci + P.inst_cost, c1 = load_uniform(P.cum + i + 1);
    const uint64_t end = hi < c1 ? hi : c1;
    if (end <= c0) continue;  // the part ends inside the fixed cost: the next wave runs it
    const uint64_t b0 = lo > c0 ? lo - c0 : 0, b1 = end - c0;
    const Inst I = load_uniform(P.insts + i);
    const BucketRecord* tab = kLds ? reinterpret_cast<const BucketRecord*>(s_mem) : I.records;
    run_blocks<Acc, false, false, false, false, !kLds, false, true, true>(I, tab, P.L, b0, b1, 1, qacc, qent, 0,
                                                                          nullptr, xsum);
  }
}

struct DeviceLimits {
  int cu_count = 0;
  int lds_per_block = 0;
};

DeviceLimits g_limits;

const DeviceLimits& limits() {
  if (g_limits.cu_count == 0) {
    int dev = 0, n = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lds <= 0)
      lds = 64 * 1024;
    g_limits.cu_count = n;
    g_limits.lds_per_block = lds;
  }
  return g_limits;
}

// Waves per workgroup a launch may take, most first: one workgroup of 16
// shares a table copy among the most waves, two of 12 fit twice a 64 KiB
// table's LDS with more waves per CU where registers allow.
constexpr uint32_t kWaveChoices[] = {16, 12, 8};
constexpr uint32_t kMinWaves = 8;

// LDS bytes after the table and the queues: the reduction's per-wave words
// and the base-K powers (or a batch's claimed item).
constexpr size_t kMiscLds = kWaves * sizeof(unsigned long long) + sizeof(KronPow);

bool fits_lds(size_t bytes) { return bytes + kMiscLds <= static_cast<size_t>(limits().lds_per_block); }

// Workgroups of kernel fn resident per CU at `waves` waves and `bytes` of
// dynamic LDS, from the runtime's occupancy calculator (cached; -1 if the
// query failed).
int resident_groups(const void* fn, uint32_t waves, size_t bytes) {
  struct Entry {
    const void* fn;
    uint32_t waves;
    size_t bytes;
    int n;
  };
  static std::mutex mu;
  static std::vector<Entry> cache;
  {
    std::lock_guard<std::mutex> lock(mu);
    for (const Entry& c : cache)
      if (c.fn == fn && c.waves == waves && c.bytes == bytes) return c.n;
  }
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, static_cast<int>(waves * 64), bytes) != hipSuccess) {
    (void)hipGetLastError();
    n = -1;
  }
  std::lock_guard<std::mutex> lock(mu);
  cache.push_back(Entry{fn, waves, bytes, n});
  return n;
}

// Layout of a launch of kernel fn over a table of `buckets` (staged when
// lds): the waves per workgroup that keep the most waves resident per CU,
// its LDS bytes and resident workgroups.  tile = 0 when no layout fits.
template <typename Acc>
TileLayout layout_for(const void* fn, uint32_t buckets, bool lds, size_t* lds_bytes, uint32_t* per_cu) {
  TileLayout L;
  L.lds_table = lds ? buckets * static_cast<uint32_t>(sizeof(BucketRecord)) : 0;
  L.wave_bytes = queue_bytes<Acc>();
  L.tile = 0;
  L.waves = 0;
  uint32_t best = 0;
  for (uint32_t w : kWaveChoices) {
    const size_t bytes = L.lds_table + static_cast<size_t>(w) * L.wave_bytes + kMiscLds;
    if (bytes > static_cast<size_t>(limits().lds_per_block)) continue;
    int n = resident_groups(fn, w, bytes);
    if (n < 0) n = 1;  // no answer: one workgroup, which the LDS allows
    if (static_cast<uint32_t>(n) * w > best) {
      best = static_cast<uint32_t>(n) * w;
      L.waves = w;
      *per_cu = static_cast<uint32_t>(n);
      *lds_bytes = bytes;
    }
  }
  if (best) L.tile = kMaxTile;
  return L;
}

template <typename Acc, bool kLds, bool kReduce, bool kGeneral, bool kDegree = false, bool kTwo = false>
hipError_t launch_one(Launch P, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&generate_kernel<Acc, kLds, kReduce, kGeneral, kDegree, kTwo>);
  size_t lds = 0;
  uint32_t per_cu = 0;
  P.L = layout_for<Acc>(fn, P.I.n_buckets * (P.I.table_mask + 1), kLds, &lds, &per_cu);
  if (P.L.tile == 0) return hipErrorInvalidValue;
  const uint64_t waves_needed = (P.I.n_blocks + P.L.tile - 1) / P.L.tile;
  const uint64_t wgs_needed = (waves_needed + P.L.waves - 1) / P.L.waves;
  uint64_t grid = static_cast<uint64_t>(limits().cu_count) * per_cu;
  if (grid > wgs_needed) grid = wgs_needed;
  if (grid < 1) grid = 1;
  if (grid * P.L.waves >= (1u << 16)) return hipErrorInvalidValue;  // the queue's 24-bit offsets
  hipLaunchKernelGGL((generate_kernel<Acc, kLds, kReduce, kGeneral, kDegree, kTwo>), dim3(static_cast<uint32_t>(grid)),
                     dim3(P.L.waves * 64), lds, s, P);
  return hipGetLastError();
}

// Distribution of out-degrees: each workgroup reads a grid-stride share of
// the counters 16 bytes at a time, keeps degrees 0..3 (most nodes of an
// R-MAT graph) in registers, counts degrees below lds_bins in LDS and larger
// ones with global atomics, then adds its counts to the caller's histogram.
// A degree above max_degree counts as max_degree.  Per-workgroup counts stay
// below 2^32 while n < 2^40.
constexpr uint32_t kDegThreads = 512;
constexpr uint32_t kDegLdsBins = 8192;  // 32 KB of counters

__global__ __launch_bounds__(kDegThreads) void degree_hist_kernel(const uint32_t* __restrict__ degree, uint64_t n,
                                                                   uint32_t max_degree, uint32_t lds_bins,
                                                                   unsigned long long* __restrict__ hist) {
  extern __shared__ uint32_t s_bins[];
  for (uint32_t i = threadIdx.x; i < lds_bins; i += kDegThreads) s_bins[i] = 0;
  __syncthreads();
  uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  auto count = [&](uint32_t v) {
    const uint32_t b = v < max_degree ? v : max_degree;
    c0 += b == 0;
    c1 += b == 1;
    c2 += b == 2;
    c3 += b == 3;
    if (b >= 4) {
      if (b < lds_bins)
        atomicAdd(s_bins + b, 1u);
      else
        atomicAdd(hist + b, 1ull);
    }
  };
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kDegThreads;
  const uint64_t first = static_cast<uint64_t>(blockIdx.x) * kDegThreads + threadIdx.x;
  const uint64_t n4 = n / 4;
  const uint4* d4 = reinterpret_cast<const uint4*>(degree);
  for (uint64_t i = first; i < n4; i += stride) {
    const uint4 v = d4[i];
    count(v.x);
    count(v.y);
    count(v.z);
    count(v.w);
  }
  for (uint64_t i = 4 * n4 + first; i < n; i += stride) count(degree[i]);
  // bins 0..3 exist (b <= max_degree) only up to max_degree; lds_bins > min(3, max_degree)
  const uint32_t cs[4] = {c0, c1, c2, c3};
  for (uint32_t b = 0; b < 4 && b <= max_degree; ++b)
    if (cs[b]) atomicAdd(s_bins + b, cs[b]);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < lds_bins; i += kDegThreads)
    if (s_bins[i]) atomicAdd(hist + i, static_cast<unsigned long long>(s_bins[i]));
}

// Histogram of 16-bit bin values: each workgroup counts its slice of the
// values in LDS, one window of 2^15 bins at a time (128 KB of uint32
// counters), and writes the window's counts to its own row of `partials`
// (row (w * G + g), kHistWindow entries).  No global atomics.
constexpr int kHistThreads = 1024;
constexpr uint32_t kHistWindow = 1u << 15;

__global__ __launch_bounds__(kHistThreads) void hist_partial_kernel(const uint16_t* __restrict__ bins, uint64_t n,
                                                                    uint32_t n_windows,
                                                                    uint32_t* __restrict__ partials) {
  extern __shared__ uint32_t s_cnt[];
  const uint32_t G = gridDim.x, g = blockIdx.x;
  const uint64_t n8 = n / 8;  // whole 16-byte groups of 8 values
  const uint64_t lo8 = n8 * g / G, hi8 = n8 * (g + 1) / G;
  const uint4* v8 = reinterpret_cast<const uint4*>(bins);
  for (uint32_t w = 0; w < n_windows; ++w) {
    for (uint32_t j = threadIdx.x; j < kHistWindow; j += kHistThreads) s_cnt[j] = 0;
    __syncthreads();
    auto count = [w](uint32_t v) {
      if ((v >> 15) == w) atomicAdd(&s_cnt[v & (kHistWindow - 1)], 1u);
    };
    for (uint64_t i = lo8 + threadIdx.x; i < hi8; i += kHistThreads) {
      const uint4 q = v8[i];
      count(q.x & 0xFFFFu);
      count(q.x >> 16);
      count(q.y & 0xFFFFu);
      count(q.y >> 16);
      count(q.z & 0xFFFFu);
      count(q.z >> 16);
      count(q.w & 0xFFFFu);
      count(q.w >> 16);
    }
    if (g == G - 1)
      for (uint64_t i = n8 * 8 + threadIdx.x; i < n; i += kHistThreads) count(bins[i]);
    __syncthreads();
    uint32_t* out = partials + (static_cast<uint64_t>(w) * G + g) * kHistWindow;
    for (uint32_t j = threadIdx.x; j < kHistWindow; j += kHistThreads) out[j] = s_cnt[j];
    __syncthreads();  // the next window clears s_cnt
  }
}

// hist[b] += sum over the G partial rows of bin b (one thread per bin, so a
// plain read-modify-write).
__global__ __launch_bounds__(256) void hist_merge_kernel(const uint32_t* __restrict__ partials, uint32_t G,
                                                         uint32_t n_bins, unsigned long long* __restrict__ hist) {
  const uint32_t b = blockIdx.x * 256 + threadIdx.x;
  if (b >= n_bins) return;
  const uint32_t w = b / kHistWindow, j = b % kHistWindow;
  uint64_t sum = 0;
  for (uint32_t g = 0; g < G; ++g) sum += partials[(static_cast<uint64_t>(w) * G + g) * kHistWindow + j];
  hist[b] += sum;
}

uint32_t hist_groups(uint64_t n) {
  const uint64_t want = (n + 65535) / 65536;
  const uint64_t cus = static_cast<uint64_t>(limits().cu_count);
  return static_cast<uint32_t>(want < 1 ? 1 : (want > cus ? cus : want));
}

// One launch's instance over the call's whole edge range.
Launch make_launch(const GenerateArgs& a) {
  Launch P;
  P.I.records = a.records;
  P.I.n_buckets = a.n_buckets;
  P.I.table_mask = a.n_tables > 1 ? a.n_tables - 1 : 0;
  P.I.bmask = ((1u << a.bucket_bits) - 1u) << 4;
  P.I.k = static_cast<uint32_t>(a.k);
  P.I.key0 = static_cast<uint32_t>(a.seed);
  P.I.key1 = static_cast<uint32_t>(a.seed >> 32);
  P.I.edge_begin = a.edge_begin;
  P.I.m = a.m;
  P.I.first_block = a.edge_begin >> 6;
  P.I.n_blocks = ((a.edge_begin + (a.m - 1)) >> 6) - P.I.first_block + 1;
  P.I.out_src = a.out_src;
  P.I.out_dst = a.out_dst;
  P.I.digest = nullptr;
  P.I.ctr3 = 0;
  P.I.first_blocks = a.first_blocks == 2 ? 2u : 1u;
  P.I.kron_k = static_cast<uint32_t>(a.kron_k);
  P.I.src_prefix = P.I.dst_prefix = 0;
  P.I.epi = 0;
  P.hist_shift = static_cast<uint32_t>(a.k - a.hist_bits);
  P.bins = a.bins;
  P.xor_out = a.xor_out;
  P.degree = a.degree;
  return P;
}

template <bool kReduce>
hipError_t dispatch(const GenerateArgs& a, hipStream_t s) {
  if (a.m == 0) return hipSuccess;
  Launch P = make_launch(a);
  if (!kReduce && a.epi) {
    P.I.epi = a.epi;
    scramble_params(a.scramble_key, a.k, &P.I);
  }
  const bool wide = a.k > 32;
  // two counter blocks in the first pass only where the kernel has the
  // unrolled copy for it (plain stores); the reduction and the epilogue take
  // one, which their pipelined path then serves
  const bool two = !kReduce && a.epi == 0 && a.first_blocks == 2;
  P.I.first_blocks = two ? 2u : 1u;
  auto gen = [&](const Launch& L) {
    auto plain = [&](auto acc, auto lds) {
      using A = decltype(acc);
      constexpr bool kL = decltype(lds)::value;
      return two ? launch_one<A, kL, false, false, false, true>(L, s) : launch_one<A, kL, false, false, false>(L, s);
    };
    using T = std::true_type;
    using F = std::false_type;
    if (!kReduce && a.kron_k > 2) {  // base-K digits; no epilogue, reduction or sets for these tables
      if (a.id_bytes == 4) return a.lds ? plain(KronAcc<uint32_t>{}, T{}) : plain(KronAcc<uint32_t>{}, F{});
      return a.lds ? plain(KronAcc<uint64_t>{}, T{}) : plain(KronAcc<uint64_t>{}, F{});
    }
    if (!kReduce && L.I.epi != 0) {
      if (a.lds) return wide ? launch_one<Acc64, true, false, true>(L, s) : launch_one<Acc32, true, false, true>(L, s);
      return wide ? launch_one<Acc64, false, false, true>(L, s) : launch_one<Acc32, false, false, true>(L, s);
    }
    if (!kReduce) {
      if (a.lds) return wide ? plain(Acc64{}, T{}) : plain(Acc32{}, T{});
      return wide ? plain(Acc64{}, F{}) : plain(Acc32{}, F{});
    }
    if (a.lds) return wide ? launch_one<Acc64, true, true, false>(L, s) : launch_one<Acc32, true, true, false>(L, s);
    return wide ? launch_one<Acc64, false, true, false>(L, s) : launch_one<Acc32, false, true, false>(L, s);
  };
  if (!kReduce) return gen(P);
  // reduction: sub-chunks of at most bins_cap edges, each generated into the
  // 16-bit bin buffer, then counted and merged into the caller's histogram
  const uint32_t n_bins = 1u << a.hist_bits;
  const uint32_t n_windows = (n_bins + kHistWindow - 1) / kHistWindow;
  for (uint64_t off = 0; off < a.m; off += a.bins_cap) {
    const uint64_t len = a.m - off < a.bins_cap ? a.m - off : a.bins_cap;
    Launch L = P;
    L.I.edge_begin = a.edge_begin + off;
    L.I.m = len;
    L.I.first_block = L.I.edge_begin >> 6;
    L.I.n_blocks = ((L.I.edge_begin + (len - 1)) >> 6) - L.I.first_block + 1;
    hipError_t e = gen(L);
    if (e != hipSuccess) return e;
    uint32_t G = hist_groups(len);
    if (a.max_hist_groups && G > a.max_hist_groups) G = a.max_hist_groups;
    hipLaunchKernelGGL(hist_partial_kernel, dim3(G), dim3(kHistThreads), kHistWindow * sizeof(uint32_t), s, a.bins,
                       len, n_windows, a.partials);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(hist_merge_kernel, dim3((n_bins + 255) / 256), dim3(256), 0, s, a.partials, G, n_bins,
                       a.hist);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename Acc, bool kLds, bool kDigest, bool kGeneral>
hipError_t launch_batch(const BatchArgs& a, hipStream_t s) {
  BatchLaunch B;
  B.insts = a.insts;
  B.items = a.items;
  B.n_items = a.n_items;
  B.counter = a.counter;
  const void* fn = reinterpret_cast<const void*>(&generate_batch_kernel<Acc, kLds, kDigest, kGeneral>);
  size_t lds = 0;
  uint32_t per_cu = 0;
  B.L = layout_for<Acc>(fn, a.max_buckets, kLds, &lds, &per_cu);
  if (B.L.tile == 0) return hipErrorInvalidValue;
  uint64_t grid = static_cast<uint64_t>(limits().cu_count) * per_cu;
  if (grid > a.n_items) grid = a.n_items;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((generate_batch_kernel<Acc, kLds, kDigest, kGeneral>), dim3(static_cast<uint32_t>(grid)),
                     dim3(B.L.waves * 64), lds, s, B);
  return hipGetLastError();
}

template <typename Acc, bool kLds>
hipError_t launch_tiles(const TilesArgs& a, hipStream_t s) {
  TilesLaunch P;
  P.insts = a.insts;
  P.cum = a.cum_cost;
  P.n_inst = a.n_inst;
  P.inst_cost = a.inst_cost;
  const void* fn = reinterpret_cast<const void*>(&generate_tiles_kernel<Acc, kLds>);
  size_t lds = 0;
  uint32_t per_cu = 0;
  P.L = layout_for<Acc>(fn, a.n_buckets, kLds, &lds, &per_cu);
  if (P.L.tile == 0) return hipErrorInvalidValue;
  // every resident wave, fewer when there are fewer blocks than waves
  uint64_t grid = static_cast<uint64_t>(limits().cu_count) * per_cu;
  const uint64_t wgs_needed = (a.total_blocks + P.L.waves - 1) / P.L.waves;
  if (grid > wgs_needed) grid = wgs_needed;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((generate_tiles_kernel<Acc, kLds>), dim3(static_cast<uint32_t>(grid)), dim3(P.L.waves * 64),
                     lds, s, P);
  return hipGetLastError();
}

template <typename F>
hipError_t allow_full_lds(F* fn) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                             limits().lds_per_block);
}

// A generation kernel: all of its LDS must be dynamic, so that a staged
// table starts at LDS address 0 (its records are addressed by offset alone).
template <typename F>
hipError_t prepare_generation(F* fn) {
  hipFuncAttributes attr;
  hipError_t e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(fn));
  if (e != hipSuccess) return e;
  if (attr.sharedSizeBytes != 0) return hipErrorInvalidDeviceFunction;
  return allow_full_lds(fn);
}

}  // namespace

// Largest power-of-two table (in buckets, at most 2^13) staged in LDS: it
// must leave room for the queues of the fewest waves a workgroup takes, in
// the widest (64-bit id) layout.
uint32_t lds_table_limit() {
  const size_t queues = static_cast<size_t>(kMinWaves) * queue_bytes<Acc64>();
  uint32_t nb = 1;
  while (nb < (1u << 13) && fits_lds(2 * nb * sizeof(BucketRecord) + queues)) nb <<= 1;
  return fits_lds(nb * sizeof(BucketRecord) + queues) ? nb : 0;
}

uint64_t reduce_partials_bytes() {
  return 2ull * static_cast<uint64_t>(limits().cu_count) * kHistWindow * sizeof(uint32_t);
}

// Workspace of the allocation-free reduction, one copy per device for the
// life of the process: 16-bit bins of one sub-chunk, then up to two windows
// of kStaticHistGroups partial rows (hist_bits <= 16).  Every byte a call
// reads is written earlier in the same call (the bins of a sub-chunk by its
// generation, each partial row by the counting kernel), so nothing needs
// clearing between calls.
constexpr uint64_t kStaticBinsBytes = kStaticReduceChunk * sizeof(uint16_t);
constexpr uint64_t kStaticScratchBytes =
    kStaticBinsBytes + 2ull * kStaticHistGroups * kHistWindow * sizeof(uint32_t);
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_reduce_workspace(GenerateArgs* a) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
      // the device address of this device's copy; host code uses only it
      void* d = nullptr;
      e = hipGetSymbolAddress(&d, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return e;
      ptr[dev] = d;
    }
    p = ptr[dev];
  }
  a->bins = static_cast<uint16_t*>(p);
  a->bins_cap = kStaticReduceChunk;
  a->partials = reinterpret_cast<uint32_t*>(static_cast<char*>(p) + kStaticBinsBytes);
  a->max_hist_groups = kStaticHistGroups;
  return hipSuccess;
}

hipError_t launch_generate(const GenerateArgs& a, hipStream_t s) { return dispatch<false>(a, s); }

hipError_t launch_generate_degrees(const GenerateArgs& a, hipStream_t s) {
  if (a.m == 0) return hipSuccess;
  Launch P = make_launch(a);
  P.I.first_blocks = 1;  // the counting kernel has no two-block unrolled copy
  if (a.k > 32)
    return a.lds ? launch_one<Acc64, true, false, false, true>(P, s) : launch_one<Acc64, false, false, false, true>(P, s);
  return a.lds ? launch_one<Acc32, true, false, false, true>(P, s) : launch_one<Acc32, false, false, false, true>(P, s);
}

hipError_t launch_degree_distribution(const uint32_t* degree, uint64_t n, uint32_t max_degree,
                                      unsigned long long* hist, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t lds_bins = max_degree + 1 < kDegLdsBins ? max_degree + 1 : kDegLdsBins;
  const uint64_t per_group = static_cast<uint64_t>(kDegThreads) * 64;  // 64 counters per thread at least
  uint64_t groups = (n + per_group - 1) / per_group;
  const uint64_t cap = 4ull * static_cast<uint64_t>(limits().cu_count);
  if (groups > cap) groups = cap;
  hipLaunchKernelGGL(degree_hist_kernel, dim3(static_cast<uint32_t>(groups)), dim3(kDegThreads),
                     lds_bins * sizeof(uint32_t), s, degree, n, max_degree, lds_bins, hist);
  return hipGetLastError();
}
hipError_t launch_generate_reduce(const GenerateArgs& a, hipStream_t s) { return dispatch<true>(a, s); }

hipError_t launch_generate_batch(const BatchArgs& a, hipStream_t s) {
  if (a.n_items == 0) return hipSuccess;
  // digests and the epilogue/prefix store each take their own instantiation
  auto pick = [&](auto digest, auto general) {
    constexpr bool kD = decltype(digest)::value, kG = decltype(general)::value;
    if (a.wide) return a.lds ? launch_batch<Acc64, true, kD, kG>(a, s) : launch_batch<Acc64, false, kD, kG>(a, s);
    return a.lds ? launch_batch<Acc32, true, kD, kG>(a, s) : launch_batch<Acc32, false, kD, kG>(a, s);
  };
  if (a.digest) return a.general ? pick(std::true_type{}, std::true_type{}) : pick(std::true_type{}, std::false_type{});
  return a.general ? pick(std::false_type{}, std::true_type{}) : pick(std::false_type{}, std::false_type{});
}

hipError_t launch_generate_tiles(const TilesArgs& a, hipStream_t s) {
  if (a.n_inst == 0 || a.total_blocks == 0) return hipSuccess;
  if (a.wide) return a.lds ? launch_tiles<Acc64, true>(a, s) : launch_tiles<Acc64, false>(a, s);
  return a.lds ? launch_tiles<Acc32, true>(a, s) : launch_tiles<Acc32, false>(a, s);
}

uint32_t tile_blocks(uint32_t table_buckets, int wide, int lds) {
  const size_t table = lds ? static_cast<size_t>(table_buckets) * sizeof(BucketRecord) : 0;
  const size_t queues = static_cast<size_t>(kMinWaves) * (wide ? queue_bytes<Acc64>() : queue_bytes<Acc32>());
  return fits_lds(table + queues) ? kMaxTile : 0;
}

hipError_t prepare_kernels() {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e = hipSuccess;
  const hipError_t r[] = {
      prepare_generation(&generate_kernel<Acc32, true, false, false>),
      prepare_generation(&generate_kernel<Acc32, false, false, false>),
      prepare_generation(&generate_kernel<Acc64, true, false, false>),
      prepare_generation(&generate_kernel<Acc64, false, false, false>),
      prepare_generation(&generate_kernel<Acc32, true, false, true>),
      prepare_generation(&generate_kernel<Acc32, false, false, true>),
      prepare_generation(&generate_kernel<Acc64, true, false, true>),
      prepare_generation(&generate_kernel<Acc64, false, false, true>),
      prepare_generation(&generate_kernel<Acc32, true, true, false>),
      prepare_generation(&generate_kernel<Acc32, false, true, false>),
      prepare_generation(&generate_kernel<Acc64, true, true, false>),
      prepare_generation(&generate_kernel<Acc64, false, true, false>),
      prepare_generation(&generate_kernel<Acc32, true, false, false, true>),
      prepare_generation(&generate_kernel<Acc32, false, false, false, true>),
      prepare_generation(&generate_kernel<Acc64, true, false, false, true>),
      prepare_generation(&generate_kernel<Acc64, false, false, false, true>),
      prepare_generation(&generate_batch_kernel<Acc32, true, false, false>),
      prepare_generation(&generate_batch_kernel<Acc32, true, false, true>),
      prepare_generation(&generate_batch_kernel<Acc32, true, true, false>),
      prepare_generation(&generate_batch_kernel<Acc32, true, true, true>),
      prepare_generation(&generate_batch_kernel<Acc32, false, false, false>),
      prepare_generation(&generate_batch_kernel<Acc32, false, false, true>),
      prepare_generation(&generate_batch_kernel<Acc32, false, true, false>),
      prepare_generation(&generate_batch_kernel<Acc32, false, true, true>),
      prepare_generation(&generate_batch_kernel<Acc64, true, false, false>),
      prepare_generation(&generate_batch_kernel<Acc64, true, false, true>),
      prepare_generation(&generate_batch_kernel<Acc64, true, true, false>),
      prepare_generation(&generate_batch_kernel<Acc64, true, true, true>),
      prepare_generation(&generate_batch_kernel<Acc64, false, false, false>),
      prepare_generation(&generate_batch_kernel<Acc64, false, false, true>),
      prepare_generation(&generate_batch_kernel<Acc64, false, true, false>),
      prepare_generation(&generate_batch_kernel<Acc64, false, true, true>),
      allow_full_lds(&hist_partial_kernel),
      prepare_generation(&generate_kernel<KronAcc<uint32_t>, true, false, false>),
      prepare_generation(&generate_kernel<KronAcc<uint64_t>, true, false, false>),
      prepare_generation(&generate_kernel<Acc32, true, false, false, false, true>),
      prepare_generation(&generate_kernel<Acc32, false, false, false, false, true>),
      prepare_generation(&generate_kernel<Acc64, true, false, false, false, true>),
      prepare_generation(&generate_kernel<Acc64, false, false, false, false, true>),
      prepare_generation(&generate_kernel<KronAcc<uint32_t>, true, false, false, false, true>),
      prepare_generation(&generate_kernel<KronAcc<uint64_t>, true, false, false, false, true>),
      prepare_generation(&generate_tiles_kernel<Acc32, true>),
      prepare_generation(&generate_tiles_kernel<Acc32, false>),
      prepare_generation(&generate_tiles_kernel<Acc64, true>),
      prepare_generation(&generate_tiles_kernel<Acc64, false>)};
  for (hipError_t x : r)
    if (x != hipSuccess) e = x;
  if (e == hipSuccess) done = true;
  return e;
}

}  // namespace rmat
