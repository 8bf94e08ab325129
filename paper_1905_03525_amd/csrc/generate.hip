// generate.hip -- the hot path: per-edge Philox draws, alias lookups in an
// LDS-resident (or L2-resident) bucket table, and bit concatenation (Sec. 2,
// the sampling loop), plus the variant that reduces edges on the device
// instead of storing them.
//
// Work split: the absolute edge index space is cut into 64-edge blocks
// aligned to multiples of 64, one block per wave at a time, so the high
// counter word e >> 32 is uniform across a wave and every store instruction
// covers 64 consecutive slots (256 or 512 contiguous bytes per id array).
#include "rmat_internal.h"

namespace rmat {
namespace {

constexpr int kGenThreads = 512;
constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// multiplications, the key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox10(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = kPhiloxM0 * x0, hi0 = __umulhi(kPhiloxM0, x0);
    const uint32_t lo1 = kPhiloxM1 * x2, hi1 = __umulhi(kPhiloxM1, x2);
    const uint32_t y0 = hi1 ^ x1 ^ k0;
    const uint32_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
}

struct Acc32 {
  uint32_t row, col;
  __device__ __forceinline__ void append(uint32_t rowL, uint32_t colL, uint32_t filled) {
    row |= rowL >> filled;
    col |= colL >> filled;
  }
  __device__ __forceinline__ uint32_t src(int k) const { return row >> (32 - k); }
  __device__ __forceinline__ uint32_t dst(int k) const { return col >> (32 - k); }
};

struct Acc64 {
  uint64_t row, col;
  __device__ __forceinline__ void append(uint32_t rowL, uint32_t colL, uint32_t filled) {
    row |= (static_cast<uint64_t>(rowL) << 32) >> filled;
    col |= (static_cast<uint64_t>(colL) << 32) >> filled;
  }
  __device__ __forceinline__ uint64_t src(int k) const { return row >> (64 - k); }
  __device__ __forceinline__ uint64_t dst(int k) const { return col >> (64 - k); }
};

template <typename Acc>
struct IdOf;
template <>
struct IdOf<Acc32> { using type = uint32_t; };
template <>
struct IdOf<Acc64> { using type = uint64_t; };

// One alias sample: bucket x >> (32 - b); own item when x < thr_abs.
template <typename Acc>
__device__ __forceinline__ void sample(const BucketRecord* __restrict__ tab, uint32_t shift, uint32_t x,
                                       Acc& acc, uint32_t& filled) {
  const BucketRecord r = tab[x >> shift];
  const bool own = x < r.thr_abs;
  const uint32_t word = own ? r.self_word : r.alias_word;
  const uint32_t len = own ? (r.lens & 0xFFFFu) : (r.lens >> 16);
  acc.append(word & 0xFFFF0000u, word << 16, filled);
  filled += len;
}

// Draws edge e: Philox counter blocks j = 0, 1, ... until k letters are known.
template <typename Acc>
__device__ __forceinline__ void draw_edge(const BucketRecord* __restrict__ tab, uint32_t shift, uint32_t k,
                                          uint32_t key0, uint32_t key1, uint64_t e, Acc& acc) {
  acc.row = 0;
  acc.col = 0;
  uint32_t filled = 0;
  const uint32_t e_lo = static_cast<uint32_t>(e), e_hi = static_cast<uint32_t>(e >> 32);
  for (uint32_t j = 0; filled < k; ++j) {
    uint32_t x0 = e_lo, x1 = e_hi, x2 = j, x3 = 0;
    philox10(x0, x1, x2, x3, key0, key1);
    sample(tab, shift, x0, acc, filled);
    if (filled < k) sample(tab, shift, x1, acc, filled);
    if (filled < k) sample(tab, shift, x2, acc, filled);
    if (filled < k) sample(tab, shift, x3, acc, filled);
  }
}

struct Launch {
  const BucketRecord* records;
  uint32_t n_buckets;
  uint32_t shift;  // 32 - b
  uint32_t k;
  uint32_t key0, key1;
  uint64_t edge_begin, m;
  uint64_t first_block, n_blocks;
  void* out_src;
  void* out_dst;
  uint32_t hist_shift;
  unsigned long long* hist;
  unsigned long long* xor_out;
};

__device__ __forceinline__ const BucketRecord* stage_table(const Launch& P, bool lds, BucketRecord* s_tab) {
  if (!lds) return P.records;
  const uint4* src = reinterpret_cast<const uint4*>(P.records);
  uint4* dst = reinterpret_cast<uint4*>(s_tab);
  for (uint32_t i = threadIdx.x; i < P.n_buckets; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  return s_tab;
}

template <typename Acc, bool kLds>
__global__ __launch_bounds__(kGenThreads) void generate_kernel(Launch P) {
  extern __shared__ BucketRecord s_tab[];
  using Id = typename IdOf<Acc>::type;
  const BucketRecord* tab = stage_table(P, kLds, s_tab);
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wave = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const uint64_t n_waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
  Id* __restrict__ out_src = static_cast<Id*>(P.out_src);
  Id* __restrict__ out_dst = static_cast<Id*>(P.out_dst);
  const uint64_t end = P.edge_begin + (P.m - 1);  // last edge, no overflow
  for (uint64_t blk = wave; blk < P.n_blocks; blk += n_waves) {
    const uint64_t e = ((P.first_block + blk) << 6) + lane;
    if (e < P.edge_begin || e > end) continue;
    Acc acc;
    draw_edge(tab, P.shift, P.k, P.key0, P.key1, e, acc);
    const uint64_t slot = e - P.edge_begin;
    out_src[slot] = static_cast<Id>(acc.src(P.k));
    out_dst[slot] = static_cast<Id>(acc.dst(P.k));
  }
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

template <typename Acc, bool kLds>
__global__ __launch_bounds__(kGenThreads) void generate_reduce_kernel(Launch P) {
  extern __shared__ BucketRecord s_tab[];
  __shared__ unsigned long long s_xor[kGenThreads / 64];
  const BucketRecord* tab = stage_table(P, kLds, s_tab);
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wave = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const uint64_t n_waves = (static_cast<uint64_t>(gridDim.x) * blockDim.x) >> 6;
  const uint64_t end = P.edge_begin + (P.m - 1);
  uint64_t x = 0;
  for (uint64_t blk = wave; blk < P.n_blocks; blk += n_waves) {
    const uint64_t e = ((P.first_block + blk) << 6) + lane;
    if (e < P.edge_begin || e > end) continue;
    Acc acc;
    draw_edge(tab, P.shift, P.k, P.key0, P.key1, e, acc);
    const uint64_t s = acc.src(P.k), d = acc.dst(P.k);
    atomicAdd(&P.hist[P.hist_shift >= 64 ? 0 : (s >> P.hist_shift)], 1ull);
    x ^= fmix64(e ^ fmix64(s ^ ((d << 32) | (d >> 32))));
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t lo = __shfl_xor(static_cast<uint32_t>(x), o, 64);
    const uint32_t hi = __shfl_xor(static_cast<uint32_t>(x >> 32), o, 64);
    x ^= (static_cast<uint64_t>(hi) << 32) | lo;
  }
  if (lane == 0) s_xor[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kGenThreads / 64; ++w) t ^= s_xor[w];
    atomicXor(P.xor_out, t);
  }
}

int g_cu_count = 0;

int cu_count() {
  if (g_cu_count == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      g_cu_count = n;
    else
      g_cu_count = 256;
  }
  return g_cu_count;
}

template <typename Acc, bool kLds>
hipError_t launch_one(const Launch& P, bool reduce, hipStream_t s) {
  const size_t lds = kLds ? static_cast<size_t>(P.n_buckets) * sizeof(BucketRecord) : 0;
  const void* fn = reduce ? reinterpret_cast<const void*>(&generate_reduce_kernel<Acc, kLds>)
                          : reinterpret_cast<const void*>(&generate_kernel<Acc, kLds>);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  const uint64_t waves_needed = P.n_blocks;
  const uint64_t wgs_needed = (waves_needed + kGenThreads / 64 - 1) / (kGenThreads / 64);
  const uint64_t per_cu = kLds ? (lds > 80 * 1024 ? 1 : (lds > 40 * 1024 ? 2 : 4)) : 4;
  uint64_t grid = static_cast<uint64_t>(cu_count()) * per_cu;
  if (grid > wgs_needed) grid = wgs_needed;
  if (grid < 1) grid = 1;
  if (reduce)
    hipLaunchKernelGGL((generate_reduce_kernel<Acc, kLds>), dim3(static_cast<uint32_t>(grid)), dim3(kGenThreads),
                       lds, s, P);
  else
    hipLaunchKernelGGL((generate_kernel<Acc, kLds>), dim3(static_cast<uint32_t>(grid)), dim3(kGenThreads), lds, s,
                       P);
  return hipGetLastError();
}

hipError_t dispatch(const GenerateArgs& a, bool reduce, hipStream_t s) {
  if (a.m == 0) return hipSuccess;
  Launch P;
  P.records = a.records;
  P.n_buckets = a.n_buckets;
  P.shift = 32u - static_cast<uint32_t>(a.bucket_bits);
  P.k = static_cast<uint32_t>(a.k);
  P.key0 = static_cast<uint32_t>(a.seed);
  P.key1 = static_cast<uint32_t>(a.seed >> 32);
  P.edge_begin = a.edge_begin;
  P.m = a.m;
  P.first_block = a.edge_begin >> 6;
  P.n_blocks = ((a.edge_begin + (a.m - 1)) >> 6) - P.first_block + 1;
  P.out_src = a.out_src;
  P.out_dst = a.out_dst;
  P.hist_shift = static_cast<uint32_t>(a.k - a.hist_bits);
  P.hist = a.hist;
  P.xor_out = a.xor_out;
  const bool wide = a.k > 32;
  if (a.lds) {
    return wide ? launch_one<Acc64, true>(P, reduce, s) : launch_one<Acc32, true>(P, reduce, s);
  }
  return wide ? launch_one<Acc64, false>(P, reduce, s) : launch_one<Acc32, false>(P, reduce, s);
}

}  // namespace

uint32_t lds_table_limit() { return 8192; }

hipError_t launch_generate(const GenerateArgs& a, hipStream_t s) { return dispatch(a, false, s); }
hipError_t launch_generate_reduce(const GenerateArgs& a, hipStream_t s) { return dispatch(a, true, s); }

}  // namespace rmat
