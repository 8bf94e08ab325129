// microbench.hip -- kernels that measure the device ceilings the sampler runs
// against (include/rmat_bench.h): streaming writes, a plain copy, Philox
// block throughput and random LDS reads.
#include "rmat.h"
#include "rmat_bench.h"
#include "rmat_internal.h"

namespace rmat {
namespace {

constexpr int kMbThreads = 256;

template <int kVec>
struct VecOf;
template <>
struct VecOf<4> { using type = uint32_t; };
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <>
struct VecOf<8> { using type = u32x2; };
template <>
struct VecOf<16> { using type = u32x4; };

template <int kVec>
__global__ __launch_bounds__(kMbThreads) void write_kernel(void* dst, uint64_t n_vec) {
  using V = typename VecOf<kVec>::type;
  V* d = static_cast<V*>(dst);
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  V v;
  uint32_t* w = reinterpret_cast<uint32_t*>(&v);
  for (int i = 0; i < kVec / 4; ++i) w[i] = 0x9E3779B9u * (threadIdx.x + i);
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n_vec; i += stride)
    __builtin_nontemporal_store(v, &d[i]);
}

__global__ __launch_bounds__(kMbThreads) void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                          uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;

__device__ __forceinline__ void philox_v0(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3, uint32_t k0,
                                          uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = M0 * x0, hi0 = __umulhi(M0, x0);
    const uint32_t lo1 = M1 * x2, hi1 = __umulhi(M1, x2);
    const uint32_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
    k0 += W0; k1 += W1;
  }
}

__device__ __forceinline__ void philox_v1(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3, uint32_t k0,
                                          uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = static_cast<uint64_t>(x0) * M0, p1 = static_cast<uint64_t>(x2) * M1;
    const uint32_t y0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p1 >> 32), x1, k0, 0x96);
    const uint32_t y2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p0 >> 32), x3, k1, 0x96);
    x0 = y0; x1 = static_cast<uint32_t>(p1); x2 = y2; x3 = static_cast<uint32_t>(p0);
    k0 += W0; k1 += W1;
  }
}

template <int kVariant>
__global__ __launch_bounds__(kMbThreads) void philox_kernel(uint64_t n_blocks, uint32_t k0, uint32_t k1,
                                                            unsigned long long* out) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wave = static_cast<uint64_t>(blockIdx.x) * (kMbThreads / 64) +
                        __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t n_waves = static_cast<uint64_t>(gridDim.x) * (kMbThreads / 64);
  uint32_t acc = 0;
  for (uint64_t blk = wave; (blk << 6) < n_blocks; blk += n_waves) {
    const uint64_t i = (blk << 6) + lane;
    // variants 0 and 1: all four counter words per lane (nothing folds);
    // variant 2: a wave-uniform high word and zero third/fourth words, as in
    // the sampler's first block of an edge
    uint32_t x0 = static_cast<uint32_t>(i);
    uint32_t x1 = kVariant == 2 ? static_cast<uint32_t>((blk << 6) >> 32) : static_cast<uint32_t>(i >> 32);
    uint32_t x2 = kVariant == 2 ? 0u : static_cast<uint32_t>(i >> 63), x3 = x2;
    if (kVariant == 0) philox_v0(x0, x1, x2, x3, k0, k1);
    else philox_v1(x0, x1, x2, x3, k0, k1);
    if (i < n_blocks) acc ^= x0 ^ x1 ^ x2 ^ x3;
  }
  for (int o = 32; o >= 1; o >>= 1) acc ^= __shfl_xor(acc, o, 64);
  if (lane == 0) atomicXor(out, static_cast<unsigned long long>(acc));
}

// Random LDS reads of kWidth bytes: eight independent address streams per
// lane (xorshift), so the rate is bounded by the LDS, not by latency.
template <int kWidth>
__global__ __launch_bounds__(512) void lds_read_kernel(uint64_t n_reads, uint32_t mask,
                                                       unsigned long long* out) {
  __shared__ uint4 tab[4096];
  for (uint32_t i = threadIdx.x; i < 4096; i += blockDim.x)
    tab[i] = make_uint4(i * 0x9E3779B9u, i ^ 0x55u, i * 3u, ~i);
  __syncthreads();
  uint32_t s[8];
  for (int i = 0; i < 8; ++i) s[i] = (blockIdx.x * blockDim.x + threadIdx.x) * 0x9E3779B9u + 0x7F4A7C15u * (i + 1);
  uint32_t acc = 0;
  const char* base = reinterpret_cast<const char*>(tab);
  for (uint64_t r = 0; r < n_reads; r += 8) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      s[i] ^= s[i] << 13;
      s[i] ^= s[i] >> 17;
      s[i] ^= s[i] << 5;
      const uint32_t off = ((s[i] >> 8) & mask) * kWidth;
      if (kWidth == 16) {
        const uint4 v = *reinterpret_cast<const uint4*>(base + off);
        acc ^= v.x ^ v.w;
      } else if (kWidth == 8) {
        const uint2 v = *reinterpret_cast<const uint2*>(base + off);
        acc ^= v.x ^ v.y;
      } else {
        acc ^= *reinterpret_cast<const uint32_t*>(base + off);
      }
    }
  }
  for (int o = 32; o >= 1; o >>= 1) acc ^= __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) atomicXor(out, static_cast<unsigned long long>(acc));
}

// Random reads of kWidth bytes from a table in global memory (an L2-sized
// table stays in L2): eight independent address streams per lane.
template <int kWidth>
__global__ __launch_bounds__(512) void gather_kernel(const char* __restrict__ base, uint64_t n_reads, uint32_t mask,
                                                     unsigned long long* out) {
  uint32_t s[8];
  for (int i = 0; i < 8; ++i) s[i] = (blockIdx.x * blockDim.x + threadIdx.x) * 0x9E3779B9u + 0x7F4A7C15u * (i + 1);
  uint32_t acc = 0;
  for (uint64_t r = 0; r < n_reads; r += 8) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      s[i] ^= s[i] << 13;
      s[i] ^= s[i] >> 17;
      s[i] ^= s[i] << 5;
      const uint64_t off = static_cast<uint64_t>((s[i] >> 4) & mask) * kWidth;
      if (kWidth == 16) {
        const uint4 v = *reinterpret_cast<const uint4*>(base + off);
        acc ^= v.x ^ v.w;
      } else if (kWidth == 8) {
        const uint2 v = *reinterpret_cast<const uint2*>(base + off);
        acc ^= v.x ^ v.y;
      } else {
        acc ^= *reinterpret_cast<const uint32_t*>(base + off);
      }
    }
  }
  for (int o = 32; o >= 1; o >>= 1) acc ^= __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) atomicXor(out, static_cast<unsigned long long>(acc));
}

int grid_for(uint64_t work_items) {
  uint64_t g = (work_items + kMbThreads - 1) / kMbThreads;
  const uint64_t cap = 256ull * 32;
  return static_cast<int>(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace
}  // namespace rmat

extern "C" {

int rmat_bench_write(void* d_dst, uint64_t bytes, int vec_bytes, void* stream) {
  if (!d_dst || bytes % 16 || (vec_bytes != 4 && vec_bytes != 8 && vec_bytes != 16))
    return rmat::set_error(RMAT_EINVAL, "rmat_bench_write: bad pointer, size or vector width");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t n = bytes / vec_bytes;
  const int g = rmat::grid_for(n);
  if (vec_bytes == 4) hipLaunchKernelGGL(rmat::write_kernel<4>, dim3(g), dim3(rmat::kMbThreads), 0, s, d_dst, n);
  if (vec_bytes == 8) hipLaunchKernelGGL(rmat::write_kernel<8>, dim3(g), dim3(rmat::kMbThreads), 0, s, d_dst, n);
  if (vec_bytes == 16) hipLaunchKernelGGL(rmat::write_kernel<16>, dim3(g), dim3(rmat::kMbThreads), 0, s, d_dst, n);
  return rmat::check_launch("rmat_bench_write");
}

int rmat_bench_copy(const void* d_src, void* d_dst, uint64_t bytes, void* stream) {
  if (!d_src || !d_dst || bytes % 16) return rmat::set_error(RMAT_EINVAL, "rmat_bench_copy: bad pointer or size");
  const uint64_t n = bytes / 16;
  hipLaunchKernelGGL(rmat::copy_kernel, dim3(rmat::grid_for(n)), dim3(rmat::kMbThreads), 0,
                     static_cast<hipStream_t>(stream), static_cast<const uint4*>(d_src), static_cast<uint4*>(d_dst), n);
  return rmat::check_launch("rmat_bench_copy");
}

int rmat_bench_philox(uint64_t n_blocks, int variant, uint64_t seed, void* d_out, void* stream) {
  if (!d_out || variant < 0 || variant > 2) return rmat::set_error(RMAT_EINVAL, "rmat_bench_philox: bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int g = rmat::grid_for(n_blocks);
  auto* out = static_cast<unsigned long long*>(d_out);
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  if (variant == 0)
    hipLaunchKernelGGL(rmat::philox_kernel<0>, dim3(g), dim3(rmat::kMbThreads), 0, s, n_blocks, k0, k1, out);
  else if (variant == 1)
    hipLaunchKernelGGL(rmat::philox_kernel<1>, dim3(g), dim3(rmat::kMbThreads), 0, s, n_blocks, k0, k1, out);
  else
    hipLaunchKernelGGL(rmat::philox_kernel<2>, dim3(g), dim3(rmat::kMbThreads), 0, s, n_blocks, k0, k1, out);
  return rmat::check_launch("rmat_bench_philox");
}

int rmat_bench_lds_read(uint64_t n_reads, uint32_t table_bytes, int width, void* d_out, void* stream) {
  if (!d_out || (width != 4 && width != 8 && width != 16) || table_bytes < 16 || table_bytes > 65536 ||
      (table_bytes & (table_bytes - 1)))
    return rmat::set_error(RMAT_EINVAL, "rmat_bench_lds_read: bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* out = static_cast<unsigned long long*>(d_out);
  const uint32_t mask = table_bytes / width - 1;
  const dim3 g(256 * 4), b(512);
  if (width == 16) hipLaunchKernelGGL(rmat::lds_read_kernel<16>, g, b, 0, s, n_reads, mask, out);
  if (width == 8) hipLaunchKernelGGL(rmat::lds_read_kernel<8>, g, b, 0, s, n_reads, mask, out);
  if (width == 4) hipLaunchKernelGGL(rmat::lds_read_kernel<4>, g, b, 0, s, n_reads, mask, out);
  return rmat::check_launch("rmat_bench_lds_read");
}

int rmat_bench_gather(uint64_t n_reads, const void* d_table, uint64_t table_bytes, int width, int blocks_per_cu,
                      void* d_out, void* stream) {
  if (!d_out || !d_table || (width != 4 && width != 8 && width != 16) || table_bytes < 16 ||
      table_bytes > (1ull << 32) || (table_bytes & (table_bytes - 1)) || blocks_per_cu < 1 || blocks_per_cu > 4 ||
      (n_reads % 8))
    return rmat::set_error(RMAT_EINVAL, "rmat_bench_gather: bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* out = static_cast<unsigned long long*>(d_out);
  const uint32_t mask = static_cast<uint32_t>(table_bytes / width - 1);
  const char* base = static_cast<const char*>(d_table);
  const dim3 g(256 * blocks_per_cu), b(512);
  if (width == 16) hipLaunchKernelGGL(rmat::gather_kernel<16>, g, b, 0, s, base, n_reads, mask, out);
  if (width == 8) hipLaunchKernelGGL(rmat::gather_kernel<8>, g, b, 0, s, base, n_reads, mask, out);
  if (width == 4) hipLaunchKernelGGL(rmat::gather_kernel<4>, g, b, 0, s, base, n_reads, mask, out);
  return rmat::check_launch("rmat_bench_gather");
}

}  // extern "C"
