// api.cpp -- the C ABI of include/rmat.h: argument validation, table
// ownership, device memory and launches.  Every step of the method runs in
// the HIP kernels of table_build.hip and generate.hip; this file only sizes,
// allocates and launches them.
#include "rmat.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "rmat_internal.h"

struct rmat_table {
  rmat_info info;
  double q[4];
  int device;
  void* d_mem;  // one allocation: records, item arrays, bucket arrays, stats
  rmat::BucketRecord* records;
  double* item_p;
  uint64_t* item_w;
  uint32_t *item_len, *item_row, *item_col;
  uint32_t *thr, *alias;
};

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? RMAT_ENOMEM : RMAT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Shape of a table (step A1): sizes derived from the arguments alone.
struct Shape {
  int cap, fixed_len, bucket_bits;
  uint64_t n_expand, n_items, n_buckets, capacity;
};

int validate_and_size(const double q[4], int k, uint64_t bound, int mode, Shape* s) {
  double sum = 0.0;
  for (int i = 0; i < 4; ++i) {
    if (!(q[i] >= 0.0) || !std::isfinite(q[i])) return fail(RMAT_EINVAL, "quadrant probability %d is %g", i, q[i]);
    sum += q[i];
  }
  if (std::fabs(sum - 1.0) > 1e-9) return fail(RMAT_EINVAL, "a+b+c+d = %.17g, not 1", sum);
  if (k < 1 || k > 64) return fail(RMAT_EINVAL, "k = %d outside 1..64", k);
  if (bound > rmat::kMaxBound) return fail(RMAT_EINVAL, "table_bound %llu above 2^24", (unsigned long long)bound);
  s->cap = k < rmat::kMaxDepthCap ? k : rmat::kMaxDepthCap;
  s->fixed_len = 0;
  if (mode == RMAT_VARIABLE) {
    if (bound < 5) return fail(RMAT_EINVAL, "variable table_bound %llu below 5", (unsigned long long)bound);
    const uint64_t t = (bound - 4 + 2) / 3;  // ceil((bound - 4) / 3)
    const uint64_t expandable = ((1ull << (2 * s->cap)) - 1) / 3;
    s->n_expand = t < expandable ? t : expandable;
    s->n_items = 1 + 3 * s->n_expand;
  } else if (mode == RMAT_FIXED) {
    int ell = 0;
    while ((1ull << (2 * (ell + 1))) <= bound) ++ell;
    if (ell < 1) return fail(RMAT_EINVAL, "fixed table_bound %llu below 4", (unsigned long long)bound);
    if (ell > s->cap) return fail(RMAT_EINVAL, "fixed path length %d exceeds min(15, k) = %d", ell, s->cap);
    s->fixed_len = ell;
    s->n_items = 1ull << (2 * ell);
    s->n_expand = (s->n_items - 1) / 3;
  } else {
    return fail(RMAT_EINVAL, "path_mode %d is neither RMAT_FIXED nor RMAT_VARIABLE", mode);
  }
  int b = 0;
  while ((1ull << b) < s->n_items) ++b;
  s->bucket_bits = b;
  s->n_buckets = 1ull << b;
  s->capacity = 1ull << (32 - b);
  return RMAT_OK;
}

int check_device() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(RMAT_EDEVICE, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
  return RMAT_OK;
}

}  // namespace

namespace rmat {

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, what);
  g_err[0] = '\0';
  return RMAT_OK;
}

}  // namespace rmat

extern "C" {

const char* rmat_last_error(void) { return g_err; }

int rmat_build_table(double a, double b, double c, double d, int k, uint64_t table_bound, int path_mode,
                     rmat_table_t* out) {
  g_err[0] = '\0';
  if (!out) return fail(RMAT_EINVAL, "out is NULL");
  *out = nullptr;
  const double q[4] = {a, b, c, d};
  Shape S;
  int rc = validate_and_size(q, k, table_bound, path_mode, &S);
  if (rc) return rc;
  if ((rc = check_device())) return rc;

  const uint64_t nb = S.n_buckets;
  // table layout in one allocation
  uint64_t off = 0;
  const uint64_t o_rec = off;   off = align_up(off + nb * sizeof(rmat::BucketRecord), 256);
  const uint64_t o_p = off;     off = align_up(off + nb * 8, 256);
  const uint64_t o_w = off;     off = align_up(off + nb * 8, 256);
  const uint64_t o_len = off;   off = align_up(off + nb * 4, 256);
  const uint64_t o_row = off;   off = align_up(off + nb * 4, 256);
  const uint64_t o_col = off;   off = align_up(off + nb * 4, 256);
  const uint64_t o_thr = off;   off = align_up(off + nb * 4, 256);
  const uint64_t o_alias = off; off = align_up(off + nb * 4, 256);
  const uint64_t o_stats = off; off = align_up(off + sizeof(rmat::BuildStats), 256);
  const uint64_t table_bytes = off;
  // scratch
  const uint64_t ne = S.n_expand;
  uint64_t so = 0;
  const uint64_t s_code = so;  so = align_up(so + ne * 4, 256);
  const uint64_t s_first = so; so = align_up(so + ne * 4, 256);
  const uint64_t s_size = so;  so = align_up(so + ne * 4, 256);
  const uint64_t s_off = so;   so = align_up(so + ne * 4, 256);
  const uint64_t s_mask = so;  so = align_up(so + ne, 256);
  const uint64_t s_lidx = so;  so = align_up(so + nb * 4, 256);
  const uint64_t s_hidx = so;  so = align_up(so + nb * 4, 256);
  const uint64_t s_lcum = so;  so = align_up(so + nb * 8, 256);
  const uint64_t s_hcum = so;  so = align_up(so + nb * 8, 256);
  const uint64_t s_job = so;   so = align_up(so + sizeof(rmat::BuildJob), 256);
  const uint64_t scratch_bytes = so;

  rmat_table* t = new (std::nothrow) rmat_table();
  if (!t) return fail(RMAT_ENOMEM, "host allocation of the table handle failed");
  if (hipGetDevice(&t->device) != hipSuccess) t->device = 0;
  hipError_t e = hipMalloc(&t->d_mem, table_bytes);
  if (e != hipSuccess) { delete t; return hip_fail(e, "hipMalloc(table)"); }
  char* base = static_cast<char*>(t->d_mem);
  t->records = reinterpret_cast<rmat::BucketRecord*>(base + o_rec);
  t->item_p = reinterpret_cast<double*>(base + o_p);
  t->item_w = reinterpret_cast<uint64_t*>(base + o_w);
  t->item_len = reinterpret_cast<uint32_t*>(base + o_len);
  t->item_row = reinterpret_cast<uint32_t*>(base + o_row);
  t->item_col = reinterpret_cast<uint32_t*>(base + o_col);
  t->thr = reinterpret_cast<uint32_t*>(base + o_thr);
  t->alias = reinterpret_cast<uint32_t*>(base + o_alias);
  auto* d_stats = reinterpret_cast<rmat::BuildStats*>(base + o_stats);

  void* scratch = nullptr;
  e = hipMalloc(&scratch, scratch_bytes);
  if (e != hipSuccess) { (void)hipFree(t->d_mem); delete t; return hip_fail(e, "hipMalloc(build scratch)"); }
  char* sb = static_cast<char*>(scratch);

  rmat::BuildJob job;
  std::memset(&job, 0, sizeof(job));
  std::memcpy(job.q, q, sizeof(q));
  job.k = k;
  job.mode = path_mode;
  job.cap = S.cap;
  job.bucket_bits = S.bucket_bits;
  job.fixed_len = S.fixed_len;
  job.n_items = static_cast<uint32_t>(S.n_items);
  job.n_expand = S.n_expand;
  job.n_buckets = nb;
  job.capacity = S.capacity;
  job.records = t->records;
  job.item_p = t->item_p;
  job.item_w = t->item_w;
  job.item_len = t->item_len;
  job.item_row = t->item_row;
  job.item_col = t->item_col;
  job.thr = t->thr;
  job.alias = t->alias;
  job.stats = d_stats;
  job.lvl_code = reinterpret_cast<uint32_t*>(sb + s_code);
  job.lvl_first = reinterpret_cast<uint32_t*>(sb + s_first);
  job.lvl_size = reinterpret_cast<uint32_t*>(sb + s_size);
  job.lvl_off = reinterpret_cast<uint32_t*>(sb + s_off);
  job.lvl_mask = reinterpret_cast<uint8_t*>(sb + s_mask);
  job.light_idx = reinterpret_cast<uint32_t*>(sb + s_lidx);
  job.heavy_idx = reinterpret_cast<uint32_t*>(sb + s_hidx);
  job.light_cum = reinterpret_cast<uint64_t*>(sb + s_lcum);
  job.heavy_cum = reinterpret_cast<uint64_t*>(sb + s_hcum);
  auto* d_job = reinterpret_cast<rmat::BuildJob*>(sb + s_job);

  rmat::BuildStats stats;
  std::memset(&stats, 0, sizeof(stats));
  stats.error = -1;
  e = hipMemcpy(d_job, &job, sizeof(job), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_stats, &stats, sizeof(stats), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = rmat::launch_table_build(d_job, 1, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(&stats, d_stats, sizeof(stats), hipMemcpyDeviceToHost);
  (void)hipFree(scratch);
  if (e != hipSuccess) { (void)hipFree(t->d_mem); delete t; return hip_fail(e, "table build"); }
  if (stats.error != 0) {
    (void)hipFree(t->d_mem);
    delete t;
    return fail(stats.error == rmat::kBuildResidual ? RMAT_EINVAL : RMAT_EDEVICE,
                "table build failed on the device (code %d)", stats.error);
  }

  std::memcpy(t->q, q, sizeof(q));
  rmat_info& I = t->info;
  I.k = k;
  I.path_mode = path_mode;
  I.depth_cap = S.cap;
  I.bucket_bits = S.bucket_bits;
  I.table_bound = table_bound;
  I.n_items = S.n_items;
  I.n_buckets = nb;
  I.capacity = S.capacity;
  I.id_bytes = k <= 32 ? 4 : 8;
  I.min_len = stats.min_len;
  I.max_len = stats.max_len;
  I.lds_resident = nb <= rmat::lds_table_limit() ? 1 : 0;
  I.expected_len = static_cast<double>(stats.sum_wl) / 4294967296.0;
  I.export_bytes = 36 * nb;
  I.device_bytes = table_bytes;
  *out = t;
  return RMAT_OK;
}

int rmat_free_table(rmat_table_t t) {
  g_err[0] = '\0';
  if (!t) return RMAT_OK;
  hipError_t e = hipFree(t->d_mem);
  delete t;
  if (e != hipSuccess) return hip_fail(e, "hipFree(table)");
  return RMAT_OK;
}

int rmat_table_info(rmat_table_t t, rmat_info* out) {
  g_err[0] = '\0';
  if (!t || !out) return fail(RMAT_EINVAL, "NULL table or info pointer");
  *out = t->info;
  return RMAT_OK;
}

int rmat_table_export(rmat_table_t t, void* host_buf, size_t nbytes) {
  g_err[0] = '\0';
  if (!t || !host_buf) return fail(RMAT_EINVAL, "NULL table or buffer");
  const uint64_t nb = t->info.n_buckets;
  if (nbytes < 36 * nb) return fail(RMAT_EINVAL, "export needs %llu bytes, got %zu", (unsigned long long)(36 * nb), nbytes);
  char* h = static_cast<char*>(host_buf);
  struct Part { const void* src; uint64_t bytes; } parts[] = {
      {t->item_w, nb * 8}, {t->item_p, nb * 8}, {t->item_len, nb * 4}, {t->item_row, nb * 4},
      {t->item_col, nb * 4}, {t->thr, nb * 4}, {t->alias, nb * 4}};
  for (const Part& p : parts) {
    hipError_t e = hipMemcpy(h, p.src, p.bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(export)");
    h += p.bytes;
  }
  return RMAT_OK;
}

static int generate_common(rmat_table_t t, uint64_t seed, uint64_t edge_begin, uint64_t m, void* out_src,
                           void* out_dst, void* stream, bool reduce, int hist_bits, void* d_hist, void* d_xor) {
  if (!t) return fail(RMAT_EINVAL, "NULL table");
  if (m == 0) return RMAT_OK;
  if (edge_begin + (m - 1) < edge_begin) return fail(RMAT_ERANGE, "edge_begin + m exceeds 2^64");
  rmat::GenerateArgs a;
  std::memset(&a, 0, sizeof(a));
  if (reduce) {
    const int hmax = t->info.k < 20 ? t->info.k : 20;
    if (hist_bits < 0 || hist_bits > hmax) return fail(RMAT_EINVAL, "hist_bits %d outside 0..%d", hist_bits, hmax);
    if (!d_hist || !d_xor) return fail(RMAT_EINVAL, "NULL histogram or checksum pointer");
    a.hist_bits = hist_bits;
    a.hist = static_cast<unsigned long long*>(d_hist);
    a.xor_out = static_cast<unsigned long long*>(d_xor);
  } else {
    if (!out_src || !out_dst) return fail(RMAT_EINVAL, "NULL output pointer");
    const uintptr_t align = t->info.id_bytes;
    if ((reinterpret_cast<uintptr_t>(out_src) | reinterpret_cast<uintptr_t>(out_dst)) % align)
      return fail(RMAT_EINVAL, "output pointers must be %u-byte aligned", (unsigned)align);
    a.out_src = out_src;
    a.out_dst = out_dst;
  }
  a.records = t->records;
  a.n_buckets = static_cast<uint32_t>(t->info.n_buckets);
  a.bucket_bits = t->info.bucket_bits;
  a.k = t->info.k;
  a.lds = t->info.lds_resident;
  a.seed = seed;
  a.edge_begin = edge_begin;
  a.m = m;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = reduce ? rmat::launch_generate_reduce(a, s) : rmat::launch_generate(a, s);
  if (e != hipSuccess) return hip_fail(e, reduce ? "generate_reduce launch" : "generate launch");
  return RMAT_OK;
}

int rmat_generate_async(rmat_table_t t, uint64_t seed, uint64_t edge_begin, uint64_t m, void* out_src,
                        void* out_dst, void* stream) {
  g_err[0] = '\0';
  return generate_common(t, seed, edge_begin, m, out_src, out_dst, stream, false, 0, nullptr, nullptr);
}

int rmat_generate(rmat_table_t t, uint64_t seed, uint64_t edge_begin, uint64_t m, void* out_src, void* out_dst) {
  g_err[0] = '\0';
  int rc = generate_common(t, seed, edge_begin, m, out_src, out_dst, nullptr, false, 0, nullptr, nullptr);
  if (rc) return rc;
  hipError_t e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return hip_fail(e, "generate");
  return RMAT_OK;
}

int rmat_generate_reduce_async(rmat_table_t t, uint64_t seed, uint64_t edge_begin, uint64_t m, int hist_bits,
                               void* d_hist, void* d_xor, void* stream) {
  g_err[0] = '\0';
  return generate_common(t, seed, edge_begin, m, nullptr, nullptr, stream, true, hist_bits, d_hist, d_xor);
}

}  // extern "C"
