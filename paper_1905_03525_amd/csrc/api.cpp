// api.cpp -- the C ABI of include/rmat.h for single tables: argument
// validation, table ownership, device memory and launches.  Every step of the
// method runs in the HIP kernels of table_build.hip and generate.hip; this
// file only sizes, allocates and launches them.  Batches are in batch.cpp.
#include "rmat.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <map>
#include <vector>
#include <new>

#include "rmat_internal.h"

struct rmat_table {
  rmat_info info;
  int device;
  void* d_mem;  // records, item arrays, bucket arrays, stats
  rmat::TableView v;
  void* d_reduce = nullptr;    // reduction workspace: 16-bit bins, then per-workgroup partial counts
  uint64_t reduce_edges = 0;   // bins it holds
  double q[4];                 // a, b, c, d as given
  std::vector<rmat::TableView> members;  // a perturbed set's tables (empty for one table)
  double p_second = 0.0;       // probability that an edge needs more than four samples
  // an asynchronous build: until finalize_table() has waited for `built`
  // and read the device statistics, info's min/max/expected length and
  // p_second are unknown
  bool pending = false;
  int build_status = RMAT_OK;  // a failed asynchronous build, once known
  hipEvent_t built = nullptr;
};

namespace rmat {
const rmat_info* table_info_of(const rmat_table* t) { return &t->info; }
const TableView* table_view_of(const rmat_table* t) { return &t->v; }
const double* table_params_of(const rmat_table* t) { return t->q; }
}  // namespace rmat

namespace {

thread_local char g_err[512] = "";

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

}  // namespace

namespace rmat {

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return set_error(e == hipErrorOutOfMemory ? RMAT_ENOMEM : RMAT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, what);
  g_err[0] = '\0';
  return RMAT_OK;
}

int validate_and_size(const double q[4], int k, uint64_t bound, int mode, Shape* s) {
  double sum = 0.0;
  for (int i = 0; i < 4; ++i) {
    if (!(q[i] >= 0.0) || !std::isfinite(q[i])) return set_error(RMAT_EINVAL, "quadrant probability %d is %g", i, q[i]);
    sum += q[i];
  }
  if (std::fabs(sum - 1.0) > 1e-9) return set_error(RMAT_EINVAL, "a+b+c+d = %.17g, not 1", sum);
  if (k < 1 || k > 64) return set_error(RMAT_EINVAL, "k = %d outside 1..64", k);
  if (bound > kMaxBound) return set_error(RMAT_EINVAL, "table_bound %llu above 2^24", (unsigned long long)bound);
  s->cap = k < kMaxDepthCap ? k : kMaxDepthCap;
  s->fixed_len = 0;
  if (mode == RMAT_VARIABLE) {
    if (bound < 5) return set_error(RMAT_EINVAL, "variable table_bound %llu below 5", (unsigned long long)bound);
    const uint64_t t = (bound - 4 + 2) / 3;  // ceil((bound - 4) / 3)
    const uint64_t expandable = ((1ull << (2 * s->cap)) - 1) / 3;
    s->n_expand = t < expandable ? t : expandable;
    s->n_items = 1 + 3 * s->n_expand;
  } else if (mode == RMAT_FIXED) {
    int ell = 0;
    while ((1ull << (2 * (ell + 1))) <= bound) ++ell;
    if (ell < 1) return set_error(RMAT_EINVAL, "fixed table_bound %llu below 4", (unsigned long long)bound);
    if (ell > s->cap) return set_error(RMAT_EINVAL, "fixed path length %d exceeds min(15, k) = %d", ell, s->cap);
    s->fixed_len = ell;
    s->n_items = 1ull << (2 * ell);
    s->n_expand = (s->n_items - 1) / 3;
  } else {
    return set_error(RMAT_EINVAL, "path_mode %d is neither RMAT_FIXED nor RMAT_VARIABLE", mode);
  }
  int b = 0;
  while ((1ull << b) < s->n_items) ++b;
  s->bucket_bits = b;
  s->n_buckets = 1ull << b;
  s->capacity = 1ull << (32 - b);
  return RMAT_OK;
}

uint64_t table_bytes(const Shape& S) {
  const uint64_t nb = S.n_buckets;
  uint64_t off = align_up(nb * sizeof(BucketRecord), 256);
  off += align_up(nb * 8, 256) * 2;  // p, w
  off += align_up(nb * 4, 256) * 5;  // len, row, col, thr, alias
  off += align_up(sizeof(BuildStats), 256);
  return off;
}

uint64_t scratch_bytes(const Shape& S) {
  const uint64_t ne = S.n_expand, nb = S.n_buckets;
  return align_up(ne * 4, 256) * 4 + align_up(ne, 256) + align_up(nb * 4, 256) * 2 + align_up(nb * 8, 256) * 2;
}

TableView place_table(char* base, const Shape& S) {
  const uint64_t nb = S.n_buckets;
  TableView v;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    char* p = base + off;
    off += align_up(bytes, 256);
    return p;
  };
  v.records = reinterpret_cast<BucketRecord*>(take(nb * sizeof(BucketRecord)));
  v.p = reinterpret_cast<double*>(take(nb * 8));
  v.w = reinterpret_cast<uint64_t*>(take(nb * 8));
  v.len = reinterpret_cast<uint32_t*>(take(nb * 4));
  v.row = reinterpret_cast<uint32_t*>(take(nb * 4));
  v.col = reinterpret_cast<uint32_t*>(take(nb * 4));
  v.thr = reinterpret_cast<uint32_t*>(take(nb * 4));
  v.alias = reinterpret_cast<uint32_t*>(take(nb * 4));
  v.stats = reinterpret_cast<BuildStats*>(take(sizeof(BuildStats)));
  return v;
}

void fill_job(BuildJob* job, const double q[4], int k, int mode, const Shape& S, const TableView& V, char* scratch) {
  std::memset(job, 0, sizeof(*job));
  std::memcpy(job->q, q, 4 * sizeof(double));
  job->k = k;
  job->mode = mode;
  job->cap = S.cap;
  job->bucket_bits = S.bucket_bits;
  job->fixed_len = S.fixed_len;
  job->n_items = static_cast<uint32_t>(S.n_items);
  job->n_expand = S.n_expand;
  job->n_buckets = S.n_buckets;
  job->capacity = S.capacity;
  job->records = V.records;
  job->item_p = V.p;
  job->item_w = V.w;
  job->item_len = V.len;
  job->item_row = V.row;
  job->item_col = V.col;
  job->thr = V.thr;
  job->alias = V.alias;
  job->stats = V.stats;
  job->reset_counter = nullptr;
  const uint64_t ne = S.n_expand, nb = S.n_buckets;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    char* p = scratch + off;
    off += align_up(bytes, 256);
    return p;
  };
  job->lvl_code = reinterpret_cast<uint32_t*>(take(ne * 4));
  job->lvl_first = reinterpret_cast<uint32_t*>(take(ne * 4));
  job->lvl_size = reinterpret_cast<uint32_t*>(take(ne * 4));
  job->lvl_off = reinterpret_cast<uint32_t*>(take(ne * 4));
  job->lvl_mask = reinterpret_cast<uint8_t*>(take(ne));
  job->light_idx = reinterpret_cast<uint32_t*>(take(nb * 4));
  job->heavy_idx = reinterpret_cast<uint32_t*>(take(nb * 4));
  job->light_cum = reinterpret_cast<uint64_t*>(take(nb * 8));
  job->heavy_cum = reinterpret_cast<uint64_t*>(take(nb * 8));
}

int export_table(const TableView& V, uint64_t nb, void* host_buf, size_t nbytes) {
  if (!host_buf) return set_error(RMAT_EINVAL, "NULL buffer");
  if (nbytes < 36 * nb)
    return set_error(RMAT_EINVAL, "export needs %llu bytes, got %zu", (unsigned long long)(36 * nb), nbytes);
  char* h = static_cast<char*>(host_buf);
  struct Part {
    const void* src;
    uint64_t bytes;
  } parts[] = {{V.w, nb * 8},   {V.p, nb * 8},   {V.len, nb * 4},  {V.row, nb * 4},
               {V.col, nb * 4}, {V.thr, nb * 4}, {V.alias, nb * 4}};
  for (const Part& p : parts) {
    hipError_t e = hipMemcpy(h, p.src, p.bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(export)");
    h += p.bytes;
  }
  return RMAT_OK;
}

void fill_info(rmat_info* I, int k, int path_mode, uint64_t table_bound, const Shape& S, const BuildStats& stats,
               uint64_t device_bytes) {
  I->k = k;
  I->path_mode = path_mode;
  I->depth_cap = S.cap;
  I->bucket_bits = S.bucket_bits;
  I->table_bound = table_bound;
  I->n_items = S.n_items;
  I->n_buckets = S.n_buckets;
  I->capacity = S.capacity;
  I->id_bytes = k <= 32 ? 4 : 8;
  I->min_len = stats.min_len;
  I->max_len = stats.max_len;
  I->lds_resident = S.n_buckets <= lds_table_limit() ? 1 : 0;
  I->expected_len = static_cast<double>(stats.sum_wl) / 4294967296.0;
  I->export_bytes = 36 * S.n_buckets;
  I->device_bytes = device_bytes;
  I->initiator_k = 2;
  I->n_tables = 1;
}

double p_second_block(const BuildStats& st, int k) {
  // distribution of the total length of four samples (each path 1..15 letters)
  double pl[16], d[61] = {1.0};
  for (int L = 0; L < 16; ++L) pl[L] = static_cast<double>(st.len_mass[L]) / 4294967296.0;
  for (int s = 0; s < 4; ++s) {
    double nd[61] = {0.0};
    for (int v = 0; v <= 15 * s; ++v)
      for (int L = 1; L < 16; ++L) nd[v + L] += d[v] * pl[L];
    std::memcpy(d, nd, sizeof(d));
  }
  double p = 0.0;
  for (int v = 0; v < k && v <= 60; ++v) p += d[v];
  return p;
}

int adopt_table(const rmat_info& info, const double q[4], int kron_K, const TableView& view, void* d_mem,
                double p_second, rmat_table_t* out) {
  rmat_table* t = new (std::nothrow) rmat_table();
  if (!t) return set_error(RMAT_ENOMEM, "host allocation of the table handle failed");
  if (hipGetDevice(&t->device) != hipSuccess) t->device = 0;
  t->info = info;
  t->info.initiator_k = static_cast<uint32_t>(kron_K);
  t->v = view;
  t->d_mem = d_mem;
  t->p_second = p_second;
  std::memcpy(t->q, q, sizeof(t->q));
  if (kron_K > 2) {
    t->info.id_bytes = 4;  // K^k <= 2^32 ?
    uint64_t n = 1;
    for (int i = 0; i < info.k; ++i) {
      if (n > (~0ull) / static_cast<uint64_t>(kron_K)) {
        t->info.id_bytes = 8;
        break;
      }
      n *= static_cast<uint64_t>(kron_K);
      if (n > (1ull << 32)) t->info.id_bytes = 8;
    }
  }
  *out = t;
  return RMAT_OK;
}

// The statistics of an asynchronous build, once: waits for its event, takes
// min/max/expected length and p_second, and records a failed build (whose
// records are the terminating sentinels) as the table's status.
int finalize_table(rmat_table* t) {
  if (!t->pending) return t->build_status;
  hipError_t e = hipEventSynchronize(t->built);
  BuildStats st;
  if (e == hipSuccess) e = hipMemcpy(&st, t->v.stats, sizeof(st), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "table build");
  t->pending = false;
  if (st.error != 0) {
    t->build_status = st.error == kBuildResidual ? RMAT_EINVAL : RMAT_EDEVICE;
    return set_error(t->build_status, "table build failed on the device (code %d)", st.error);
  }
  t->info.min_len = st.min_len;
  t->info.max_len = st.max_len;
  t->info.expected_len = static_cast<double>(st.sum_wl) / 4294967296.0;
  t->p_second = p_second_block(st, static_cast<int>(t->info.k));
  return RMAT_OK;
}

// Orders work on `stream` after a table's build: a finished asynchronous
// build is finalized (no wait); one still running makes the stream wait for
// its event.  Returns the table's status (a failed build is an error).
int order_after_build(rmat_table* t, hipStream_t stream) {
  if (t->pending) {
    const hipError_t q = hipEventQuery(t->built);
    if (q == hipSuccess) return finalize_table(t);
    if (q != hipErrorNotReady) return hip_fail(q, "table build");
    const hipError_t e = hipStreamWaitEvent(stream, t->built, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent(table build)");
    return RMAT_OK;
  }
  return t->build_status;
}

// SplitMix64 [Steele, Lea, Flood, OOPSLA'14]: state advanced by the golden
// gamma, output mixed by two multiply-xorshift steps.
uint64_t splitmix64(uint64_t& state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void scramble_params(uint64_t key, int k, GenInst* I) {
  uint64_t st = key;
  for (int r = 0; r < 3; ++r) {
    I->scr_mul[r] = splitmix64(st) | 1ull;
    I->scr_add[r] = splitmix64(st);
  }
  I->scr_mask = k >= 64 ? ~0ull : ((1ull << k) - 1);
  I->scr_shift = static_cast<uint32_t>((k + 1) / 2);
}

void clear_error() { g_err[0] = '\0'; }

int check_device() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_error(RMAT_EDEVICE, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
  e = prepare_kernels();
  if (e != hipSuccess) return hip_fail(e, "kernel attributes");
  return RMAT_OK;
}

}  // namespace rmat

using rmat::set_error;

extern "C" {

const char* rmat_last_error(void) { return g_err; }

namespace {
std::mutex g_scratch_mu;
std::map<int, std::pair<void*, uint64_t>> g_scratch;  // device -> (buffer, bytes); held until exit

// A build scratch buffer of at least `bytes` on `device` (call with
// g_scratch_mu held); grows by reallocation, never shrinks.
hipError_t build_scratch(int device, uint64_t bytes, void** out) {
  auto& slot = g_scratch[device];
  if (slot.second < bytes) {
    if (slot.first) (void)hipFree(slot.first);
    slot = {nullptr, 0};
    hipError_t e = hipMalloc(&slot.first, bytes);
    if (e != hipSuccess) {
      slot.first = nullptr;
      return e;
    }
    slot.second = bytes;
  }
  *out = slot.first;
  return hipSuccess;
}
}  // namespace

// A synchronous build waits for the device and reads the statistics at
// once, using the per-device scratch buffer; an asynchronous one launches on
// `stream` with working arrays of its own in the table's allocation (builds
// on different streams may overlap), records an event and returns.
static int build_table_common(double a, double b, double c, double d, int k, uint64_t table_bound, int path_mode,
                              bool async, hipStream_t stream, rmat_table_t* out) {
  g_err[0] = '\0';
  if (!out) return set_error(RMAT_EINVAL, "out is NULL");
  *out = nullptr;
  const double q[4] = {a, b, c, d};
  rmat::Shape S;
  int rc = rmat::validate_and_size(q, k, table_bound, path_mode, &S);
  if (rc) return rc;
  if ((rc = rmat::check_device())) return rc;

  rmat_table* t = new (std::nothrow) rmat_table();
  if (!t) return set_error(RMAT_ENOMEM, "host allocation of the table handle failed");
  if (hipGetDevice(&t->device) != hipSuccess) t->device = 0;
  auto release = [t]() {
    if (t->built) (void)hipEventDestroy(t->built);
    if (t->d_mem) (void)hipFree(t->d_mem);
    delete t;
  };
  const uint64_t tb = rmat::table_bytes(S);
  // an asynchronous build keeps its working arrays behind the table
  const uint64_t scratch_off = align_up(tb, 256);
  hipError_t e = hipMalloc(&t->d_mem, async ? scratch_off + rmat::scratch_bytes(S) : tb);
  if (e != hipSuccess) {
    t->d_mem = nullptr;
    release();
    return rmat::hip_fail(e, "hipMalloc(table)");
  }
  t->v = rmat::place_table(static_cast<char*>(t->d_mem), S);
  std::memcpy(t->q, q, sizeof(t->q));
  if (async) {
    e = hipEventCreateWithFlags(&t->built, hipEventDisableTiming);
    if (e != hipSuccess) {
      t->built = nullptr;
      release();
      return rmat::hip_fail(e, "hipEventCreate(table build)");
    }
    rmat::BuildJob job;
    rmat::fill_job(&job, q, k, path_mode, S, t->v, static_cast<char*>(t->d_mem) + scratch_off);
    e = rmat::launch_table_build_one(job, stream);
    if (e == hipSuccess) e = hipEventRecord(t->built, stream);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(stream);  // nothing of this build may still run when its memory goes
      release();
      return rmat::hip_fail(e, "table build launch");
    }
    // shape-derived fields now; the statistics when the build is finalized
    const rmat::BuildStats none{};
    rmat::fill_info(&t->info, k, path_mode, table_bound, S, none, scratch_off + rmat::scratch_bytes(S));
    t->pending = true;
    *out = t;
    return RMAT_OK;
  }
  rmat::BuildStats stats;
  {
    // the build's working arrays come from a per-device buffer kept between
    // synchronous builds (serialised here)
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    void* scratch = nullptr;
    e = build_scratch(t->device, rmat::scratch_bytes(S), &scratch);
    if (e != hipSuccess) {
      release();
      return rmat::hip_fail(e, "hipMalloc(build scratch)");
    }
    rmat::BuildJob job;
    rmat::fill_job(&job, q, k, path_mode, S, t->v, static_cast<char*>(scratch));
    e = rmat::launch_table_build_one(job, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e == hipSuccess) e = hipMemcpy(&stats, t->v.stats, sizeof(stats), hipMemcpyDeviceToHost);
  }
  if (e != hipSuccess) {
    release();
    return rmat::hip_fail(e, "table build");
  }
  if (stats.error != 0) {
    release();
    return set_error(stats.error == rmat::kBuildResidual ? RMAT_EINVAL : RMAT_EDEVICE,
                     "table build failed on the device (code %d)", stats.error);
  }

  rmat::fill_info(&t->info, k, path_mode, table_bound, S, stats, tb);
  t->p_second = rmat::p_second_block(stats, k);
  *out = t;
  return RMAT_OK;
}

int rmat_build_table(double a, double b, double c, double d, int k, uint64_t table_bound, int path_mode,
                     rmat_table_t* out) {
  RMAT_GUARD("rmat_build_table",
             build_table_common(a, b, c, d, k, table_bound, path_mode, false, nullptr, out));
}

int rmat_build_table_async(double a, double b, double c, double d, int k, uint64_t table_bound, int path_mode,
                           void* stream, rmat_table_t* out) {
  RMAT_GUARD("rmat_build_table_async", build_table_common(a, b, c, d, k, table_bound, path_mode, true,
                                                          static_cast<hipStream_t>(stream), out));
}

static int rmat_build_perturbed_table_body(double a, double b, double c, double d, int k, uint64_t table_bound,
                                           int path_mode, int n_tables, double epsilon, uint64_t perturb_seed,
                                           rmat_table_t* out) {
  g_err[0] = '\0';
  if (!out) return set_error(RMAT_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_tables < 1 || n_tables > 64 || (n_tables & (n_tables - 1)))
    return set_error(RMAT_EINVAL, "n_tables %d is not a power of two in 1..64", n_tables);
  if (!(epsilon >= 0.0 && epsilon < 1.0)) return set_error(RMAT_EINVAL, "epsilon must be in [0, 1)");
  const double q0[4] = {a, b, c, d};
  rmat::Shape S;
  int rc = rmat::validate_and_size(q0, k, table_bound, path_mode, &S);
  if (rc) return rc;
  // parameter sets: each entry scaled by 1 + eps (2u - 1), u from SplitMix64, then normalised
  std::vector<double> qs(4 * static_cast<size_t>(n_tables));
  uint64_t st = perturb_seed;
  for (int i = 0; i < n_tables; ++i) {
    double v[4];
    for (int x = 0; x < 4; ++x) {
      const double u = static_cast<double>(rmat::splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
      v[x] = q0[x] * (1.0 + epsilon * (2.0 * u - 1.0));
    }
    const double sum = v[0] + v[1] + v[2] + v[3];
    for (int x = 0; x < 4; ++x) qs[4 * i + x] = v[x] / sum;
    rmat::Shape Si;
    if ((rc = rmat::validate_and_size(&qs[4 * i], k, table_bound, path_mode, &Si))) return rc;
  }
  // a set's members are addressed by 32-bit byte offsets, and the queue's
  // continuation takes a member's offset with a 24-bit multiply
  if (n_tables > 1 && S.n_buckets * sizeof(rmat::BucketRecord) >= (1ull << 24))
    return set_error(RMAT_EINVAL, "a set of %d tables takes tables of at most 2^19 buckets, not %llu", n_tables,
                     (unsigned long long)S.n_buckets);
  if ((rc = rmat::check_device())) return rc;
  const uint64_t nb = S.n_buckets;
  const uint64_t tb = rmat::table_bytes(S);
  const uint64_t rec_bytes = (static_cast<uint64_t>(n_tables) * nb * sizeof(rmat::BucketRecord) + 255) / 256 * 256;
  void* d_mem = nullptr;
  hipError_t e = hipMalloc(&d_mem, tb * n_tables + rec_bytes);
  if (e != hipSuccess) return rmat::hip_fail(e, "hipMalloc(perturbed tables)");
  char* base = static_cast<char*>(d_mem);
  auto* recs = reinterpret_cast<rmat::BucketRecord*>(base + tb * n_tables);
  std::vector<rmat::TableView> views(n_tables);
  for (int i = 0; i < n_tables; ++i) {
    views[i] = rmat::place_table(base + tb * i, S);
    views[i].records = recs + static_cast<uint64_t>(i) * nb;  // the members' records back to back
  }
  const uint64_t sb = (rmat::scratch_bytes(S) + 255) / 256 * 256;
  void* scratch = nullptr;
  e = hipMalloc(&scratch, sb * n_tables + sizeof(rmat::BuildJob) * n_tables + 256);
  if (e != hipSuccess) {
    (void)hipFree(d_mem);
    return rmat::hip_fail(e, "hipMalloc(build scratch)");
  }
  std::vector<rmat::BuildJob> jobs(n_tables);
  rmat::BuildStats init;
  std::memset(&init, 0, sizeof(init));
  init.error = -1;
  for (int i = 0; i < n_tables && e == hipSuccess; ++i) {
    rmat::fill_job(&jobs[i], &qs[4 * i], k, path_mode, S, views[i], static_cast<char*>(scratch) + sb * i);
    e = hipMemcpy(views[i].stats, &init, sizeof(init), hipMemcpyHostToDevice);
  }
  auto* d_jobs = reinterpret_cast<rmat::BuildJob*>(static_cast<char*>(scratch) + sb * n_tables);
  if (e == hipSuccess) e = hipMemcpy(d_jobs, jobs.data(), sizeof(rmat::BuildJob) * n_tables, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = rmat::launch_table_build(d_jobs, n_tables, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  std::vector<rmat::BuildStats> stats(n_tables);
  for (int i = 0; i < n_tables && e == hipSuccess; ++i)
    e = hipMemcpy(&stats[i], views[i].stats, sizeof(rmat::BuildStats), hipMemcpyDeviceToHost);
  (void)hipFree(scratch);
  if (e != hipSuccess) {
    (void)hipFree(d_mem);
    return rmat::hip_fail(e, "perturbed table build");
  }
  for (int i = 0; i < n_tables; ++i)
    if (stats[i].error != 0) {
      (void)hipFree(d_mem);
      return set_error(stats[i].error == rmat::kBuildResidual ? RMAT_EINVAL : RMAT_EDEVICE,
                       "table %d: build failed on the device (code %d)", i, stats[i].error);
    }
  rmat_info info;
  rmat::fill_info(&info, k, path_mode, table_bound, S, stats[0], tb * n_tables + rec_bytes);
  info.n_tables = static_cast<uint32_t>(n_tables);
  info.lds_resident = nb * n_tables <= rmat::lds_table_limit() ? 1 : 0;
  rmat_table* t = new (std::nothrow) rmat_table();
  if (!t) {
    (void)hipFree(d_mem);
    return set_error(RMAT_ENOMEM, "host allocation of the table handle failed");
  }
  if (hipGetDevice(&t->device) != hipSuccess) t->device = 0;
  t->info = info;
  t->d_mem = d_mem;
  t->v = views[0];
  t->members = views;
  for (int i = 0; i < n_tables; ++i) t->p_second += rmat::p_second_block(stats[i], k) / n_tables;  // edge e: member e mod P
  std::memcpy(t->q, q0, sizeof(t->q));
  *out = t;
  return RMAT_OK;
}

int rmat_build_perturbed_table(double a, double b, double c, double d, int k, uint64_t table_bound, int path_mode,
                               int n_tables, double epsilon, uint64_t perturb_seed, rmat_table_t* out) {
  RMAT_GUARD("rmat_build_perturbed_table", rmat_build_perturbed_table_body(a, b, c, d, k, table_bound, path_mode,
                                                                           n_tables, epsilon, perturb_seed, out));
}

int rmat_table_export_member(rmat_table_t t, int i, void* host_buf, size_t nbytes) {
  g_err[0] = '\0';
  if (!t) return set_error(RMAT_EINVAL, "NULL table");
  if (int rc = rmat::finalize_table(t)) return rc;
  if (i < 0 || static_cast<uint32_t>(i) >= t->info.n_tables)
    return set_error(RMAT_EINVAL, "member %d outside 0..%u", i, t->info.n_tables - 1);
  const rmat::TableView& V = t->members.empty() ? t->v : t->members[static_cast<size_t>(i)];
  return rmat::export_table(V, t->info.n_buckets, host_buf, nbytes);
}

int rmat_free_table(rmat_table_t t) {
  g_err[0] = '\0';
  if (!t) return RMAT_OK;
  // an asynchronous build still running must end before its memory goes
  if (t->built) (void)hipEventSynchronize(t->built);
  if (t->d_reduce) (void)hipFree(t->d_reduce);
  if (t->built) (void)hipEventDestroy(t->built);
  hipError_t e = hipFree(t->d_mem);
  delete t;
  if (e != hipSuccess) return rmat::hip_fail(e, "hipFree(table)");
  return RMAT_OK;
}

int rmat_table_info(rmat_table_t t, rmat_info* out) {
  g_err[0] = '\0';
  if (!t || !out) return set_error(RMAT_EINVAL, "NULL table or info pointer");
  const int rc = rmat::finalize_table(t);
  if (rc) return rc;
  *out = t->info;
  return RMAT_OK;
}

int rmat_table_export(rmat_table_t t, void* host_buf, size_t nbytes) {
  g_err[0] = '\0';
  if (!t) return set_error(RMAT_EINVAL, "NULL table");
  const int rc = rmat::finalize_table(t);
  if (rc) return rc;
  return rmat::export_table(t->v, t->info.n_buckets, host_buf, nbytes);
}

static int generate_common(rmat_table_t t, uint64_t seed, uint64_t edge_begin, uint64_t m, void* out_src,
                           void* out_dst, void* stream, bool reduce, int hist_bits, void* d_hist, void* d_xor,
                           int flags = 0, uint64_t scramble_key = 0, bool static_workspace = false) {
  if (!t) return set_error(RMAT_EINVAL, "NULL table");
  if (int rc = rmat::order_after_build(t, static_cast<hipStream_t>(stream))) return rc;
  if (t->info.initiator_k > 2 && (reduce || flags))
    return set_error(RMAT_EINVAL, "a K x K Kronecker table supports plain generation only");
  if (flags & ~(RMAT_UNDIRECTED | RMAT_SCRAMBLE)) return set_error(RMAT_EINVAL, "unknown flags 0x%x", flags);
  if (m == 0) return RMAT_OK;
  if (edge_begin + (m - 1) < edge_begin) return set_error(RMAT_ERANGE, "edge_begin + m exceeds 2^64");
  rmat::GenerateArgs a;
  std::memset(&a, 0, sizeof(a));
  if (reduce) {
    const int hmax = t->info.k < 16 ? t->info.k : 16;
    if (hist_bits < 0 || hist_bits > hmax)
      return set_error(RMAT_EINVAL, "hist_bits %d outside 0..%d", hist_bits, hmax);
    if (!d_hist || !d_xor) return set_error(RMAT_EINVAL, "NULL histogram or checksum pointer");
    a.hist_bits = hist_bits;
    a.hist = static_cast<unsigned long long*>(d_hist);
    a.xor_out = static_cast<unsigned long long*>(d_xor);
  }
  if (reduce && static_workspace) {
    hipError_t e = rmat::static_reduce_workspace(&a);
    if (e != hipSuccess) return rmat::hip_fail(e, "hipGetSymbolAddress(reduction workspace)");
  } else if (reduce) {
    // workspace: bins for one sub-chunk, grown on demand (a larger one replaces it)
    const uint64_t want = std::min<uint64_t>(rmat::kReduceChunk, (m + (1u << 20) - 1) & ~static_cast<uint64_t>((1u << 20) - 1));
    if (t->reduce_edges < want) {
      if (t->d_reduce) {
        (void)hipFree(t->d_reduce);
        t->d_reduce = nullptr;
        t->reduce_edges = 0;
      }
      hipError_t e = hipMalloc(&t->d_reduce, want * sizeof(uint16_t) + rmat::reduce_partials_bytes());
      if (e != hipSuccess) return rmat::hip_fail(e, "hipMalloc(reduction workspace)");
      t->reduce_edges = want;
    }
    a.bins = static_cast<uint16_t*>(t->d_reduce);
    a.bins_cap = t->reduce_edges;
    a.partials = reinterpret_cast<uint32_t*>(static_cast<char*>(t->d_reduce) + t->reduce_edges * sizeof(uint16_t));
  } else {
    if (!out_src || !out_dst) return set_error(RMAT_EINVAL, "NULL output pointer");
    const uintptr_t align = t->info.id_bytes;
    if ((reinterpret_cast<uintptr_t>(out_src) | reinterpret_cast<uintptr_t>(out_dst)) % align)
      return set_error(RMAT_EINVAL, "output pointers must be %u-byte aligned", (unsigned)align);
    a.out_src = out_src;
    a.out_dst = out_dst;
  }
  a.records = t->v.records;
  a.n_buckets = static_cast<uint32_t>(t->info.n_buckets);
  a.bucket_bits = t->info.bucket_bits;
  a.k = t->info.k;
  a.lds = t->info.lds_resident;
  a.seed = seed;
  a.edge_begin = edge_begin;
  a.m = m;
  a.epi = static_cast<uint32_t>(flags);
  a.scramble_key = scramble_key;
  a.kron_k = t->info.initiator_k;
  a.id_bytes = t->info.id_bytes;
  a.n_tables = t->info.n_tables;
  a.first_blocks = rmat::first_blocks_for(t->p_second);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = reduce ? rmat::launch_generate_reduce(a, s) : rmat::launch_generate(a, s);
  if (e != hipSuccess) return rmat::hip_fail(e, reduce ? "generate_reduce launch" : "generate launch");
  return RMAT_OK;
}

int rmat_generate_async(rmat_table_t t, uint64_t seed, uint64_t edge_begin, uint64_t m, void* out_src,
                        void* out_dst, void* stream) {
  g_err[0] = '\0';
  return generate_common(t, seed, edge_begin, m, out_src, out_dst, stream, false, 0, nullptr, nullptr);
}

int rmat_generate_ex_async(rmat_table_t t, uint64_t seed, uint64_t edge_begin, uint64_t m, int flags,
                           uint64_t scramble_key, void* out_src, void* out_dst, void* stream) {
  g_err[0] = '\0';
  return generate_common(t, seed, edge_begin, m, out_src, out_dst, stream, false, 0, nullptr, nullptr, flags,
                         scramble_key);
}

int rmat_generate(rmat_table_t t, uint64_t seed, uint64_t edge_begin, uint64_t m, void* out_src, void* out_dst) {
  g_err[0] = '\0';
  int rc = generate_common(t, seed, edge_begin, m, out_src, out_dst, nullptr, false, 0, nullptr, nullptr);
  if (rc) return rc;
  hipError_t e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return rmat::hip_fail(e, "generate");
  return RMAT_OK;
}

int rmat_generate_reduce_async(rmat_table_t t, uint64_t seed, uint64_t edge_begin, uint64_t m, int hist_bits,
                               void* d_hist, void* d_xor, void* stream) {
  g_err[0] = '\0';
  return generate_common(t, seed, edge_begin, m, nullptr, nullptr, stream, true, hist_bits, d_hist, d_xor);
}

int rmat_generate_reduce_noalloc_async(rmat_table_t t, uint64_t seed, uint64_t edge_begin, uint64_t m, int hist_bits,
                                       void* d_hist, void* d_xor, void* stream) {
  g_err[0] = '\0';
  return generate_common(t, seed, edge_begin, m, nullptr, nullptr, stream, true, hist_bits, d_hist, d_xor, 0, 0,
                         true);
}

int rmat_generate_degrees_async(rmat_table_t t, uint64_t seed, uint64_t edge_begin, uint64_t m, void* d_degree,
                                void* stream) {
  g_err[0] = '\0';
  if (!t) return set_error(RMAT_EINVAL, "NULL table");
  if (int rc = rmat::order_after_build(t, static_cast<hipStream_t>(stream))) return rc;
  if (t->info.initiator_k > 2) return set_error(RMAT_EINVAL, "out-degrees are for R-MAT tables (K = 2)");
  if (m == 0) return RMAT_OK;
  if (edge_begin + (m - 1) < edge_begin) return set_error(RMAT_ERANGE, "edge_begin + m exceeds 2^64");
  if (!d_degree || reinterpret_cast<uintptr_t>(d_degree) % 4)
    return set_error(RMAT_EINVAL, "d_degree must be a non-NULL, 4-byte aligned device pointer");
  rmat::GenerateArgs a;
  std::memset(&a, 0, sizeof(a));
  a.records = t->v.records;
  a.n_buckets = static_cast<uint32_t>(t->info.n_buckets);
  a.bucket_bits = t->info.bucket_bits;
  a.k = t->info.k;
  a.lds = t->info.lds_resident;
  a.seed = seed;
  a.edge_begin = edge_begin;
  a.m = m;
  a.kron_k = 2;
  a.id_bytes = t->info.id_bytes;
  a.n_tables = t->info.n_tables;
  a.first_blocks = 1;  // the counting kernel draws one counter block in its first pass
  a.degree = static_cast<uint32_t*>(d_degree);
  hipError_t e = rmat::launch_generate_degrees(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return rmat::hip_fail(e, "generate_degrees launch");
  return RMAT_OK;
}

int rmat_degree_distribution_async(const void* d_degree, uint64_t n_nodes, uint32_t max_degree, void* d_hist,
                                   void* stream) {
  g_err[0] = '\0';
  if (n_nodes > (1ull << 40)) return set_error(RMAT_EINVAL, "n_nodes above 2^40");
  if (max_degree >= (1u << 31)) return set_error(RMAT_EINVAL, "max_degree must be below 2^31");
  if (!d_hist || reinterpret_cast<uintptr_t>(d_hist) % 8)
    return set_error(RMAT_EINVAL, "d_hist must be a non-NULL, 8-byte aligned device pointer");
  if (n_nodes == 0) return RMAT_OK;
  if (!d_degree || reinterpret_cast<uintptr_t>(d_degree) % 16)
    return set_error(RMAT_EINVAL, "d_degree must be a non-NULL, 16-byte aligned device pointer");
  int rc = rmat::check_device();
  if (rc) return rc;
  hipError_t e = rmat::launch_degree_distribution(static_cast<const uint32_t*>(d_degree), n_nodes, max_degree,
                                                  static_cast<unsigned long long*>(d_hist),
                                                  static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return rmat::hip_fail(e, "degree_distribution launch");
  return RMAT_OK;
}

}  // extern "C"
