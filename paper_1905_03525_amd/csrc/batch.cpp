// batch.cpp -- batches of independent instances (include/rmat.h): one
// table-build launch for all tables, then persistent generation launches
// over a list of work items, capturable in a hipGraph; and the autotuner that
// picks each instance's table size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "rmat.h"
#include "rmat_internal.h"

namespace {

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Instances of one id width and table residency share a generation launch.
struct Group {
  int wide, lds;
  int general;  // some instance has epilogue flags
  uint32_t max_buckets;
  uint32_t n_items;
  rmat::GenWorkItem* items;  // device, this group's items in instance order
  unsigned int* counter;     // device, zeroed by the build launch
};

}  // namespace

struct rmat_batch {
  int n = 0;
  uint32_t work_blocks = 0;
  std::vector<rmat_instance> inst;
  std::vector<rmat::Shape> shape;
  std::vector<rmat::TableView> views;
  std::vector<Group> groups;
  void* d_tables = nullptr;  // all tables
  void* d_aux = nullptr;     // build scratch, build jobs, instances, items, counters
  rmat::BuildJob* d_jobs = nullptr;
  rmat::GenInst* d_insts = nullptr;
  uint64_t device_bytes = 0, total_edges = 0;
  uint32_t n_items = 0, max_buckets = 0, tile = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

using rmat::set_error;

void destroy(rmat_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_tables) (void)hipFree(b->d_tables);
  if (b->d_aux) (void)hipFree(b->d_aux);
  delete b;
}

int validate_instance(const rmat_instance& x, int i, rmat::Shape* S) {
  const double q[4] = {x.a, x.b, x.c, x.d};
  int rc = rmat::validate_and_size(q, x.k, x.table_bound, x.path_mode, S);
  if (rc) {
    char msg[512];
    std::snprintf(msg, sizeof(msg), "instance %d: %s", i, rmat_last_error());
    return set_error(rc, "%s", msg);
  }
  if (x.m > 0 && x.edge_begin + (x.m - 1) < x.edge_begin)
    return set_error(RMAT_ERANGE, "instance %d: edge_begin + m exceeds 2^64", i);
  if (x.flags & ~(RMAT_UNDIRECTED | RMAT_SCRAMBLE)) return set_error(RMAT_EINVAL, "instance %d: unknown flags", i);
  if (x.m > 0) {
    if (!x.out_src || !x.out_dst) return set_error(RMAT_EINVAL, "instance %d: NULL output pointer", i);
    const uintptr_t align = x.k <= 32 ? 4 : 8;
    if ((reinterpret_cast<uintptr_t>(x.out_src) | reinterpret_cast<uintptr_t>(x.out_dst)) % align)
      return set_error(RMAT_EINVAL, "instance %d: output pointers must be %u-byte aligned", i, (unsigned)align);
  }
  return RMAT_OK;
}

// A set of tables laid out in one allocation, their build scratch and jobs
// (plus `extra` bytes for the caller) in another.
struct TableSet {
  void* d_tables = nullptr;
  void* d_aux = nullptr;
  std::vector<rmat::TableView> views;
  std::vector<rmat::BuildJob> jobs;
  rmat::BuildJob* d_jobs = nullptr;
  char* d_extra = nullptr;
  uint64_t bytes = 0, table_bytes = 0;
};

int alloc_tables(const std::vector<rmat::Shape>& shapes, const std::vector<rmat_instance>& params, uint64_t extra,
                 TableSet* T) {
  const size_t n = shapes.size();
  std::vector<uint64_t> toff(n), soff(n);
  uint64_t tb = 0, sb = 0;
  for (size_t i = 0; i < n; ++i) {
    toff[i] = tb;
    tb += align_up(rmat::table_bytes(shapes[i]), 256);
    soff[i] = sb;
    sb += align_up(rmat::scratch_bytes(shapes[i]), 256);
  }
  const uint64_t jobs_off = sb;
  sb += align_up(n * sizeof(rmat::BuildJob), 256);
  const uint64_t extra_off = sb;
  sb += align_up(extra, 256);
  hipError_t e = hipMalloc(&T->d_tables, tb);
  if (e != hipSuccess) return rmat::hip_fail(e, "hipMalloc(batch tables)");
  e = hipMalloc(&T->d_aux, sb);
  if (e != hipSuccess) {
    (void)hipFree(T->d_tables);
    T->d_tables = nullptr;
    return rmat::hip_fail(e, "hipMalloc(batch scratch)");
  }
  T->bytes = tb + sb;
  T->table_bytes = tb;
  char* aux = static_cast<char*>(T->d_aux);
  T->d_jobs = reinterpret_cast<rmat::BuildJob*>(aux + jobs_off);
  T->d_extra = aux + extra_off;
  T->views.resize(n);
  T->jobs.resize(n);
  for (size_t i = 0; i < n; ++i) {
    T->views[i] = rmat::place_table(static_cast<char*>(T->d_tables) + toff[i], shapes[i]);
    const rmat_instance& x = params[i];
    const double q[4] = {x.a, x.b, x.c, x.d};
    rmat::fill_job(&T->jobs[i], q, x.k, x.path_mode, shapes[i], T->views[i], aux + soff[i]);
  }
  return RMAT_OK;
}

void free_tables(TableSet* T) {
  if (T->d_tables) (void)hipFree(T->d_tables);
  if (T->d_aux) (void)hipFree(T->d_aux);
  T->d_tables = T->d_aux = nullptr;
}

int enqueue(rmat_batch* b, hipStream_t s) {
  hipError_t e = rmat::launch_table_build(b->d_jobs, b->n, s);
  if (e != hipSuccess) return rmat::hip_fail(e, "batch table build launch");
  for (const Group& g : b->groups) {
    rmat::BatchArgs a;
    a.insts = b->d_insts;
    a.items = g.items;
    a.n_items = g.n_items;
    a.counter = g.counter;
    a.max_buckets = g.max_buckets;
    a.wide = g.wide;
    a.lds = g.lds;
    a.digest = 0;
    a.general = g.general;
    e = rmat::launch_generate_batch(a, s);
    if (e != hipSuccess) return rmat::hip_fail(e, "batch generation launch");
  }
  return RMAT_OK;
}

// E[ceil(N/4)] and E[N] for N = samples until k letters, given the law of
// one sample's path length (mass[L] / 2^32): a renewal recursion over the
// number of letters known.
void sample_laws(const uint64_t mass[16], int k, double* blocks, double* samples) {
  double pl[16];
  for (int L = 0; L < 16; ++L) pl[L] = static_cast<double>(mass[L]) / 4294967296.0;
  std::vector<double> state(k, 0.0), next(k, 0.0);
  state[0] = 1.0;
  double en = 0.0, eb = 0.0, left = 1.0;
  for (int n = 1; n <= 4 * k + 8 && left > 1e-15; ++n) {
    std::fill(next.begin(), next.end(), 0.0);
    double done = 0.0;
    for (int f = 0; f < k; ++f) {
      if (state[f] == 0.0) continue;
      for (int L = 1; L < 16; ++L) {
        if (pl[L] == 0.0) continue;
        if (f + L >= k) done += state[f] * pl[L];
        else next[f + L] += state[f] * pl[L];
      }
    }
    en += n * done;
    eb += ((n + 3) / 4) * done;
    left -= done;
    state.swap(next);
  }
  *blocks = eb;
  *samples = en;
}

constexpr double kOpsPerBlock = 40.0;  // Philox4x32-10: 20 products + 20 three-input XORs
constexpr double kOpsPerSample = 11.0;
// Staging one table into a workgroup's LDS: ~1 us of latency plus its bytes at
// 64 B per clock (2.2 GHz), during which the other workgroups keep generating.
constexpr double kStageLatencyNs = 1000.0;
constexpr double kStageBytesPerNs = 64.0 * 2.2;
constexpr double kResidentWorkgroups = 256.0;

// Candidate table sizes: VARIABLE bounds 2^8 .. 2^16 (LDS-resident up to
// 2^13, read from L2 above), FIXED 4^4 .. 4^8.
constexpr int kMinBoundLog2 = 8, kMaxBoundLog2 = 16;

// Measured device time per (edge x integer op) of the batch generation
// kernel, one figure per launch class: each LDS table size (its bytes set
// how many workgroups a CU holds beside it) and one for tables read from L2;
// one-instance batches of 2^25 and 2^27 edges at k = 26 (a = .57, b = c =
// .19, d = .05) on a table of the class's size, best of three runs each;
// the slope between the two leaves out the table build and the launches.
// Measured once per process and class.
struct ClassRate {
  bool lds;
  uint32_t n_buckets;  // LDS classes: the table's buckets (0 for the L2 class)
  double ns_per_op;
};
std::vector<ClassRate> g_rates;

double laws_ops(const uint64_t mass[16], int k) {
  double eb, en;
  sample_laws(mass, k, &eb, &en);
  return kOpsPerBlock * eb + kOpsPerSample * en;
}

// Best of three eager runs (after one that loads the code) of a one-instance
// batch of m edges into buf; *ops gets the table's ops per edge.
int time_one_instance(uint64_t bound, uint64_t m, void* buf, float* ms, double* ops) {
  rmat_instance x;
  std::memset(&x, 0, sizeof(x));
  x.a = 0.57, x.b = 0.19, x.c = 0.19, x.d = 0.05;
  x.k = 26;
  x.path_mode = RMAT_VARIABLE;
  x.table_bound = bound;
  x.seed = 1;
  x.m = m;
  x.out_src = buf;
  x.out_dst = static_cast<uint32_t*>(buf) + m;
  rmat_batch_t b = nullptr;
  int rc = rmat_batch_create(&x, 1, 2048, &b);
  hipEvent_t ea = nullptr, ez = nullptr;
  float best = 1e30f;
  if (rc == RMAT_OK) {
    (void)hipEventCreate(&ea);
    (void)hipEventCreate(&ez);
    for (int rep = 0; rep < 4 && rc == RMAT_OK; ++rep) {
      (void)hipEventRecord(ea, nullptr);
      rc = rmat_batch_enqueue(b, nullptr);
      (void)hipEventRecord(ez, nullptr);
      (void)hipEventSynchronize(ez);
      float t = 0.0f;
      (void)hipEventElapsedTime(&t, ea, ez);
      if (rep > 0) best = std::min(best, t);
    }
    if (rc == RMAT_OK) rc = rmat_batch_check(b);
  }
  if (rc == RMAT_OK) {
    std::vector<char> ex(36 * (1ull << 16));
    rmat_info info;
    rc = rmat_batch_table_info(b, 0, &info);
    if (rc == RMAT_OK) rc = rmat_batch_table_export(b, 0, ex.data(), ex.size());
    if (rc == RMAT_OK) {
      uint64_t mass[16] = {0};
      const uint64_t nb = info.n_buckets;
      const uint64_t* w = reinterpret_cast<const uint64_t*>(ex.data());
      const uint32_t* len = reinterpret_cast<const uint32_t*>(ex.data() + 16 * nb);
      for (uint64_t j = 0; j < nb; ++j) mass[len[j] & 15] += w[j];
      *ops = laws_ops(mass, 26);
    }
  }
  if (ea) (void)hipEventDestroy(ea);
  if (ez) (void)hipEventDestroy(ez);
  rmat_batch_free(b);
  *ms = best;
  return rc;
}

int measure_class(uint64_t bound, double* ns_per_op) {
  const uint64_t m1 = 1ull << 25, m2 = 1ull << 27;
  void* buf = nullptr;
  hipError_t e = hipMalloc(&buf, 2 * m2 * sizeof(uint32_t));
  if (e != hipSuccess) return rmat::hip_fail(e, "hipMalloc(autotune calibration)");
  float t1 = 0.0f, t2 = 0.0f;
  double ops = 0.0;
  int rc = time_one_instance(bound, m1, buf, &t1, &ops);
  if (rc == RMAT_OK) rc = time_one_instance(bound, m2, buf, &t2, &ops);
  (void)hipFree(buf);
  if (rc) return rc;
  const double slope = static_cast<double>(t2 - t1) * 1e6 / (static_cast<double>(m2 - m1) * ops);
  *ns_per_op = slope > 0.0 ? slope : static_cast<double>(t2) * 1e6 / (static_cast<double>(m2) * ops);
  return RMAT_OK;
}

// The rate of the launch class of a table of nb buckets (32-bit ids).
int class_rate(uint32_t nb, double* ns_per_op) {
  const bool lds = nb <= rmat::lds_table_limit();
  const uint32_t key = lds ? nb : 0u;
  for (const ClassRate& c : g_rates)
    if (c.lds == lds && c.n_buckets == key) {
      *ns_per_op = c.ns_per_op;
      return RMAT_OK;
    }
  double ns = 0.0;
  int rc = measure_class(nb, &ns);
  if (rc) return rc;
  g_rates.push_back(ClassRate{lds, key, ns});
  *ns_per_op = ns;
  return RMAT_OK;
}

// Host-clock ms of one eager run of a batch of `inst` with work items of
// work_blocks blocks (the best of two runs after a first one).
int time_batch(const std::vector<rmat_instance>& inst, uint32_t work_blocks, double* ms) {
  rmat_batch_t b = nullptr;
  int rc = rmat_batch_create(inst.data(), static_cast<int>(inst.size()), work_blocks, &b);
  if (rc) return rc;
  double best = 1e300;
  for (int rep = 0; rep < 3 && rc == RMAT_OK; ++rep) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      rc = rmat::hip_fail(e, "autotune timing");
      break;
    }
    const auto t0 = std::chrono::steady_clock::now();
    rc = rmat_batch_enqueue(b, nullptr);
    e = hipDeviceSynchronize();
    if (rc == RMAT_OK && e != hipSuccess) rc = rmat::hip_fail(e, "autotune timing");
    const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep > 0) best = std::min(best, t);
  }
  if (rc == RMAT_OK) rc = rmat_batch_check(b);
  rmat_batch_free(b);
  if (rc == RMAT_OK) *ms = best;
  return rc;
}

}  // namespace

// Largest work list of one batch (24 bytes per item on the host and the device).
constexpr uint64_t kMaxWorkItems = 1ull << 28;

extern "C" {

static int rmat_batch_create_body(const rmat_instance* inst, int n, uint32_t work_blocks, rmat_batch_t* out) {
  rmat::clear_error();
  if (!out) return set_error(RMAT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!inst || n <= 0) return set_error(RMAT_EINVAL, "empty instance list");
  rmat_batch* b = new (std::nothrow) rmat_batch();
  if (!b) return set_error(RMAT_ENOMEM, "host allocation of the batch failed");
  b->n = n;
  b->work_blocks = work_blocks ? work_blocks : 2048;
  b->inst.assign(inst, inst + n);
  b->shape.resize(n);
  int rc = RMAT_OK;
  for (int i = 0; i < n && rc == RMAT_OK; ++i) rc = validate_instance(b->inst[i], i, &b->shape[i]);
  if (rc == RMAT_OK) rc = rmat::check_device();
  if (rc) {
    destroy(b);
    return rc;
  }
  // the work list is bounded before it is built (it grows with m)
  uint64_t n_work = 0;
  for (int i = 0; i < n; ++i) {
    const rmat_instance& x = b->inst[i];
    if (x.m == 0) continue;
    const uint64_t nblk = ((x.edge_begin + (x.m - 1)) >> 6) - (x.edge_begin >> 6) + 1;
    n_work += (nblk + b->work_blocks - 1) / b->work_blocks;
    if (n_work > kMaxWorkItems) {
      destroy(b);
      return set_error(RMAT_EINVAL, "the batch needs more than %llu work items of %u blocks (instance %d)",
                       static_cast<unsigned long long>(kMaxWorkItems), b->work_blocks, i);
    }
  }
  // groups by id width and table residency; work items in instance order
  const uint32_t lds_limit = rmat::lds_table_limit();
  for (int i = 0; i < n; ++i) {
    const uint32_t nb = static_cast<uint32_t>(b->shape[i].n_buckets);
    if (rmat::tile_blocks(nb, b->inst[i].k > 32, nb <= lds_limit) == 0) {
      destroy(b);
      return set_error(RMAT_EINVAL, "instance %d: a table of %u buckets leaves no LDS for the generation queues", i,
                       nb);
    }
  }
  std::vector<rmat::GenWorkItem> items;
  items.reserve(n_work);
  std::vector<uint32_t> group_first;
  for (int wide = 0; wide < 2; ++wide)
    for (int lds = 1; lds >= 0; --lds) {
      Group g;
      g.wide = wide;
      g.lds = lds;
      g.general = 0;
      g.max_buckets = 0;
      g.items = nullptr;
      g.counter = nullptr;
      const uint32_t first_item = static_cast<uint32_t>(items.size());
      for (int i = 0; i < n; ++i) {
        const rmat_instance& x = b->inst[i];
        const rmat::Shape& S = b->shape[i];
        if ((x.k > 32) != (wide != 0) || (S.n_buckets <= lds_limit) != (lds != 0)) continue;
        g.max_buckets = std::max<uint32_t>(g.max_buckets, static_cast<uint32_t>(S.n_buckets));
        if (x.m == 0) continue;
        if (x.flags & (RMAT_UNDIRECTED | RMAT_SCRAMBLE)) g.general = 1;
        const uint64_t first = x.edge_begin >> 6;
        const uint64_t nblk = ((x.edge_begin + (x.m - 1)) >> 6) - first + 1;
        for (uint64_t f = 0; f < nblk; f += b->work_blocks) {
          rmat::GenWorkItem w;
          w.inst = static_cast<uint32_t>(i);
          w.first = f;
          w.n_blocks = static_cast<uint32_t>(std::min<uint64_t>(b->work_blocks, nblk - f));
          items.push_back(w);
        }
      }
      g.n_items = static_cast<uint32_t>(items.size()) - first_item;
      b->max_buckets = std::max(b->max_buckets, g.max_buckets);
      if (g.n_items == 0) continue;
      b->groups.push_back(g);
      group_first.push_back(first_item);
    }
  b->n_items = static_cast<uint32_t>(items.size());
  if (b->groups.size() > static_cast<size_t>(n)) {  // cannot happen: every group holds an instance
    destroy(b);
    return set_error(RMAT_EDEVICE, "internal: more generation groups than instances");
  }
  // device memory: tables | scratch, jobs, instances, items, counters (one 256-byte line each)
  const uint64_t inst_bytes = align_up(n * sizeof(rmat::GenInst), 256);
  const uint64_t item_bytes = align_up(items.size() * sizeof(rmat::GenWorkItem), 256);
  const uint64_t ctr_bytes = 256 * std::max<size_t>(1, b->groups.size());
  TableSet T;
  rc = alloc_tables(b->shape, b->inst, inst_bytes + item_bytes + ctr_bytes, &T);
  if (rc) {
    destroy(b);
    return rc;
  }
  b->d_tables = T.d_tables;
  b->d_aux = T.d_aux;
  b->views = T.views;
  b->d_jobs = T.d_jobs;
  b->device_bytes = T.bytes;
  b->d_insts = reinterpret_cast<rmat::GenInst*>(T.d_extra);
  auto* d_items = reinterpret_cast<rmat::GenWorkItem*>(T.d_extra + inst_bytes);
  auto* d_counters = reinterpret_cast<unsigned int*>(T.d_extra + inst_bytes + item_bytes);
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    b->groups[gi].items = d_items + group_first[gi];
    b->groups[gi].counter = d_counters + 64 * gi;
    T.jobs[gi].reset_counter = b->groups[gi].counter;  // build job gi zeroes group gi's counter
  }
  std::vector<rmat::GenInst> dinst(n);
  for (int i = 0; i < n; ++i) {
    const rmat_instance& x = b->inst[i];
    rmat::GenInst& d = dinst[i];
    d.records = b->views[i].records;
    d.n_buckets = static_cast<uint32_t>(b->shape[i].n_buckets);
    d.table_mask = 0;
    d.bmask = ((1u << b->shape[i].bucket_bits) - 1u) << 4;
    d.k = static_cast<uint32_t>(x.k);
    d.key0 = static_cast<uint32_t>(x.seed);
    d.key1 = static_cast<uint32_t>(x.seed >> 32);
    d.edge_begin = x.edge_begin;
    d.m = x.m;
    d.first_block = x.edge_begin >> 6;
    d.n_blocks = x.m ? ((x.edge_begin + (x.m - 1)) >> 6) - d.first_block + 1 : 0;
    d.out_src = x.out_src;
    d.out_dst = x.out_dst;
    d.digest = nullptr;
    d.ctr3 = 0;
    d.kron_k = 2;
    d.src_prefix = d.dst_prefix = 0;
    d.epi = static_cast<uint32_t>(x.flags);
    if (d.epi) rmat::scramble_params(x.scramble_key, x.k, &d);
    b->total_edges += x.m;
  }
  // every byte 0xFF: each table's build status reads -1 (not built) until the first run
  hipError_t e = hipMemset(b->d_tables, 0xFF, T.table_bytes);
  if (e == hipSuccess) e = hipMemcpy(b->d_jobs, T.jobs.data(), n * sizeof(rmat::BuildJob), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_insts, dinst.data(), n * sizeof(rmat::GenInst), hipMemcpyHostToDevice);
  if (e == hipSuccess && !items.empty())
    e = hipMemcpy(d_items, items.data(), items.size() * sizeof(rmat::GenWorkItem), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(d_counters, 0, ctr_bytes);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    destroy(b);
    return rmat::hip_fail(e, "batch upload");
  }
  for (const Group& g : b->groups) b->tile = std::max(b->tile, rmat::tile_blocks(g.max_buckets, g.wide, g.lds));
  *out = b;
  return RMAT_OK;
}

int rmat_batch_create(const rmat_instance* inst, int n, uint32_t work_blocks, rmat_batch_t* out) {
  RMAT_GUARD("rmat_batch_create", rmat_batch_create_body(inst, n, work_blocks, out));
}

int rmat_batch_enqueue(rmat_batch_t b, void* stream) {
  rmat::clear_error();
  if (!b) return set_error(RMAT_EINVAL, "NULL batch");
  return enqueue(b, static_cast<hipStream_t>(stream));
}

int rmat_batch_launch_graph(rmat_batch_t b, void* stream) {
  rmat::clear_error();
  if (!b) return set_error(RMAT_EINVAL, "NULL batch");
  if (!b->exec) {
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return rmat::hip_fail(e, "hipStreamCreate(capture)");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int rc = e == hipSuccess ? enqueue(b, cs) : rmat::hip_fail(e, "hipStreamBeginCapture");
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e2 != hipSuccess) return rmat::hip_fail(e2, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return rmat::hip_fail(e, "hipGraphInstantiate");
    }
    b->graph = g;
  }
  hipError_t e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return rmat::hip_fail(e, "hipGraphLaunch");
  return RMAT_OK;
}

int rmat_batch_check(rmat_batch_t b) {
  rmat::clear_error();
  if (!b) return set_error(RMAT_EINVAL, "NULL batch");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return rmat::hip_fail(e, "batch run");
  for (int i = 0; i < b->n; ++i) {
    int32_t err = 0;
    e = hipMemcpy(&err, &b->views[i].stats->error, sizeof(err), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return rmat::hip_fail(e, "batch check");
    if (err != 0)
      return set_error(err == rmat::kBuildResidual ? RMAT_EINVAL : RMAT_EDEVICE,
                       "instance %d: table build failed on the device (code %d)", i, err);
  }
  return RMAT_OK;
}

int rmat_batch_table_export(rmat_batch_t b, int i, void* host_buf, size_t nbytes) {
  rmat::clear_error();
  if (!b || i < 0 || i >= b->n) return set_error(RMAT_EINVAL, "NULL batch or instance index out of range");
  return rmat::export_table(b->views[i], b->shape[i].n_buckets, host_buf, nbytes);
}

int rmat_batch_table_info(rmat_batch_t b, int i, rmat_info* out) {
  rmat::clear_error();
  if (!b || !out || i < 0 || i >= b->n) return set_error(RMAT_EINVAL, "NULL batch or info pointer, or index out of range");
  rmat::BuildStats st;
  hipError_t e = hipMemcpy(&st, b->views[i].stats, sizeof(st), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return rmat::hip_fail(e, "batch table info");
  if (st.error != 0) return set_error(RMAT_EINVAL, "instance %d: table not built (code %d)", i, st.error);
  const rmat_instance& x = b->inst[i];
  rmat::fill_info(out, x.k, x.path_mode, x.table_bound, b->shape[i], st, rmat::table_bytes(b->shape[i]));
  return RMAT_OK;
}

int rmat_batch_get_info(rmat_batch_t b, rmat_batch_info* out) {
  rmat::clear_error();
  if (!b || !out) return set_error(RMAT_EINVAL, "NULL batch or info pointer");
  out->n_instances = static_cast<uint32_t>(b->n);
  out->n_launches = static_cast<uint32_t>(b->groups.size());
  out->n_work_items = b->n_items;
  out->work_blocks = b->work_blocks;
  out->tile_blocks = b->tile;
  out->max_buckets = b->max_buckets;
  out->total_edges = b->total_edges;
  out->device_bytes = b->device_bytes;
  return RMAT_OK;
}

int rmat_batch_free(rmat_batch_t b) {
  rmat::clear_error();
  destroy(b);
  return RMAT_OK;
}

static int rmat_batch_autotune_body(rmat_instance* inst, int n, rmat_autotune_report* report) {
  rmat::clear_error();
  const auto t0 = std::chrono::steady_clock::now();
  if (!inst || n <= 0) return set_error(RMAT_EINVAL, "empty instance list");
  // candidate tables of every instance to tune (host only)
  std::vector<int> who;
  std::vector<rmat_instance> cand;
  std::vector<rmat::Shape> shapes;
  uint32_t n_tuned = 0, n_cand = 0;
  bool outputs = true;
  for (int i = 0; i < n; ++i) {
    if (inst[i].table_bound != 0) continue;
    ++n_tuned;
    if (inst[i].m > 0 && (!inst[i].out_src || !inst[i].out_dst)) outputs = false;
    const int cap = std::min(std::max(inst[i].k, 1), rmat::kMaxDepthCap);
    std::vector<uint64_t> bounds;
    if (inst[i].path_mode == RMAT_FIXED) {
      for (int l = std::min(4, cap); l <= std::min(kMaxBoundLog2 / 2, cap); ++l) bounds.push_back(1ull << (2 * l));
    } else {
      for (int e2 = kMinBoundLog2; e2 <= kMaxBoundLog2; ++e2) bounds.push_back(1ull << e2);
    }
    n_cand = std::max<uint32_t>(n_cand, static_cast<uint32_t>(bounds.size()));
    for (uint64_t bound : bounds) {
      rmat_instance c = inst[i];
      c.table_bound = bound;
      rmat::Shape S;
      const double q[4] = {c.a, c.b, c.c, c.d};
      if (rmat::validate_and_size(q, c.k, c.table_bound, c.path_mode, &S) != RMAT_OK) {
        char msg[512];
        std::snprintf(msg, sizeof(msg), "instance %d: %s", i, rmat_last_error());
        return set_error(RMAT_EINVAL, "%s", msg);
      }
      cand.push_back(c);
      shapes.push_back(S);
      who.push_back(i);
    }
  }
  int rc = rmat::check_device();
  if (rc) return rc;
  uint64_t total_blocks = 0;
  for (int i = 0; i < n; ++i) total_blocks += (inst[i].m + 63) / 64;
  uint32_t work_blocks = static_cast<uint32_t>(std::min<uint64_t>(
      8192, std::max<uint64_t>(128, total_blocks / (static_cast<uint64_t>(256) * 8))));
  std::vector<uint64_t> model(n, 0);
  double model_cost = 0.0;
  if (!cand.empty()) {
    TableSet T;
    if ((rc = alloc_tables(shapes, cand, 0, &T))) return rc;
    hipError_t e = hipMemcpy(T.d_jobs, T.jobs.data(), T.jobs.size() * sizeof(rmat::BuildJob), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = rmat::launch_table_build(T.d_jobs, static_cast<int>(T.jobs.size()), nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    std::vector<rmat::BuildStats> st(cand.size());
    for (size_t c = 0; c < cand.size() && e == hipSuccess; ++c)
      e = hipMemcpy(&st[c], T.views[c].stats, sizeof(rmat::BuildStats), hipMemcpyDeviceToHost);
    free_tables(&T);
    if (e != hipSuccess) return rmat::hip_fail(e, "autotune candidate tables");
    // the model: exact ops per edge of each candidate (its length law) at
    // the measured rate of its launch class, plus table staging.  The LDS
    // tables of a batch share one launch laid out for the largest of them,
    // so they all run at that table's rate: for each largest LDS size M,
    // every instance takes its cheapest candidate among the LDS tables of at
    // most M buckets (at M's rate) and the tables read from L2 (at theirs),
    // and the M with the least total cost wins (M = 0: L2 tables only).
    auto is_lds = [&](size_t c) { return shapes[c].n_buckets <= rmat::lds_table_limit(); };
    auto cost_at = [&](size_t c, double rate) {
      const double gen = static_cast<double>(cand[c].m) * rate * laws_ops(st[c].len_mass, cand[c].k);
      const double items = std::ceil(static_cast<double>((cand[c].m + 63) / 64) / work_blocks);
      const double stage_one =
          is_lds(c) ? kStageLatencyNs + static_cast<double>(shapes[c].n_buckets) * 16.0 / kStageBytesPerNs : 0.0;
      return gen + items * stage_one / kResidentWorkgroups;
    };
    std::vector<uint32_t> sizes{0u};  // the largest LDS sizes to try
    double l2_rate = 0.0;
    bool have_l2 = false;
    for (size_t c = 0; c < cand.size(); ++c) {
      if (st[c].error != 0) continue;
      const uint32_t nb = static_cast<uint32_t>(shapes[c].n_buckets);
      if (!is_lds(c)) {
        if (!have_l2 && (rc = class_rate(nb, &l2_rate))) return rc;
        have_l2 = true;
      } else if (std::find(sizes.begin(), sizes.end(), nb) == sizes.end()) {
        sizes.push_back(nb);
      }
    }
    std::vector<double> best(n, 1e300);
    double best_total = 1e300;
    for (uint32_t M : sizes) {
      double rate_m = 0.0;
      if (M != 0 && (rc = class_rate(M, &rate_m))) return rc;
      std::vector<double> cost_i(n, 1e300);
      std::vector<uint64_t> pick_i(n, 0);
      for (size_t c = 0; c < cand.size(); ++c) {
        if (st[c].error != 0) continue;
        const bool lds = is_lds(c);
        if (lds && shapes[c].n_buckets > M) continue;
        const double cost = cost_at(c, lds ? rate_m : l2_rate);
        const int i = who[c];
        if (cost < cost_i[i]) {
          cost_i[i] = cost;
          pick_i[i] = cand[c].table_bound;
        }
      }
      double total = 0.0;
      bool every = true;
      for (int i = 0; i < n; ++i)
        if (inst[i].table_bound == 0) {
          every = every && pick_i[i] != 0;
          total += cost_i[i];
        }
      if (every && total < best_total) {
        best_total = total;
        best = cost_i;
        model = pick_i;
      }
    }
    for (int i = 0; i < n; ++i)
      if (inst[i].table_bound == 0) {
        if (model[i] == 0) return set_error(RMAT_EDEVICE, "instance %d: every candidate table failed", i);
        model_cost += best[i];
      }
  }
  // With the callers' outputs, the model's choice is checked by measurement
  // against one table size for all (2^12 and 2^13: the largest LDS tables
  // with two workgroups per CU and with one), and the fastest is kept; then the
  // work-item size is measured.  Without outputs the model decides alone.
  uint32_t chosen = 0;
  double times[3] = {0.0, 0.0, 0.0};
  std::vector<uint64_t> pick = model;
  if (outputs && n_tuned > 0) {
    std::vector<std::vector<uint64_t>> configs(3, model);
    for (int i = 0; i < n; ++i) {
      if (inst[i].table_bound != 0) continue;
      const bool fixed = inst[i].path_mode == RMAT_FIXED;
      const int cap = std::min(std::max(inst[i].k, 1), rmat::kMaxDepthCap);
      configs[1][i] = fixed ? (1ull << (2 * std::min(6, cap))) : 4096;
      configs[2][i] = fixed ? (1ull << (2 * std::min(6, cap))) : 8192;
    }
    std::vector<rmat_instance> trial(inst, inst + n);
    for (uint32_t c = 0; c < 3; ++c) {
      for (int i = 0; i < n; ++i)
        if (inst[i].table_bound == 0) trial[i].table_bound = configs[c][i];
      if ((rc = time_batch(trial, work_blocks, &times[c]))) return rc;
    }
    // a single size for all replaces the model's bounds only when it is
    // faster by more than the run-to-run spread (1%)
    double best = times[0];
    for (uint32_t c = 1; c < 3; ++c)
      if (times[c] < 0.99 * best) {
        best = times[c];
        chosen = c;
      }
    pick = configs[chosen];
    for (int i = 0; i < n; ++i)
      if (inst[i].table_bound == 0) trial[i].table_bound = pick[i];
    uint32_t best_wb = work_blocks;
    for (uint32_t wb : {work_blocks / 4, work_blocks * 4}) {
      if (wb < 64 || wb > 65536) continue;
      double t = 0.0;
      if ((rc = time_batch(trial, wb, &t))) return rc;
      if (t < 0.99 * best) {
        best = t;
        best_wb = wb;
      }
    }
    work_blocks = best_wb;
  }
  for (int i = 0; i < n; ++i)
    if (inst[i].table_bound == 0) inst[i].table_bound = pick[i];
  if (report) {
    std::memset(report, 0, sizeof(*report));
    report->search_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    double r4096 = 0.0;
    if ((rc = class_rate(4096, &r4096))) return rc;
    report->calibration_ns = r4096;
    report->n_tuned = n_tuned;
    report->n_candidates = n_cand;
    report->work_blocks = work_blocks;
    report->chosen = chosen;
    report->measured = outputs && n_tuned > 0 ? 1u : 0u;
    report->model_ms = model_cost * 1e-6;
    report->tuned_ms = times[0];
    report->all_4096_ms = times[1];
    report->all_8192_ms = times[2];
  }
  return RMAT_OK;
}

int rmat_batch_autotune(rmat_instance* inst, int n, rmat_autotune_report* report) {
  RMAT_GUARD("rmat_batch_autotune", rmat_batch_autotune_body(inst, n, report));
}

}  // extern "C"
