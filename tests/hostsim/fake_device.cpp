// Host-only fake of the HIP runtime calls and of the sampler's kernel
// launchers, for testing the server's scheduling logic with g++ and the host
// sanitizers.  "Device" memory is host memory; a launch acts at once on it:
// the table build writes a tag naming its parameters, the batch generation
// checks its work list and records which edges of which request it covered
// and XORs a per-edge word into the request's digest.  Events complete at
// random (seeded), never out of order.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <vector>

#include "rmat_internal.h"
#include "sim_hash.h"

namespace {
std::mt19937_64 g_rng(1);
double g_ready_p = 0.5;
int g_fail = 0;
std::map<uint64_t, std::vector<uint32_t>> g_cov;  // request seed -> per-edge write count
uint64_t g_launches = 0;
bool g_whole_cover = false;   // partitioned launches: every instance covered once
uint64_t g_cover_insts = 0;   // instances the last such launch covered

void fail(const char* what) {
  std::fprintf(stderr, "fake device: %s\n", what);
  g_fail = 1;
}
}  // namespace

struct ihipStream_t {
  int dummy;
};
struct ihipEvent_t {
  bool recorded = false, ready = false;
};

extern "C" {
void sim_seed(uint64_t s, double ready_p) {
  g_rng.seed(s);
  g_ready_p = ready_p;
}
int sim_failed() { return g_fail; }
// Partitioned-graph mode: each batch launch must cover every block of every
// instance it lists exactly once (instances 0 .. n-1); tiles may be narrower
// than the launch's ids (their prefixes widen them).
void sim_whole_cover(int on) { g_whole_cover = on != 0; }
uint64_t sim_cover_insts() { return g_cover_insts; }
uint64_t sim_launches() { return g_launches; }
// 0 if every edge of the request with this seed was generated exactly once
// (partial: at most once, for a request cut short by a failed build), else
// -1; forgets the request.
int sim_take_coverage(uint64_t seed, uint64_t m, int partial) {
  auto it = g_cov.find(seed);
  if (m == 0 || (partial && it == g_cov.end())) return it == g_cov.end() ? 0 : -1;
  if (it == g_cov.end() || it->second.size() != m) return -1;
  for (uint32_t c : it->second)
    if (c > 1 || (c == 0 && !partial)) return -1;
  g_cov.erase(it);
  return 0;
}
}

static uint64_t g_mallocs = 0;
extern "C" uint64_t sim_mallocs() { return g_mallocs; }

hipError_t hipMalloc(void** p, size_t n) {
  ++g_mallocs;
  *p = std::aligned_alloc(256, (n + 255) / 256 * 256);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  std::memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) {
  return hipMemcpy(d, s, n, k);
}
hipError_t hipMemset(void* d, int v, size_t n) {
  std::memset(d, v, n);
  return hipSuccess;
}
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  std::memset(p, 0, sizeof(*p));
  std::strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-");
  p->multiProcessorCount = 256;
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "fake device error"; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new ihipStream_t();
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new ihipEvent_t();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  e->recorded = true;
  e->ready = false;
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  if (!e->recorded) return hipSuccess;
  if (!e->ready && std::uniform_real_distribution<double>(0, 1)(g_rng) < g_ready_p) e->ready = true;
  return e->ready ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  e->ready = true;
  return hipSuccess;
}
// streams run in order on the fake device: a wait on an event changes nothing
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned int) { return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}

namespace rmat {

hipError_t launch_table_build(const BuildJob* jobs, int n, hipStream_t) {
  ++g_launches;
  for (int j = 0; j < n; ++j) {
    const BuildJob& J = jobs[j];
    if (!J.records || !J.stats || J.n_buckets == 0) fail("build job without outputs");
    uint64_t tag[2] = {sim::table_tag(J.q, J.k, J.mode), J.n_buckets};
    std::memcpy(J.records, tag, sizeof(tag));
    std::memset(J.stats, 0, sizeof(BuildStats));
    J.stats->error = sim::build_fails(J.q) ? kBuildResidual : kBuildOk;
    J.stats->n_items = J.n_items;
    J.stats->min_len = J.stats->max_len = 1;
    if (J.reset_counter) *J.reset_counter = 0;
  }
  return hipSuccess;
}

hipError_t launch_table_build_one(const BuildJob& job, hipStream_t s) { return launch_table_build(&job, 1, s); }

hipError_t launch_generate_batch(const BatchArgs& a, hipStream_t) {
  ++g_launches;
  if (a.n_items == 0) return hipSuccess;
  if (*a.counter != 0) fail("work counter not zero at launch");
  // one instance's blocks [first, first + n_blocks)
  auto run = [&](const GenInst& I, uint64_t first, uint64_t n_blocks) {
    uint64_t tag[2];
    std::memcpy(tag, I.records, sizeof(tag));
    if (tag[1] != I.n_buckets) fail("instance table of another size");
    if (n_blocks == 0 || first + n_blocks > I.n_blocks) fail("work item outside its instance");
    if (g_whole_cover ? (I.k > 32 && !a.wide) : ((I.k > 32) != (a.wide != 0))) fail("id width of the launch");
    if ((I.n_buckets <= lds_table_limit()) != (a.lds != 0)) fail("table residency of the launch");
    if (I.n_buckets > a.max_buckets) fail("table larger than the launch's LDS layout");
    if (I.first_block != I.edge_begin >> 6) fail("first block");
    const uint64_t seed = static_cast<uint64_t>(I.key0) | static_cast<uint64_t>(I.key1) << 32;
    std::vector<uint32_t>& cov = g_cov[seed];
    if (cov.size() != I.m) cov.assign(I.m, 0);
    const uint64_t last = I.edge_begin + (I.m - 1);
    for (uint64_t b = first; b < first + n_blocks; ++b) {
      const uint64_t base = (I.first_block + b) << 6;
      for (uint64_t l = 0; l < 64; ++l) {
        const uint64_t e = base + l;
        if (e < I.edge_begin || e > last) continue;
        ++cov[e - I.edge_begin];
        if (a.digest && I.digest) *I.digest ^= sim::edge_word(e, seed, tag[0]);
      }
    }
  };
  std::map<uint32_t, std::vector<uint32_t>> blocks;  // instance -> per-block visits
  auto visit = [&](uint32_t inst, uint64_t first, uint64_t n) {
    if (!g_whole_cover) return;
    std::vector<uint32_t>& v = blocks[inst];
    if (v.empty()) v.assign(a.insts[inst].n_blocks, 0);
    for (uint64_t b = first; b < first + n && b < v.size(); ++b) ++v[b];
  };
  for (uint32_t it = 0; it < a.n_items; ++it) {
    const GenWorkItem& W = a.items[it];
    if (W.n_inst > 1) {  // whole instances on the first one's table
      uint64_t sum = 0;
      for (uint32_t j = 0; j < W.n_inst; ++j) {
        const GenInst& I = a.insts[W.inst + j];
        if (I.records != a.insts[W.inst].records) fail("packed instances on different tables");
        run(I, 0, I.n_blocks);
        visit(W.inst + j, 0, I.n_blocks);
        sum += I.n_blocks;
      }
      if (sum != W.n_blocks) fail("packed item's block count");
    } else {
      run(a.insts[W.inst], W.first, W.n_blocks);
      visit(W.inst, W.first, W.n_blocks);
    }
  }
  if (g_whole_cover) {
    uint32_t expect = 0;
    for (const auto& kv : blocks) {
      if (kv.first != expect++) fail("an instance without work items");
      for (uint32_t c : kv.second)
        if (c != 1) fail("a block of an instance not covered exactly once");
    }
    g_cover_insts = blocks.size();
  }
  *a.counter = a.n_items;
  return hipSuccess;
}

// The partitioned tiles' launch: the list must hold one table, instances with
// blocks and their running costs; then the waves' parts of the cost line are
// cut and searched exactly as generate_tiles_kernel does, for several grid
// sizes, and every block of every instance must fall in exactly one part.
hipError_t launch_generate_tiles(const TilesArgs& a, hipStream_t) {
  ++g_launches;
  if (a.n_inst == 0 || a.total_blocks == 0) return hipSuccess;
  const uint64_t* cum = a.cum_cost;
  uint64_t blocks = 0;
  if (cum[0] != 0) fail("running costs: start");
  for (uint32_t i = 0; i < a.n_inst; ++i) {
    const GenInst& I = a.insts[i];
    if (I.n_blocks == 0 || cum[i + 1] - cum[i] != a.inst_cost + I.n_blocks) fail("running costs");
    if (I.records != a.insts[0].records || I.n_buckets != a.n_buckets) fail("tiles on different tables");
    if (g_whole_cover ? (I.k > 32 && !a.wide) : ((I.k > 32) != (a.wide != 0))) fail("id width of the launch");
    if ((I.n_buckets <= lds_table_limit()) != (a.lds != 0)) fail("table residency of the launch");
    blocks += I.n_blocks;
  }
  if (blocks != a.total_blocks) fail("total blocks");
  std::vector<std::vector<uint8_t>> seen(a.n_inst);
  const uint64_t total = cum[a.n_inst];
  for (uint64_t n_waves : {uint64_t{1}, uint64_t{7}, uint64_t{6144}, total + 5}) {
    for (uint32_t i = 0; i < a.n_inst; ++i) seen[i].assign(a.insts[i].n_blocks, 0);
    for (uint64_t w = 0; w < n_waves; ++w) {
      const uint64_t q = total / n_waves, r = total % n_waves;
      const uint64_t lo = q * w + (w < r ? w : r), hi = lo + q + (w < r ? 1 : 0);
      if (lo >= hi) continue;
      uint32_t lo_i = 0, hi_i = a.n_inst;  // the kernel's 64-way search, lane by lane
      while (hi_i - lo_i > 1) {
        const uint32_t step = (hi_i - lo_i + 63) / 64;
        uint32_t last = 64;
        for (uint32_t lane = 0; lane < 64; ++lane) {
          const uint32_t idx = lo_i + lane * step;
          if (idx < hi_i && cum[idx] <= lo) last = lane;
          else if (last == 64) fail("search: lane 0 below the range");
        }
        lo_i += last * step;
        hi_i = lo_i + step < hi_i ? lo_i + step : hi_i;
      }
      if (!(cum[lo_i] <= lo && lo < cum[lo_i + 1])) fail("search: wrong instance");
      for (uint32_t i = lo_i; i < a.n_inst && cum[i] < hi; ++i) {
        const uint64_t c0 = cum[i] + a.inst_cost, end = hi < cum[i + 1] ? hi : cum[i + 1];
        if (end <= c0) continue;
        for (uint64_t b = lo > c0 ? lo - c0 : 0; b < end - c0; ++b) ++seen[i][b];
      }
    }
    for (const auto& v : seen)
      for (uint8_t c : v)
        if (c != 1) fail("a block of the tiles not in exactly one wave's part");
  }
  if (g_whole_cover) g_cover_insts = a.n_inst;
  return hipSuccess;
}

hipError_t launch_generate(const GenerateArgs&, hipStream_t) { return hipSuccess; }
hipError_t launch_generate_reduce(const GenerateArgs&, hipStream_t) { return hipSuccess; }
hipError_t launch_generate_degrees(const GenerateArgs&, hipStream_t) { return hipSuccess; }
hipError_t launch_degree_distribution(const uint32_t*, uint64_t, uint32_t, unsigned long long*, hipStream_t) {
  return hipSuccess;
}
hipError_t prepare_kernels() { return hipSuccess; }
uint32_t lds_table_limit() { return 8192; }
uint32_t tile_blocks(uint32_t, int, int) { return 8; }
uint64_t reduce_partials_bytes() { return 1u << 20; }
hipError_t static_reduce_workspace(GenerateArgs*) { return hipErrorInvalidValue; }

}  // namespace rmat
