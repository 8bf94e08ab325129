// partition.cpp -- partitioned, communication-free generation (Sec. 3): the
// adjacency matrix is cut into 2^t x 2^t tiles, the m edges are divided over
// the tiles top-down through the quadrant tree (only into the subtrees that
// meet the requested tile rows), and every tile's edges are generated on the
// device by the batch kernel, one instance per tile.
//
// Counting is host work, O(nodes visited): each node splits its count n
// into four by three binomial draws, n_a = Bin(n, a), n_b = Bin(n - n_a,
// b / (b + c + d)), n_c = Bin(n - n_a - n_b, c / (c + d)), n_d = the rest.
// Bin(n, p) is inversion for n min(p, 1 - p) < 30 and BTPE (Kachitvichyanukul
// & Schmeiser, CACM 31(2), 1988) above, p > 1/2 as n - Bin(n, 1 - p).  The
// uniforms of node (level l, row prefix R, column prefix C) come from
// Philox4x32-10 under the seed with counter (R, C, i, 2^31 + l), two 53-bit
// uniforms per counter block.  Every floating-point step is a fixed sequence
// of IEEE operations and libm calls, so the counts are reproducible.
//
// Edge j of tile (R, C) uses the counter stream (j_lo, j_hi, block,
// 1 + R 2^t + C) for the remaining k - t letters, and its ids get the tile's
// prefixes R 2^(k-t) and C 2^(k-t).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <thread>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "rmat.h"
#include "rmat_internal.h"

struct rmat_table;  // defined in api.cpp; reached through the accessors below

namespace {

using rmat::set_error;

// Philox4x32-10 [Salmon et al., SC'11] on the host.
void philox_host(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3], k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    const uint64_t m0 = static_cast<uint64_t>(x0) * 0xD2511F53u;
    const uint64_t m1 = static_cast<uint64_t>(x2) * 0xCD9E8D57u;
    const uint32_t n0 = static_cast<uint32_t>(m1 >> 32) ^ x1 ^ k0;
    const uint32_t n2 = static_cast<uint32_t>(m0 >> 32) ^ x3 ^ k1;
    x1 = static_cast<uint32_t>(m1);
    x3 = static_cast<uint32_t>(m0);
    x0 = n0;
    x2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

// The uniform stream of one quadrant-tree node.
class NodeStream {
 public:
  NodeStream(uint64_t seed, uint32_t r, uint32_t c, int level) {
    key_[0] = static_cast<uint32_t>(seed);
    key_[1] = static_cast<uint32_t>(seed >> 32);
    ctr_[0] = r;
    ctr_[1] = c;
    ctr_[2] = 0;
    ctr_[3] = 0x80000000u | static_cast<uint32_t>(level);
  }
  // [0, 1) with 53 random bits: words (2i, 2i+1) of a block, high word first
  double next() {
    if (half_ == 2) {
      philox_host(ctr_, key_, w_);
      ++ctr_[2];
      half_ = 0;
    }
    const uint64_t bits = (static_cast<uint64_t>(w_[2 * half_]) << 32) | w_[2 * half_ + 1];
    ++half_;
    return static_cast<double>(bits >> 11) * (1.0 / 9007199254740992.0);
  }

 private:
  uint32_t key_[2], ctr_[4], w_[4] = {0, 0, 0, 0};
  int half_ = 2;
};

// Inversion, 0 < p <= 1/2 and n p < 30: f(0) = (1 - p)^n, then
// f(x) = f(x - 1) ((n + 1) p / (1 - p) / x - p / (1 - p)); restart past 110.
uint64_t bin_inversion(NodeStream& st, uint64_t n, double p) {
  const double q = 1.0 - p;
  const double s = p / q;
  const double a = (static_cast<double>(n) + 1.0) * s;
  const double f0 = std::pow(q, static_cast<double>(n));
  for (;;) {
    double u = st.next();
    double f = f0;
    uint64_t x = 0;
    bool again = false;
    while (u > f) {
      u -= f;
      ++x;
      if (x > n || x > 110) {
        again = true;
        break;
      }
      f *= a / static_cast<double>(x) - s;
    }
    if (!again) return x;
  }
}

// (13860 - (462 - (132 - (99 - 140/a^2)/a^2)/a^2)/a^2) / a / 166320: the
// Stirling-series remainder 1/(12a) - 1/(360a^3) + 1/(1260a^5) - 1/(1680a^7).
double lnfact_tail(double a) {
  const double a2 = a * a;
  return (13860.0 - (462.0 - (132.0 - (99.0 - 140.0 / a2) / a2) / a2) / a2) / a / 166320.0;
}

// BTPE, 0 < p <= 1/2 and n p >= 30.
uint64_t bin_btpe(NodeStream& st, uint64_t n, double p) {
  const double dn = static_cast<double>(n);
  const double r = p;
  const double q = 1.0 - p;
  const double nrq = dn * r * q;
  const double fm = dn * r + r;
  const double mode = std::floor(fm);
  const double p1 = std::floor(2.195 * std::sqrt(nrq) - 4.6 * q) + 0.5;
  const double xm = mode + 0.5;
  const double xl = xm - p1;
  const double xr = xm + p1;
  const double c = 0.134 + 20.5 / (15.3 + mode);
  const double al = (fm - xl) / (fm - xl * r);
  const double lam_l = al * (1.0 + al / 2.0);
  const double ar = (xr - fm) / (xr * q);
  const double lam_r = ar * (1.0 + ar / 2.0);
  const double p2 = p1 * (1.0 + 2.0 * c);
  const double p3 = p2 + c / lam_l;
  const double p4 = p3 + c / lam_r;
  for (;;) {
    const double u = st.next() * p4;
    double v = st.next();
    double y;
    if (u <= p1) return static_cast<uint64_t>(std::floor(xm - p1 * v + u));  // triangle
    if (u <= p2) {                                                             // parallelogram
      const double x = xl + (u - p1) / c;
      v = v * c + 1.0 - std::fabs(mode - x + 0.5) / p1;
      if (v > 1.0) continue;
      y = std::floor(x);
    } else if (u <= p3) {  // left tail
      y = std::floor(xl + std::log(v) / lam_l);
      if (y < 0.0) continue;
      v = v * (u - p2) * lam_l;
    } else {  // right tail
      y = std::floor(xr - std::log(v) / lam_r);
      if (y > dn) continue;
      v = v * (u - p3) * lam_r;
    }
    const double k = std::fabs(y - mode);
    if (k <= 20.0 || k >= nrq / 2.0 - 1.0) {
      // f(y) / f(mode) through the pmf ratio
      const double s = r / q;
      const double a = s * (dn + 1.0);
      double f = 1.0;
      if (mode < y) {
        for (double i = mode + 1.0; i <= y; i += 1.0) f *= a / i - s;
      } else if (mode > y) {
        for (double i = y + 1.0; i <= mode; i += 1.0) f /= a / i - s;
      }
      if (v <= f) return static_cast<uint64_t>(y);
      continue;
    }
    const double rho = (k / nrq) * ((k * (k / 3.0 + 0.625) + 0.1666666666666) / nrq + 0.5);
    const double t = -k * k / (2.0 * nrq);
    const double lv = std::log(v);
    if (lv < t - rho) return static_cast<uint64_t>(y);
    if (lv > t + rho) continue;
    const double x1 = y + 1.0;
    const double f1 = mode + 1.0;
    const double z = dn + 1.0 - mode;
    const double w = dn - y + 1.0;
    const double bound = xm * std::log(f1 / x1) + (dn - mode + 0.5) * std::log(z / w) +
                         (y - mode) * std::log(w * r / (x1 * q)) + lnfact_tail(f1) + lnfact_tail(z) -
                         lnfact_tail(x1) - lnfact_tail(w);
    if (lv <= bound) return static_cast<uint64_t>(y);
  }
}

uint64_t bin(NodeStream& st, uint64_t n, double p) {
  if (n == 0 || p <= 0.0) return 0;
  if (p >= 1.0) return n;
  const bool flip = p > 0.5;
  const double pp = flip ? 1.0 - p : p;
  const uint64_t x = static_cast<double>(n) * pp < 30.0 ? bin_inversion(st, n, pp) : bin_btpe(st, n, pp);
  return flip ? n - x : x;
}

constexpr size_t kCountTasks = 256;   // subtrees handed to the counting threads
constexpr size_t kCountThreads = 16;  // host threads for one count

struct Counter {
  double q[4];
  uint64_t seed;
  int t;
  uint32_t row_begin, row_end;
  uint64_t* counts;  // (row_end - row_begin) x 2^t, row-major

  struct Node {
    int level;
    uint32_t r, c;
    uint64_t n;
  };

  // The four children of node (level, r, c) holding n edges, those whose
  // tile rows meet [row_begin, row_end), in quadrant order.
  int split(const Node& x, Node out[4]) const {
    NodeStream st(seed, x.r, x.c, x.level);
    const double bcd = q[1] + q[2] + q[3];
    const double cd = q[2] + q[3];
    uint64_t child[4];
    child[0] = bin(st, x.n, q[0]);
    uint64_t rest = x.n - child[0];
    child[1] = bin(st, rest, bcd > 0.0 ? q[1] / bcd : 0.0);
    rest -= child[1];
    child[2] = bin(st, rest, cd > 0.0 ? q[2] / cd : 0.0);
    child[3] = rest - child[2];
    const int below = t - x.level - 1;
    int k = 0;
    for (int quad = 0; quad < 4; ++quad) {
      const uint32_t cr = 2 * x.r + static_cast<uint32_t>(quad >> 1);
      const uint32_t cc = 2 * x.c + static_cast<uint32_t>(quad & 1);
      const uint64_t first = static_cast<uint64_t>(cr) << below, end = static_cast<uint64_t>(cr + 1) << below;
      if (end <= row_begin || first >= row_end) continue;
      out[k++] = Node{x.level + 1, cr, cc, child[quad]};
    }
    return k;
  }

  void visit(const Node& x) {
    if (x.level == t) {
      counts[(static_cast<uint64_t>(x.r - row_begin) << t) | x.c] = x.n;
      return;
    }
    if (x.n == 0) return;
    Node ch[4];
    const int k = split(x, ch);
    for (int i = 0; i < k; ++i) visit(ch[i]);
  }

  // Every node's draws depend only on the seed and the node, so the subtrees
  // below a frontier of up to kCountTasks nodes are counted on several host
  // threads with the same result as one.
  void run(uint64_t m) {
    std::vector<Node> frontier{Node{0, 0, 0, m}};
    while (frontier.size() < kCountTasks && frontier[0].level < t - 1) {
      std::vector<Node> next;
      for (const Node& x : frontier) {
        if (x.n == 0) continue;
        Node ch[4];
        const int k = split(x, ch);
        next.insert(next.end(), ch, ch + k);
      }
      if (next.empty()) return;
      frontier.swap(next);
    }
    const size_t hw = std::max(2u, std::thread::hardware_concurrency());
    const size_t n_threads = std::min<size_t>({frontier.size(), hw, kCountThreads});
    std::atomic<size_t> next_task{0};
    auto worker = [&]() {
      for (size_t i; (i = next_task.fetch_add(1)) < frontier.size();) visit(frontier[i]);
    };
    std::vector<std::thread> pool;
    pool.reserve(n_threads);
    for (size_t i = 1; i < n_threads; ++i) {
      try {
        pool.emplace_back(worker);
      } catch (...) {  // no more threads: the ones running take the rest, same counts
        break;
      }
    }
    worker();
    for (std::thread& th : pool) th.join();
  }
};

constexpr uint64_t kMaxTilesPerCall = 1ull << 18;

int check_args(const rmat_info& info, uint64_t m, int tbits, uint32_t row_begin, uint32_t row_end) {
  if (info.initiator_k > 2 || info.n_tables > 1)
    return set_error(RMAT_EINVAL, "partitioned generation needs a single 2 x 2 (R-MAT) table");
  if (tbits < 1 || tbits > 15 || tbits >= info.k)
    return set_error(RMAT_EINVAL, "tile_bits %d outside 1..min(k - 1, 15)", tbits);
  if (row_begin >= row_end || row_end > (1u << tbits))
    return set_error(RMAT_EINVAL, "tile rows [%u, %u) not inside [0, %u)", row_begin, row_end, 1u << tbits);
  if (m > (1ull << 53)) return set_error(RMAT_EINVAL, "m above 2^53");
  if ((static_cast<uint64_t>(row_end - row_begin) << tbits) > kMaxTilesPerCall)
    return set_error(RMAT_EINVAL, "more than 2^18 tiles in one call");
  return RMAT_OK;
}

}  // namespace

namespace rmat {
// Access to the table handle (api.cpp).
const rmat_info* table_info_of(const rmat_table* t);
const TableView* table_view_of(const rmat_table* t);
const double* table_params_of(const rmat_table* t);
int finalize_table(rmat_table* t);  // waits for an asynchronous build; its status
}  // namespace rmat

namespace {
// The last counts computed, so that generating the tiles right after asking
// for their counts (the usual order) does not draw the tree twice.  Counts
// are a function of (a, b, c, d, seed, m, tile_bits, rows) alone, which is
// the key.
struct CountCache {
  std::mutex mu;
  bool valid = false;
  double q[4] = {0, 0, 0, 0};
  uint64_t seed = 0, m = 0;
  int tbits = 0;
  uint32_t row_begin = 0, row_end = 0;
  std::vector<uint64_t> counts;
};
CountCache g_count_cache;

// Per-device rings of buffers (device and pinned host) for a generation's
// instance list and running costs, grown on demand and kept until the
// process ends.  A call takes the next buffer of its device's ring and waits
// first for the launch that used it last, so that up to kListRing
// asynchronous calls per device can be in flight.
constexpr int kListRing = 4;
struct ListBuf {
  void* dev = nullptr;   // device copy
  void* host = nullptr;  // pinned staging
  uint64_t bytes = 0;
  hipEvent_t done = nullptr;  // recorded after the launch that used the buffer last
  bool pending = false;
};
struct Lists {
  ListBuf buf[kListRing];
  int next = 0;
  uint64_t largest = 0;  // the largest buffer of the ring so far
};
std::mutex g_lists_mu;
std::map<int, Lists> g_lists;

int counts_cached(rmat_table_t t, uint64_t seed, uint64_t m, int tbits, uint32_t row_begin, uint32_t row_end,
                  uint64_t* counts);
}  // namespace

extern "C" {

static int rmat_partition_counts_body(rmat_table_t t, uint64_t seed, uint64_t m, int tile_bits, uint32_t row_begin,
                                      uint32_t row_end, uint64_t* counts) {
  rmat::clear_error();
  if (!t || !counts) return set_error(RMAT_EINVAL, "NULL table or counts");
  if (int rc0 = rmat::finalize_table(t)) return rc0;
  const rmat_info& info = *rmat::table_info_of(t);
  int rc = check_args(info, m, tile_bits, row_begin, row_end);
  if (rc) return rc;
  std::memset(counts, 0, sizeof(uint64_t) * (static_cast<uint64_t>(row_end - row_begin) << tile_bits));
  Counter C;
  std::memcpy(C.q, rmat::table_params_of(t), sizeof(C.q));
  C.seed = seed;
  C.t = tile_bits;
  C.row_begin = row_begin;
  C.row_end = row_end;
  C.counts = counts;
  try {
    C.run(m);
  } catch (const std::bad_alloc&) {
    return set_error(RMAT_ENOMEM, "host allocation while counting");
  }
  std::lock_guard<std::mutex> lock(g_count_cache.mu);
  g_count_cache.valid = false;
  try {
    g_count_cache.counts.assign(counts, counts + (static_cast<uint64_t>(row_end - row_begin) << tile_bits));
  } catch (const std::bad_alloc&) {
    return RMAT_OK;  // the counts are in `counts`; only the cache for the next generation is lost
  }
  g_count_cache.valid = true;
  std::memcpy(g_count_cache.q, C.q, sizeof(C.q));
  g_count_cache.seed = seed;
  g_count_cache.m = m;
  g_count_cache.tbits = tile_bits;
  g_count_cache.row_begin = row_begin;
  g_count_cache.row_end = row_end;
  return RMAT_OK;
}

int rmat_partition_counts(rmat_table_t t, uint64_t seed, uint64_t m, int tile_bits, uint32_t row_begin,
                          uint32_t row_end, uint64_t* counts) {
  RMAT_GUARD("rmat_partition_counts", rmat_partition_counts_body(t, seed, m, tile_bits, row_begin, row_end, counts));
}

static int rmat_generate_partition_body(rmat_table_t t, uint64_t seed, uint64_t m, int tile_bits, uint32_t row_begin,
                                        uint32_t row_end, void* out_src, void* out_dst, uint64_t n_out,
                                        hipStream_t stream, bool sync) {
  rmat::clear_error();
  if (!t) return set_error(RMAT_EINVAL, "NULL table");
  if (int rc0 = rmat::finalize_table(t)) return rc0;
  const rmat_info& info = *rmat::table_info_of(t);
  int rc = check_args(info, m, tile_bits, row_begin, row_end);
  if (rc) return rc;
  const uint64_t n_tiles = static_cast<uint64_t>(row_end - row_begin) << tile_bits;
  std::vector<uint64_t> counts(n_tiles);
  if ((rc = counts_cached(t, seed, m, tile_bits, row_begin, row_end, counts.data()))) return rc;
  uint64_t total = 0;
  for (uint64_t x : counts) total += x;
  if (total != n_out)
    return set_error(RMAT_EINVAL, "the tiles hold %llu edges, the outputs %llu", (unsigned long long)total,
                     (unsigned long long)n_out);
  if (total == 0) return RMAT_OK;
  if (!out_src || !out_dst) return set_error(RMAT_EINVAL, "NULL output pointer");
  const uintptr_t idb = info.id_bytes;
  if ((reinterpret_cast<uintptr_t>(out_src) | reinterpret_cast<uintptr_t>(out_dst)) % idb)
    return set_error(RMAT_EINVAL, "output pointers must be %u-byte aligned", (unsigned)idb);
  // one instance per non-empty tile, outputs back to back in row-major
  // order, and the running cost before each (kInstCost blocks per instance
  // for its setup, partial tiles and drains, plus its blocks): the generation
  // launch cuts that line into one equal part per wave, so that a run of
  // tiny tiles is not one wave's alone.  Both arrays are written straight
  // into pinned memory and sent in one copy.
  constexpr uint32_t kInstCost = 4;
  const rmat::TableView& V = *rmat::table_view_of(t);
  const int kk = info.k - tile_bits;
  uint64_t n_inst = 0;
  for (uint64_t i = 0; i < n_tiles; ++i) n_inst += counts[i] != 0;
  const uint64_t inst_bytes = (n_inst * sizeof(rmat::GenInst) + 255) / 256 * 256;
  const uint64_t bytes = inst_bytes + (n_inst + 1) * sizeof(uint64_t);
  // the next buffer of the device's ring, once its last launch is done
  std::lock_guard<std::mutex> lock(g_lists_mu);
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return rmat::hip_fail(e, "hipGetDevice");
  Lists& ring = g_lists[device];
  ListBuf& L = ring.buf[ring.next];
  ring.next = (ring.next + 1) % kListRing;
  if (L.pending) {
    e = hipEventSynchronize(L.done);
    if (e != hipSuccess) return rmat::hip_fail(e, "waiting for an earlier partitioned generation");
    L.pending = false;
  }
  if (!L.done) {
    e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      L.done = nullptr;
      return rmat::hip_fail(e, "hipEventCreateWithFlags");
    }
  }
  if (L.bytes < bytes) {
    // grown to at least twice its size and to the ring's largest, so that
    // calls of varying sizes rotating through the ring settle after a few
    // reallocations (each one waits for the device)
    const uint64_t cap = std::max(std::max(bytes, 2 * L.bytes), ring.largest);
    if (L.dev) (void)hipFree(L.dev);
    if (L.host) (void)hipHostFree(L.host);
    L.dev = L.host = nullptr;
    L.bytes = 0;
    e = hipMalloc(&L.dev, cap);
    if (e == hipSuccess) e = hipHostMalloc(&L.host, cap, hipHostMallocDefault);
    if (e != hipSuccess) {
      if (L.dev) (void)hipFree(L.dev);
      L.dev = L.host = nullptr;
      return rmat::hip_fail(e, "allocation of the partition lists");
    }
    L.bytes = cap;
    ring.largest = std::max(ring.largest, cap);
  }
  char* host = static_cast<char*>(L.host);
  auto* h_inst = reinterpret_cast<rmat::GenInst*>(host);
  auto* h_cum = reinterpret_cast<uint64_t*>(host + inst_bytes);
  uint64_t ii = 0, off = 0, blocks = 0, cost = 0;
  for (uint64_t i = 0; i < n_tiles; ++i) {
    const uint64_t n = counts[i];
    if (n == 0) continue;
    const uint32_t r = row_begin + static_cast<uint32_t>(i >> tile_bits);
    const uint32_t c = static_cast<uint32_t>(i & ((1u << tile_bits) - 1));
    rmat::GenInst I{};  // zero, one first-pass counter block
    I.records = V.records;
    I.n_buckets = static_cast<uint32_t>(info.n_buckets);
    I.table_mask = 0;
    I.bmask = ((1u << info.bucket_bits) - 1u) << 4;
    I.k = static_cast<uint32_t>(kk);
    I.key0 = static_cast<uint32_t>(seed);
    I.key1 = static_cast<uint32_t>(seed >> 32);
    I.edge_begin = 0;
    I.m = n;
    I.first_block = 0;
    I.n_blocks = (n + 63) / 64;
    I.out_src = static_cast<char*>(out_src) + off * idb;
    I.out_dst = static_cast<char*>(out_dst) + off * idb;
    I.digest = nullptr;
    I.ctr3 = 1u + ((r << tile_bits) | c);
    I.kron_k = 2;
    I.src_prefix = static_cast<uint64_t>(r) << kk;
    I.dst_prefix = static_cast<uint64_t>(c) << kk;
    I.epi = 0;
    off += n;
    h_cum[ii] = cost;
    cost += kInstCost + I.n_blocks;
    blocks += I.n_blocks;
    h_inst[ii++] = I;
  }
  h_cum[n_inst] = cost;
  char* base = static_cast<char*>(L.dev);
  e = hipMemcpyAsync(base, host, bytes, hipMemcpyHostToDevice, stream);
  const bool copying = e == hipSuccess;  // the buffer is in use from here on, whatever follows
  if (e == hipSuccess) {
    rmat::TilesArgs a;
    a.insts = reinterpret_cast<const rmat::GenInst*>(base);
    a.cum_cost = reinterpret_cast<const uint64_t*>(base + inst_bytes);
    a.n_inst = static_cast<uint32_t>(n_inst);
    a.inst_cost = kInstCost;
    a.total_blocks = blocks;
    a.n_buckets = static_cast<uint32_t>(info.n_buckets);
    a.wide = info.k > 32;
    a.lds = info.lds_resident != 0;
    e = rmat::launch_generate_tiles(a, stream);
  }
  if (copying) {  // the next user of this buffer waits for the copy (and the launch, if any)
    const hipError_t r = hipEventRecord(L.done, stream);
    if (r == hipSuccess) {
      L.pending = true;
    } else {  // no event to wait for: let the copy finish before the buffer can be reused
      (void)hipStreamSynchronize(stream);
      if (e == hipSuccess) e = r;
    }
  }
  if (e == hipSuccess && sync) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return rmat::hip_fail(e, "partitioned generation");
  return RMAT_OK;
}

int rmat_generate_partition(rmat_table_t t, uint64_t seed, uint64_t m, int tile_bits, uint32_t row_begin,
                            uint32_t row_end, void* out_src, void* out_dst, uint64_t n_out) {
  RMAT_GUARD("rmat_generate_partition", rmat_generate_partition_body(t, seed, m, tile_bits, row_begin, row_end,
                                                                     out_src, out_dst, n_out, nullptr, true));
}

int rmat_generate_partition_async(rmat_table_t t, uint64_t seed, uint64_t m, int tile_bits, uint32_t row_begin,
                                  uint32_t row_end, void* out_src, void* out_dst, uint64_t n_out, void* stream) {
  RMAT_GUARD("rmat_generate_partition_async",
             rmat_generate_partition_body(t, seed, m, tile_bits, row_begin, row_end, out_src, out_dst, n_out,
                                          static_cast<hipStream_t>(stream), false));
}

}  // extern "C"

namespace {
// Counts from the cache when the last count had the same key, else counted
// afresh (the arguments were checked by the caller).
int counts_cached(rmat_table_t t, uint64_t seed, uint64_t m, int tbits, uint32_t row_begin, uint32_t row_end,
                  uint64_t* counts) {
  {
    std::lock_guard<std::mutex> lock(g_count_cache.mu);
    const CountCache& c = g_count_cache;
    if (c.valid && std::memcmp(c.q, rmat::table_params_of(t), sizeof(c.q)) == 0 && c.seed == seed && c.m == m &&
        c.tbits == tbits && c.row_begin == row_begin && c.row_end == row_end) {
      std::memcpy(counts, c.counts.data(), c.counts.size() * sizeof(uint64_t));
      return RMAT_OK;
    }
  }
  return rmat_partition_counts(t, seed, m, tbits, row_begin, row_end, counts);
}
}  // namespace
