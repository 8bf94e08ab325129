// serve.cpp -- the continuous-batching request server of include/rmat_serve.h.
//
// Host side only: admission, the table cache, the output arena and the round
// scheduler.  Device work goes through the same launchers as the batch API
// (one table-build launch and persistent generation launches per round), so
// a served request produces exactly the edges of a plain launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rmat.h"
#include "rmat_internal.h"
#include "rmat_serve.h"

namespace {

using rmat::set_error;

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// First-fit allocator over one device allocation.  Free ranges are kept by
// offset and merged with their neighbours on release.
class Arena {
 public:
  void init(char* base, uint64_t size) {
    base_ = base;
    free_.clear();
    free_[0] = size;
    used_ = peak_ = 0;
  }
  char* alloc(uint64_t bytes) {
    bytes = align_up(std::max<uint64_t>(bytes, 1), kAlign);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const uint64_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return base_ + off;
    }
    return nullptr;
  }
  void release(char* p, uint64_t bytes) {
    bytes = align_up(std::max<uint64_t>(bytes, 1), kAlign);
    uint64_t start = static_cast<uint64_t>(p - base_), len = bytes;
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
    used_ -= bytes;
  }
  uint64_t used() const { return used_; }
  uint64_t peak() const { return peak_; }

 private:
  static constexpr uint64_t kAlign = 256;
  char* base_ = nullptr;
  std::map<uint64_t, uint64_t> free_;
  uint64_t used_ = 0, peak_ = 0;
};

struct TableKey {
  uint64_t q[4];
  int32_t k, mode;
  uint64_t bound;
  bool operator==(const TableKey& o) const {
    return std::memcmp(q, o.q, sizeof(q)) == 0 && k == o.k && mode == o.mode && bound == o.bound;
  }
};

struct TableKeyHash {
  size_t operator()(const TableKey& x) const {
    uint64_t h = 0x9E3779B97F4A7C15ull;
    auto mix = [&h](uint64_t v) {
      h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    };
    for (uint64_t v : x.q) mix(v);
    mix(static_cast<uint64_t>(static_cast<uint32_t>(x.k)) << 32 | static_cast<uint32_t>(x.mode));
    mix(x.bound);
    return static_cast<size_t>(h);
  }
};

struct Slot {
  TableKey key;
  bool valid = false;     // holds (or is building) the table of `key`
  int32_t error = 0;      // build status, known once its round retired
  uint32_t refs = 0;      // active requests using it
  bool in_lru = false;
  std::list<uint32_t>::iterator lru_it;
  rmat::Shape shape;
  rmat::TableView view;
};

struct Req {
  uint64_t ticket;
  rmat_request r;
  rmat::Shape shape;
  double t_submit = 0, t_admit = 0;
  uint32_t slot = 0;
  bool hit = false;
  char* arena = nullptr;
  uint64_t arena_bytes = 0;
  void* out_src = nullptr;
  void* out_dst = nullptr;
  uint64_t n_blocks = 0, next_block = 0;
  uint64_t last_round = 0;
  uint64_t digest = 0;
  int wide = 0, lds = 0;
};

// One launch round: its packet (device copy and pinned host mirror) and what
// the host needs to finish it.  Packet layout, 256-byte aligned parts:
//   [counters: 4 x 256 B][digests][build stats][instances][work items][build jobs]
// Everything is uploaded with one copy; digests and build stats come back
// with one copy.
struct Round {
  uint64_t id = 0;
  bool busy = false;
  hipEvent_t done = nullptr;
  char* h = nullptr;
  char* d = nullptr;
  uint64_t off_dig = 0, off_stats = 0;
  std::vector<Req*> inst_req;
  std::vector<uint32_t> build_slot;
};

constexpr int kGroups = 4;  // (wide, lds)
constexpr uint64_t kCounterBytes = 256;

}  // namespace

struct rmat_server {
  rmat_server_config cfg;
  std::chrono::steady_clock::time_point t0;
  hipStream_t stream = nullptr;
  // device memory
  void* d_arena = nullptr;
  void* d_tables = nullptr;
  void* d_scratch = nullptr;
  void* d_packets = nullptr;
  void* h_packets = nullptr;
  uint64_t device_bytes = 0;
  uint64_t slot_bytes = 0, scratch_slot = 0, packet_bytes = 0;
  uint32_t lds_limit = 0;
  Arena arena;
  // tables
  std::vector<Slot> slots;
  std::unordered_map<TableKey, uint32_t, TableKeyHash> index;
  std::list<uint32_t> lru;         // valid slots with refs == 0, least recent first
  std::vector<uint32_t> free_slots;
  // requests
  uint64_t next_ticket = 1;
  std::deque<Req*> pending;
  std::vector<Req*> active;        // round-robin order
  size_t rr = 0;
  std::deque<rmat_completion> completions;
  std::unordered_map<uint64_t, std::pair<char*, uint64_t>> delivered;  // ticket -> arena outputs
  // rounds
  std::vector<Round> rounds;
  uint64_t next_round = 1;
  std::deque<uint32_t> inflight;   // round indices, oldest first
  rmat_server_stats st;
  int sticky = RMAT_OK;            // a device error ends the server
};

namespace {

double now(const rmat_server* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

void destroy(rmat_server* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (Round& r : s->rounds)
    if (r.done) (void)hipEventDestroy(r.done);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->d_arena) (void)hipFree(s->d_arena);
  if (s->d_tables) (void)hipFree(s->d_tables);
  if (s->d_scratch) (void)hipFree(s->d_scratch);
  if (s->d_packets) (void)hipFree(s->d_packets);
  if (s->h_packets) (void)hipHostFree(s->h_packets);
  for (Req* q : s->pending) delete q;
  for (Req* q : s->active) delete q;
  delete s;
}

uint64_t packet_capacity(const rmat_server_config& c) {
  const uint64_t n_inst = c.max_active, n_build = c.max_builds;
  const uint64_t n_items = c.tick_blocks / c.work_blocks + n_inst + kGroups;
  return kCounterBytes * kGroups + align_up(n_inst * 8, 256) + align_up(n_build * sizeof(rmat::BuildStats), 256) +
         align_up(n_inst * sizeof(rmat::GenInst), 256) + align_up(n_items * sizeof(rmat::GenWorkItem), 256) +
         align_up(n_build * sizeof(rmat::BuildJob), 256);
}

int validate_request(const rmat_server* s, const rmat_request& r, rmat::Shape* S) {
  const double q[4] = {r.a, r.b, r.c, r.d};
  int rc = rmat::validate_and_size(q, r.k, r.table_bound, r.path_mode, S);
  if (rc) return rc;
  if (r.table_bound > s->cfg.max_table_bound)
    return set_error(RMAT_EINVAL, "table_bound %llu exceeds the server's max_table_bound %llu",
                     (unsigned long long)r.table_bound, (unsigned long long)s->cfg.max_table_bound);
  if (rmat::table_bytes(*S) > s->slot_bytes || rmat::scratch_bytes(*S) > s->scratch_slot)
    return set_error(RMAT_EINVAL, "table larger than a cache slot");
  if (r.m > 0 && r.edge_begin + (r.m - 1) < r.edge_begin)
    return set_error(RMAT_ERANGE, "edge_begin + m exceeds 2^64");
  if ((r.out_src == nullptr) != (r.out_dst == nullptr))
    return set_error(RMAT_EINVAL, "give both out_src and out_dst, or neither (arena outputs)");
  const uint64_t idb = r.k <= 32 ? 4 : 8;
  if (r.out_src && ((reinterpret_cast<uintptr_t>(r.out_src) | reinterpret_cast<uintptr_t>(r.out_dst)) % idb))
    return set_error(RMAT_EINVAL, "output pointers must be %u-byte aligned", (unsigned)idb);
  if (!r.out_src && r.m > 0 && 2 * align_up(r.m * idb, 256) > s->cfg.hbm_budget_bytes)
    return set_error(RMAT_EINVAL, "outputs of %llu edges exceed the whole arena", (unsigned long long)r.m);
  if (r.flags & ~static_cast<uint32_t>(RMAT_REQ_DIGEST | RMAT_REQ_DISCARD | RMAT_REQ_UNDIRECTED | RMAT_REQ_SCRAMBLE))
    return set_error(RMAT_EINVAL, "unknown request flags 0x%x", r.flags);
  return RMAT_OK;
}

void complete(rmat_server* s, Req* q, int32_t status) {
  rmat_completion c;
  std::memset(&c, 0, sizeof(c));
  c.ticket = q->ticket;
  c.status = status;
  c.table_hit = q->hit ? 1u : 0u;
  c.t_submit = q->t_submit;
  c.t_admit = q->t_admit;
  c.t_done = now(s);
  c.digest = (status == RMAT_OK && (q->r.flags & RMAT_REQ_DIGEST)) ? q->digest : 0;
  if (q->r.m > 0) {
    Slot& sl = s->slots[q->slot];
    if (--sl.refs == 0) {
      if (sl.valid) {
        s->lru.push_back(q->slot);
        sl.lru_it = std::prev(s->lru.end());
        sl.in_lru = true;
      } else {
        s->free_slots.push_back(q->slot);  // a failed build: the slot holds nothing
      }
    }
  }
  if (q->arena) {
    if ((q->r.flags & RMAT_REQ_DISCARD) || status != RMAT_OK) {  // nothing to deliver
      s->arena.release(q->arena, q->arena_bytes);
    } else {
      s->delivered[q->ticket] = {q->arena, q->arena_bytes};
      c.out_src = q->out_src;
      c.out_dst = q->out_dst;
    }
  } else {
    c.out_src = q->out_src;
    c.out_dst = q->out_dst;
  }
  s->completions.push_back(c);
  ++s->st.completed;
  if (status != RMAT_OK)
    ++s->st.failed;
  else
    s->st.edges_done += q->r.m;
  delete q;
}

// Takes a request out of the round-robin order; the cursor keeps pointing at
// the same next request (and never past the end).
void remove_active(rmat_server* s, Req* q) {
  const auto it = std::find(s->active.begin(), s->active.end(), q);
  if (it == s->active.end()) return;
  const size_t idx = static_cast<size_t>(it - s->active.begin());
  s->active.erase(it);
  if (idx < s->rr) --s->rr;
  if (s->rr >= s->active.size()) s->rr = 0;
}

// Retires finished rounds, oldest first.
int retire(rmat_server* s) {
  while (!s->inflight.empty()) {
    Round& R = s->rounds[s->inflight.front()];
    const hipError_t e = hipEventQuery(R.done);
    if (e == hipErrorNotReady) return RMAT_OK;
    if (e != hipSuccess) return s->sticky = rmat::hip_fail(e, "served round");
    const auto* dig = reinterpret_cast<const uint64_t*>(R.h + R.off_dig);
    const auto* bst = reinterpret_cast<const rmat::BuildStats*>(R.h + R.off_stats);
    for (size_t j = 0; j < R.build_slot.size(); ++j) {
      Slot& sl = s->slots[R.build_slot[j]];
      sl.error = bst[j].error;
      if (sl.error != 0 && sl.valid) {  // never reuse a failed table
        s->index.erase(sl.key);
        sl.valid = false;
      }
    }
    for (size_t i = 0; i < R.inst_req.size(); ++i) R.inst_req[i]->digest ^= dig[i];
    auto status_of = [](int32_t err) {
      return err == 0 ? RMAT_OK : (err == rmat::kBuildResidual ? RMAT_EINVAL : RMAT_EDEVICE);
    };
    for (size_t i = 0; i < R.inst_req.size(); ++i) {
      Req* q = R.inst_req[i];
      if (q->last_round != R.id || q->next_block != q->n_blocks) continue;
      const int32_t err = s->slots[q->slot].error;
      remove_active(s, q);
      complete(s, q, status_of(err));
    }
    // A request whose table failed to build gets no further blocks.  It
    // completes now unless a round still in flight holds some of its blocks
    // (round ids grow, so that is a last_round above this round's); such a
    // request completes when that round retires, by the loop above.
    for (size_t i = 0; i < s->active.size();) {
      Req* q = s->active[i];
      const int32_t err = s->slots[q->slot].error;
      if (err == 0) {
        ++i;
        continue;
      }
      q->next_block = q->n_blocks;
      if (q->last_round > R.id) {
        ++i;
        continue;
      }
      remove_active(s, q);
      complete(s, q, status_of(err));
    }
    R.busy = false;
    R.inst_req.clear();
    R.build_slot.clear();
    s->inflight.pop_front();
  }
  return RMAT_OK;
}

// A slot for a new table: a never-used one, else the least recently used
// idle one.  UINT32_MAX if every slot is held by an active request.
uint32_t take_slot(rmat_server* s) {
  if (!s->free_slots.empty()) {
    const uint32_t i = s->free_slots.back();
    s->free_slots.pop_back();
    return i;
  }
  if (s->lru.empty()) return UINT32_MAX;
  const uint32_t i = s->lru.front();
  s->lru.pop_front();
  Slot& sl = s->slots[i];
  sl.in_lru = false;
  s->index.erase(sl.key);
  sl.valid = false;
  return i;
}

// Forms and launches one round.  Returns RMAT_OK (also when there was nothing to launch).
int issue_round(rmat_server* s, bool* launched) {
  *launched = false;
  uint32_t ri = 0;
  while (ri < s->rounds.size() && s->rounds[ri].busy) ++ri;
  if (ri == s->rounds.size()) return RMAT_OK;
  Round& R = s->rounds[ri];
  const rmat_server_config& c = s->cfg;

  // admission, FIFO
  std::vector<rmat::BuildJob> jobs;
  std::vector<Req*> admitted;
  while (!s->pending.empty() && s->active.size() + admitted.size() < c.max_active && jobs.size() < c.max_builds) {
    Req* q = s->pending.front();
    const rmat_request& r = q->r;
    if (r.m == 0) {  // nothing to generate, no table needed
      s->pending.pop_front();
      q->t_admit = now(s);
      ++s->st.admitted;
      complete(s, q, RMAT_OK);
      continue;
    }
    const uint64_t idb = r.k <= 32 ? 4 : 8;
    const uint64_t half = align_up(r.m * idb, 256);
    char* out = nullptr;
    if (!r.out_src) {
      out = s->arena.alloc(2 * half);
      if (!out) break;  // wait for outputs to be released
    }
    TableKey key;
    std::memcpy(&key.q[0], &r.a, 8);
    std::memcpy(&key.q[1], &r.b, 8);
    std::memcpy(&key.q[2], &r.c, 8);
    std::memcpy(&key.q[3], &r.d, 8);
    key.k = r.k;
    key.mode = r.path_mode;
    key.bound = r.table_bound;
    uint32_t slot;
    bool hit = false;
    auto it = s->index.find(key);
    if (it != s->index.end()) {
      slot = it->second;
      hit = true;
    } else {
      slot = take_slot(s);
      if (slot == UINT32_MAX) {
        if (out) s->arena.release(out, 2 * half);
        break;  // every slot is in use
      }
      Slot& sl = s->slots[slot];
      sl.key = key;
      sl.valid = true;
      sl.error = 0;
      sl.shape = q->shape;
      sl.view = rmat::place_table(static_cast<char*>(s->d_tables) + slot * s->slot_bytes, q->shape);
      s->index[key] = slot;
      rmat::BuildJob job;
      const double qq[4] = {r.a, r.b, r.c, r.d};
      rmat::fill_job(&job, qq, r.k, r.path_mode, q->shape, sl.view,
                     static_cast<char*>(s->d_scratch) + jobs.size() * s->scratch_slot);
      jobs.push_back(job);
      R.build_slot.push_back(slot);
      ++s->st.table_builds;
    }
    Slot& sl = s->slots[slot];
    if (sl.in_lru) {
      s->lru.erase(sl.lru_it);
      sl.in_lru = false;
    }
    ++sl.refs;
    if (hit) ++s->st.table_hits;
    s->pending.pop_front();
    q->slot = slot;
    q->hit = hit;
    q->t_admit = now(s);
    if (out) {
      q->arena = out;
      q->arena_bytes = 2 * half;
      q->out_src = out;
      q->out_dst = out + half;
    } else {
      q->out_src = r.out_src;
      q->out_dst = r.out_dst;
    }
    q->n_blocks = ((r.edge_begin + (r.m - 1)) >> 6) - (r.edge_begin >> 6) + 1;
    q->wide = r.k > 32;
    q->lds = q->shape.n_buckets <= s->lds_limit;
    admitted.push_back(q);
    ++s->st.admitted;
  }
  // new requests are served first in this round, then the others in turn
  if (!admitted.empty()) s->active.insert(s->active.begin() + static_cast<long>(s->rr), admitted.begin(), admitted.end());

  // blocks of this round
  std::vector<rmat::GenInst> insts;
  std::vector<rmat::GenWorkItem> items[kGroups];
  uint32_t max_buckets[kGroups] = {0, 0, 0, 0};
  bool digest[kGroups] = {false, false, false, false};
  bool general[kGroups] = {false, false, false, false};
  uint64_t budget = c.tick_blocks;
  const size_t n_act = s->active.size();
  size_t last_served = s->rr;
  for (size_t t = 0; t < n_act && budget > 0; ++t) {
    const size_t pos = (s->rr + t) % n_act;
    Req* q = s->active[pos];
    if (q->next_block == q->n_blocks) continue;
    const uint64_t take = std::min({q->n_blocks - q->next_block, c.request_quantum, budget});
    const uint32_t ti = static_cast<uint32_t>(insts.size());
    const int g = q->wide * 2 + q->lds;
    rmat::GenInst I;
    const Slot& sl = s->slots[q->slot];
    I.records = sl.view.records;
    I.n_buckets = static_cast<uint32_t>(q->shape.n_buckets);
    I.table_mask = 0;
    I.bmask = ((1u << q->shape.bucket_bits) - 1u) << 4;
    I.k = static_cast<uint32_t>(q->r.k);
    I.key0 = static_cast<uint32_t>(q->r.seed);
    I.key1 = static_cast<uint32_t>(q->r.seed >> 32);
    I.edge_begin = q->r.edge_begin;
    I.m = q->r.m;
    I.first_block = q->r.edge_begin >> 6;
    I.n_blocks = q->n_blocks;
    I.out_src = q->out_src;
    I.out_dst = q->out_dst;
    I.digest = nullptr;  // set below once the packet layout is known
    I.ctr3 = 0;
    I.kron_k = 2;
    I.src_prefix = I.dst_prefix = 0;
    I.epi = ((q->r.flags & RMAT_REQ_UNDIRECTED) ? rmat::kEpiUndirected : 0u) |
            ((q->r.flags & RMAT_REQ_SCRAMBLE) ? rmat::kEpiScramble : 0u);
    if (I.epi) rmat::scramble_params(q->r.scramble_key, q->r.k, &I);
    insts.push_back(I);
    R.inst_req.push_back(q);
    for (uint64_t f = 0; f < take; f += c.work_blocks) {
      rmat::GenWorkItem w;
      w.inst = ti;
      w.first = q->next_block + f;
      w.n_blocks = static_cast<uint32_t>(std::min<uint64_t>(c.work_blocks, take - f));
      items[g].push_back(w);
    }
    max_buckets[g] = std::max(max_buckets[g], I.n_buckets);
    if (q->r.flags & RMAT_REQ_DIGEST) digest[g] = true;
    if (q->r.flags & (RMAT_REQ_UNDIRECTED | RMAT_REQ_SCRAMBLE)) general[g] = true;
    q->next_block += take;
    q->last_round = s->next_round;
    budget -= take;
    last_served = pos;
  }
  if (n_act) s->rr = (last_served + 1) % n_act;
  if (jobs.empty() && insts.empty()) return RMAT_OK;

  // packet
  size_t n_items = 0;
  for (auto& v : items) n_items += v.size();
  const uint64_t off_dig = kCounterBytes * kGroups;
  const uint64_t off_stats = off_dig + align_up(insts.size() * 8, 256);
  const uint64_t off_insts = off_stats + align_up(jobs.size() * sizeof(rmat::BuildStats), 256);
  const uint64_t off_items = off_insts + align_up(insts.size() * sizeof(rmat::GenInst), 256);
  const uint64_t off_jobs = off_items + align_up(n_items * sizeof(rmat::GenWorkItem), 256);
  const uint64_t end = off_jobs + jobs.size() * sizeof(rmat::BuildJob);
  if (end > s->packet_bytes) return s->sticky = set_error(RMAT_EDEVICE, "internal: round packet overflow");
  std::memset(R.h, 0, off_insts);  // counters, digests, stats start at zero
  for (size_t i = 0; i < insts.size(); ++i)
    if (R.inst_req[i]->r.flags & RMAT_REQ_DIGEST)
      insts[i].digest = reinterpret_cast<unsigned long long*>(R.d + off_dig + 8 * i);
  if (!insts.empty()) std::memcpy(R.h + off_insts, insts.data(), insts.size() * sizeof(rmat::GenInst));
  uint64_t item_first[kGroups];
  {
    char* p = R.h + off_items;
    uint64_t n = 0;
    for (int g = 0; g < kGroups; ++g) {
      item_first[g] = n;
      if (!items[g].empty())
        std::memcpy(p + n * sizeof(rmat::GenWorkItem), items[g].data(), items[g].size() * sizeof(rmat::GenWorkItem));
      n += items[g].size();
    }
  }
  for (size_t j = 0; j < jobs.size(); ++j) {
    jobs[j].stats = reinterpret_cast<rmat::BuildStats*>(R.d + off_stats) + j;
    jobs[j].reset_counter = nullptr;
  }
  if (!jobs.empty()) std::memcpy(R.h + off_jobs, jobs.data(), jobs.size() * sizeof(rmat::BuildJob));

  hipError_t e = hipMemcpyAsync(R.d, R.h, end, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess && !jobs.empty())
    e = rmat::launch_table_build(reinterpret_cast<rmat::BuildJob*>(R.d + off_jobs), static_cast<int>(jobs.size()),
                                 s->stream);
  for (int g = 0; g < kGroups && e == hipSuccess; ++g) {
    if (items[g].empty()) continue;
    rmat::BatchArgs a;
    a.insts = reinterpret_cast<const rmat::GenInst*>(R.d + off_insts);
    a.items = reinterpret_cast<const rmat::GenWorkItem*>(R.d + off_items) + item_first[g];
    a.n_items = static_cast<uint32_t>(items[g].size());
    a.counter = reinterpret_cast<unsigned int*>(R.d + kCounterBytes * g);
    a.max_buckets = max_buckets[g];
    a.wide = g >> 1;
    a.lds = g & 1;
    a.digest = digest[g] ? 1 : 0;
    a.general = general[g] ? 1 : 0;
    e = rmat::launch_generate_batch(a, s->stream);
  }
  const uint64_t back = off_insts - off_dig;
  if (e == hipSuccess) e = hipMemcpyAsync(R.h + off_dig, R.d + off_dig, back, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipEventRecord(R.done, s->stream);
  if (e != hipSuccess) return s->sticky = rmat::hip_fail(e, "served round launch");
  R.id = s->next_round++;
  R.off_dig = off_dig;
  R.off_stats = off_stats;
  R.busy = true;
  s->inflight.push_back(ri);
  ++s->st.rounds;
  *launched = true;
  return RMAT_OK;
}

int step(rmat_server* s, bool* progressed) {
  *progressed = false;
  if (s->sticky) return s->sticky;
  const size_t before = s->inflight.size();
  int rc = retire(s);
  if (rc) return rc;
  if (s->inflight.size() != before) *progressed = true;
  while (s->inflight.size() < s->cfg.max_inflight) {
    bool launched = false;
    const size_t done_before = s->completions.size();
    if ((rc = issue_round(s, &launched))) return rc;
    if (s->completions.size() != done_before) *progressed = true;  // m = 0 requests
    if (!launched) break;
    *progressed = true;
  }
  return RMAT_OK;
}

bool busy(const rmat_server* s) { return !s->pending.empty() || !s->active.empty() || !s->inflight.empty(); }

}  // namespace

extern "C" {

static int rmat_server_create_body(const rmat_server_config* cfg_in, rmat_server_t* out) {
  rmat::clear_error();
  if (!out) return set_error(RMAT_EINVAL, "out is NULL");
  *out = nullptr;
  rmat_server_config c;
  std::memset(&c, 0, sizeof(c));
  if (cfg_in) c = *cfg_in;
  if (!c.hbm_budget_bytes) c.hbm_budget_bytes = 200000000000ull;
  if (!c.max_table_bound) c.max_table_bound = 8192;
  if (!c.tick_blocks) c.tick_blocks = 1ull << 24;
  if (!c.request_quantum) c.request_quantum = 1ull << 21;
  if (!c.max_active) c.max_active = 256;
  if (!c.table_slots) c.table_slots = std::max<uint32_t>(1024, c.max_active);
  if (!c.work_blocks) c.work_blocks = 2048;
  if (!c.max_inflight) c.max_inflight = 2;
  if (!c.max_builds) c.max_builds = 256;
  if (c.table_slots < c.max_active) return set_error(RMAT_EINVAL, "table_slots must be at least max_active");
  if (c.max_table_bound < 4 || c.max_table_bound > rmat::kMaxBound)
    return set_error(RMAT_EINVAL, "max_table_bound must be in 4..2^24");
  if (c.max_inflight > 8 || c.max_active > 65536 || c.max_builds > 4096 || c.tick_blocks > (1ull << 32))
    return set_error(RMAT_EINVAL, "config value out of range");
  int rc = rmat::check_device();
  if (rc) return rc;
  rmat_server* s = new (std::nothrow) rmat_server();
  if (!s) return set_error(RMAT_ENOMEM, "host allocation of the server failed");
  s->cfg = c;
  s->t0 = std::chrono::steady_clock::now();
  std::memset(&s->st, 0, sizeof(s->st));
  s->lds_limit = rmat::lds_table_limit();
  // slot sizes: the largest tables the bound admits (either path mode, no saturation)
  const double q[4] = {0.25, 0.25, 0.25, 0.25};
  for (int mode = 0; mode < 2; ++mode) {
    rmat::Shape S;
    const uint64_t bound = mode == RMAT_FIXED ? std::max<uint64_t>(4, c.max_table_bound) : std::max<uint64_t>(5, c.max_table_bound);
    if (rmat::validate_and_size(q, 64, bound, mode, &S) != RMAT_OK) continue;
    s->slot_bytes = std::max(s->slot_bytes, align_up(rmat::table_bytes(S), 256));
    s->scratch_slot = std::max(s->scratch_slot, align_up(rmat::scratch_bytes(S), 256));
  }
  rmat::clear_error();
  s->packet_bytes = packet_capacity(c);
  hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&s->d_arena, c.hbm_budget_bytes);
  if (e == hipSuccess) e = hipMalloc(&s->d_tables, s->slot_bytes * c.table_slots);
  if (e == hipSuccess) e = hipMalloc(&s->d_scratch, s->scratch_slot * c.max_builds);
  if (e == hipSuccess) e = hipMalloc(&s->d_packets, s->packet_bytes * c.max_inflight);
  if (e == hipSuccess) e = hipHostMalloc(&s->h_packets, s->packet_bytes * c.max_inflight, hipHostMallocDefault);
  if (e != hipSuccess) {
    destroy(s);
    return e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation ? set_error(RMAT_ENOMEM, "server memory")
                                                                       : rmat::hip_fail(e, "server setup");
  }
  s->device_bytes = c.hbm_budget_bytes + s->slot_bytes * c.table_slots + s->scratch_slot * c.max_builds +
                    s->packet_bytes * c.max_inflight;
  s->arena.init(static_cast<char*>(s->d_arena), c.hbm_budget_bytes);
  s->slots.resize(c.table_slots);
  for (uint32_t i = c.table_slots; i-- > 0;) s->free_slots.push_back(i);
  s->rounds.resize(c.max_inflight);
  for (uint32_t i = 0; i < c.max_inflight; ++i) {
    Round& R = s->rounds[i];
    R.h = static_cast<char*>(s->h_packets) + i * s->packet_bytes;
    R.d = static_cast<char*>(s->d_packets) + i * s->packet_bytes;
    e = hipEventCreateWithFlags(&R.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      destroy(s);
      return rmat::hip_fail(e, "hipEventCreate");
    }
  }
  *out = s;
  return RMAT_OK;
}

int rmat_server_create(const rmat_server_config* cfg_in, rmat_server_t* out) {
  RMAT_GUARD("rmat_server_create", rmat_server_create_body(cfg_in, out));
}

static int rmat_server_submit_body(rmat_server_t s, const rmat_request* r, double t_arrival, uint64_t* ticket) {
  rmat::clear_error();
  if (!s || !r) return set_error(RMAT_EINVAL, "NULL server or request");
  rmat::Shape S;
  int rc = validate_request(s, *r, &S);
  if (rc) return rc;
  Req* q = new (std::nothrow) Req();
  if (!q) return set_error(RMAT_ENOMEM, "host allocation of a request failed");
  q->ticket = s->next_ticket++;
  q->r = *r;
  q->shape = S;
  q->t_submit = t_arrival >= 0 ? t_arrival : now(s);
  s->pending.push_back(q);
  ++s->st.submitted;
  if (ticket) *ticket = q->ticket;
  return RMAT_OK;
}

int rmat_server_submit(rmat_server_t s, const rmat_request* r, double t_arrival, uint64_t* ticket) {
  RMAT_GUARD("rmat_server_submit", rmat_server_submit_body(s, r, t_arrival, ticket));
}

static int rmat_server_step_body(rmat_server_t s, int* is_busy) {
  rmat::clear_error();
  if (!s) return set_error(RMAT_EINVAL, "NULL server");
  bool progressed = false;
  int rc = step(s, &progressed);
  if (is_busy) *is_busy = busy(s) ? 1 : 0;
  return rc;
}

int rmat_server_step(rmat_server_t s, int* is_busy) {
  RMAT_GUARD("rmat_server_step", rmat_server_step_body(s, is_busy));
}

static int rmat_server_drain_body(rmat_server_t s) {
  rmat::clear_error();
  if (!s) return set_error(RMAT_EINVAL, "NULL server");
  while (busy(s)) {
    bool progressed = false;
    int rc = step(s, &progressed);
    if (rc) return rc;
    if (!progressed && !s->inflight.empty()) {
      const hipError_t e = hipEventSynchronize(s->rounds[s->inflight.front()].done);
      if (e != hipSuccess) return s->sticky = rmat::hip_fail(e, "served round");
    } else if (!progressed && s->inflight.empty() && busy(s)) {
      // only delivered outputs that the caller still holds can block admission
      return set_error(RMAT_EINVAL, "%zu waiting requests need arena space held by delivered outputs; release them",
                       s->pending.size());
    }
  }
  return RMAT_OK;
}

int rmat_server_drain(rmat_server_t s) {
  RMAT_GUARD("rmat_server_drain", rmat_server_drain_body(s));
}

int rmat_server_poll(rmat_server_t s, rmat_completion* out, int max, int* n) {
  rmat::clear_error();
  if (!s || !n || (max > 0 && !out)) return set_error(RMAT_EINVAL, "NULL argument");
  int k = 0;
  while (k < max && !s->completions.empty()) {
    out[k++] = s->completions.front();
    s->completions.pop_front();
  }
  *n = k;
  return RMAT_OK;
}

int rmat_server_release(rmat_server_t s, uint64_t ticket) {
  rmat::clear_error();
  if (!s) return set_error(RMAT_EINVAL, "NULL server");
  auto it = s->delivered.find(ticket);
  if (it == s->delivered.end()) return set_error(RMAT_EINVAL, "ticket %llu holds no arena outputs", (unsigned long long)ticket);
  s->arena.release(it->second.first, it->second.second);
  s->delivered.erase(it);
  return RMAT_OK;
}

static int rmat_server_run_trace_body(rmat_server_t s, const rmat_request* reqs, const double* t_arrival, int n,
                                      rmat_completion* out, rmat_progress_fn progress, void* user) {
  rmat::clear_error();
  if (!s || n < 0 || (n > 0 && (!reqs || !t_arrival || !out))) return set_error(RMAT_EINVAL, "NULL argument");
  for (int i = 0; i < n; ++i) {
    rmat::Shape S;
    if (i > 0 && t_arrival[i] < t_arrival[i - 1]) return set_error(RMAT_EINVAL, "arrivals must be ascending");
    int rc = validate_request(s, reqs[i], &S);
    if (rc) {
      char msg[512];
      std::snprintf(msg, sizeof(msg), "request %d: %s", i, rmat_last_error());
      return set_error(rc, "%s", msg);
    }
  }
  if (busy(s) || !s->completions.empty()) return set_error(RMAT_EINVAL, "the server must be idle");
  const double base = now(s);
  std::unordered_map<uint64_t, int> slot_of;
  int next = 0, done = 0;
  double last_report = base;
  while (done < n) {
    if (progress && now(s) - last_report >= 1.0) {
      last_report = now(s);
      progress(user, static_cast<uint64_t>(done), static_cast<uint64_t>(n));
    }
    const double t = now(s) - base;
    while (next < n && t_arrival[next] <= t) {
      uint64_t ticket = 0;
      int rc = rmat_server_submit(s, &reqs[next], base + t_arrival[next], &ticket);
      if (rc) return rc;
      slot_of[ticket] = next++;
    }
    bool progressed = false;
    int rc = step(s, &progressed);
    if (rc) return rc;
    while (!s->completions.empty()) {
      rmat_completion c = s->completions.front();
      s->completions.pop_front();
      const int i = slot_of[c.ticket];
      if (s->delivered.count(c.ticket)) rmat_server_release(s, c.ticket);
      c.t_submit -= base;
      c.t_admit -= base;
      c.t_done -= base;
      out[i] = c;
      ++done;
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  return RMAT_OK;
}

int rmat_server_run_trace(rmat_server_t s, const rmat_request* reqs, const double* t_arrival, int n,
                          rmat_completion* out, rmat_progress_fn progress, void* user) {
  RMAT_GUARD("rmat_server_run_trace", rmat_server_run_trace_body(s, reqs, t_arrival, n, out, progress, user));
}

int rmat_server_get_stats(rmat_server_t s, rmat_server_stats* out) {
  rmat::clear_error();
  if (!s || !out) return set_error(RMAT_EINVAL, "NULL server or stats pointer");
  *out = s->st;
  out->arena_bytes = s->arena.used();
  out->arena_peak = s->arena.peak();
  out->active = static_cast<uint32_t>(s->active.size());
  out->pending = static_cast<uint32_t>(s->pending.size());
  out->device_bytes = s->device_bytes;
  return RMAT_OK;
}

double rmat_server_clock(rmat_server_t s) { return s ? now(s) : 0.0; }

int rmat_server_free(rmat_server_t s) {
  rmat::clear_error();
  destroy(s);
  return RMAT_OK;
}

}  // extern "C"
