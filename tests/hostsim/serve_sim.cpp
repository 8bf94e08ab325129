// Randomised test of the request server's host logic (admission, table
// cache, arena, round scheduling, completion) against the fake device of
// fake_device.cpp.  Every request must complete exactly once, with every
// edge generated exactly once, the digest of its own table and seed, the
// status of its table build, and the arena empty at the end.
//
//   serve_sim <scenarios> <seed>      exit status 0 when every check passes
#include <algorithm>
#include <array>
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <vector>

#include "rmat.h"
#include "rmat_serve.h"
#include "sim_hash.h"

extern "C" {
void sim_seed(uint64_t s, double ready_p);
int sim_failed();
int sim_take_coverage(uint64_t seed, uint64_t m, int partial);
}

namespace {

int g_errors = 0;

#define CHECK(cond, ...)                                        \
  do {                                                          \
    if (!(cond)) {                                              \
      if (g_errors++ < 20) {                                    \
        std::fprintf(stderr, "%s:%d: ", __FILE__, __LINE__);    \
        std::fprintf(stderr, __VA_ARGS__);                      \
        std::fprintf(stderr, "\n");                             \
      }                                                         \
    }                                                           \
  } while (0)

struct Expect {
  rmat_request r;
  uint64_t digest = 0;
  int status = RMAT_OK;
  bool arena = false;
  bool seen = false;
  std::vector<char> caller;  // caller-owned outputs
};

uint64_t expected_digest(const rmat_request& r) {
  const double q[4] = {r.a, r.b, r.c, r.d};
  const uint64_t tag = sim::table_tag(q, r.k, r.path_mode);
  uint64_t x = 0;
  for (uint64_t i = 0; i < r.m; ++i) x ^= sim::edge_word(r.edge_begin + i, r.seed, tag);
  return x;
}

void run_scenario(int sc, std::mt19937_64& rng) {
  auto uni = [&rng](uint64_t lo, uint64_t hi) { return std::uniform_int_distribution<uint64_t>(lo, hi)(rng); };
  sim_seed(rng(), 0.05 + 0.9 * std::uniform_real_distribution<double>(0, 1)(rng));
  rmat_server_config c;
  std::memset(&c, 0, sizeof(c));
  c.hbm_budget_bytes = uni(1, 64) << 16;
  c.max_table_bound = uni(0, 2) == 0 ? 256 : (uni(0, 1) ? 8192 : 1 << 15);
  c.tick_blocks = uni(1, 4096);
  c.request_quantum = uni(1, 600);
  c.max_active = static_cast<uint32_t>(uni(1, 16));
  c.table_slots = c.max_active + static_cast<uint32_t>(uni(0, 6));
  c.work_blocks = static_cast<uint32_t>(uni(1, 70));
  c.max_inflight = static_cast<uint32_t>(uni(1, 4));
  c.max_builds = static_cast<uint32_t>(uni(1, 8));
  rmat_server_t s = nullptr;
  if (rmat_server_create(&c, &s) != RMAT_OK) {
    CHECK(false, "scenario %d: create failed: %s", sc, rmat_last_error());
    return;
  }
  // a small pool of parameter sets, so that tables are shared and evicted
  std::vector<std::array<double, 4>> pool;
  for (int j = 0; j < 5; ++j) {
    double w[4], t = 0;
    for (double& v : w) t += (v = 0.05 + std::uniform_real_distribution<double>(0, 1)(rng));
    pool.push_back({w[0] / t, w[1] / t, w[2] / t, 1.0 - w[0] / t - w[1] / t - w[2] / t});
  }
  pool.push_back({0.125, 0.375, 0.25, 0.25});  // its build fails on the fake device
  const int n = static_cast<int>(uni(1, 120));
  std::map<uint64_t, Expect> want;  // ticket -> expectation
  std::vector<rmat_request> trace;
  uint64_t seed_base = rng() & ~0xFFFFFull;
  for (int i = 0; i < n; ++i) {
    rmat_request r;
    std::memset(&r, 0, sizeof(r));
    const auto& q = pool[uni(0, pool.size() - 1)];
    r.a = q[0], r.b = q[1], r.c = q[2], r.d = q[3];
    r.k = static_cast<int32_t>(uni(0, 3) == 0 ? uni(33, 40) : uni(1, 24));
    const int cap = std::min(r.k, 15);
    if (uni(0, 3) == 0 && cap >= 1) {
      r.path_mode = RMAT_FIXED;
      int l = static_cast<int>(uni(1, std::min(cap, 7)));
      while (l > 1 && (1ull << (2 * l)) > c.max_table_bound) --l;
      r.table_bound = 1ull << (2 * l);
    } else {
      r.path_mode = RMAT_VARIABLE;
      r.table_bound = uni(5, c.max_table_bound);
    }
    r.seed = seed_base + static_cast<uint64_t>(i);
    const uint64_t idb = r.k <= 32 ? 4 : 8;
    const uint64_t m_arena_max = c.hbm_budget_bytes / (2 * idb) > 512 ? c.hbm_budget_bytes / (2 * idb) - 512 : 0;
    r.m = uni(0, 5) == 0 ? 0 : uni(1, std::min<uint64_t>(30000, std::max<uint64_t>(1, m_arena_max)));
    const int eb = static_cast<int>(uni(0, 3));
    r.edge_begin = eb == 0 ? 0 : eb == 1 ? uni(0, 1000) : eb == 2 ? uni(0, 1ull << 40) : ~0ull - r.m - uni(0, 100) + 1;
    r.flags = static_cast<uint32_t>(uni(0, 3));
    Expect x;
    x.r = r;
    x.digest = (r.flags & RMAT_REQ_DIGEST) ? expected_digest(r) : 0;
    const double qq[4] = {r.a, r.b, r.c, r.d};
    x.status = (sim::build_fails(qq) && r.m > 0) ? RMAT_EINVAL : RMAT_OK;
    if (uni(0, 2) == 0 && r.m > 0) {
      x.caller.resize(2 * r.m * idb + 16);
      uintptr_t base = reinterpret_cast<uintptr_t>(x.caller.data());
      base = (base + 7) / 8 * 8;
      r.out_src = reinterpret_cast<void*>(base);
      r.out_dst = reinterpret_cast<void*>(base + r.m * idb);
      x.r = r;
    } else {
      x.arena = r.m > 0;
    }
    if (2 * ((r.m * idb + 255) / 256 * 256) > c.hbm_budget_bytes && !r.out_src) {
      uint64_t t;  // larger than the arena: refused at submission
      CHECK(rmat_server_submit(s, &r, -1.0, &t) == RMAT_EINVAL, "scenario %d: oversized request accepted", sc);
      continue;
    }
    trace.push_back(r);
    want.emplace(static_cast<uint64_t>(trace.size() - 1), std::move(x));
  }
  const int mode = static_cast<int>(uni(0, 2));
  std::map<uint64_t, uint64_t> ticket_to_idx;
  std::vector<uint64_t> to_release;
  int done = 0;
  auto check_completion = [&](const rmat_completion& cpl, uint64_t idx) {
    auto it = want.find(idx);
    CHECK(it != want.end(), "scenario %d: unknown completion", sc);
    if (it == want.end()) return;
    Expect& x = it->second;
    CHECK(!x.seen, "scenario %d: request %" PRIu64 " completed twice", sc, idx);
    x.seen = true;
    ++done;
    CHECK(cpl.status == x.status, "scenario %d: request %" PRIu64 " status %d, want %d", sc, idx, cpl.status,
          x.status);
    const bool failed = x.status != RMAT_OK;  // cut short: no digest, no arena outputs
    CHECK(cpl.digest == (failed ? 0 : x.digest), "scenario %d: request %" PRIu64 " digest", sc, idx);
    CHECK(sim_take_coverage(x.r.seed, x.r.m, failed) == 0, "scenario %d: request %" PRIu64 " coverage (m=%" PRIu64 ")",
          sc, idx, x.r.m);
    CHECK(cpl.t_submit <= cpl.t_admit && cpl.t_admit <= cpl.t_done, "scenario %d: times", sc);
    const bool discard = x.r.flags & RMAT_REQ_DISCARD;
    if (x.arena && !discard && !failed) {
      CHECK(cpl.out_src != nullptr, "scenario %d: arena outputs missing", sc);
    } else if (x.arena) {
      CHECK(cpl.out_src == nullptr, "scenario %d: discarded outputs returned", sc);
    } else if (x.r.m > 0) {
      CHECK(cpl.out_src == x.r.out_src, "scenario %d: caller outputs", sc);
    }
  };
  if (mode == 2) {  // a recorded trace, arrivals a few microseconds apart
    std::vector<double> t(trace.size());
    double now = 0;
    for (double& v : t) v = (now += 2e-6 * static_cast<double>(uni(0, 10)));
    std::vector<rmat_completion> out(trace.size());
    const int rc = rmat_server_run_trace(s, trace.data(), t.data(), static_cast<int>(trace.size()), out.data(),
                                         nullptr, nullptr);
    CHECK(rc == RMAT_OK, "scenario %d: run_trace: %s", sc, rmat_last_error());
    if (rc == RMAT_OK)
      for (size_t i = 0; i < out.size(); ++i) check_completion(out[i], i);
  } else {
    size_t next = 0;
    int guard = 0;
    while (done < static_cast<int>(trace.size()) && guard++ < 10000000) {
      // submit some (all at once in mode 0)
      const size_t k = mode == 0 ? trace.size() : std::min(trace.size(), next + static_cast<size_t>(uni(0, 3)));
      for (; next < k; ++next) {
        uint64_t ticket = 0;
        const int rc = rmat_server_submit(s, &trace[next], -1.0, &ticket);
        CHECK(rc == RMAT_OK, "scenario %d: submit: %s", sc, rmat_last_error());
        ticket_to_idx[ticket] = next;
      }
      int busy = 0;
      CHECK(rmat_server_step(s, &busy) == RMAT_OK, "scenario %d: step: %s", sc, rmat_last_error());
      rmat_completion buf[8];
      int got = 0;
      CHECK(rmat_server_poll(s, buf, static_cast<int>(uni(0, 8)), &got) == RMAT_OK, "poll");
      for (int i = 0; i < got; ++i) {
        check_completion(buf[i], ticket_to_idx[buf[i].ticket]);
        const Expect& x = want[ticket_to_idx[buf[i].ticket]];
        if (x.arena && !(x.r.flags & RMAT_REQ_DISCARD) && x.status == RMAT_OK) to_release.push_back(buf[i].ticket);
      }
      // release delivered outputs late and in random order
      while (!to_release.empty() && uni(0, 2) == 0) {
        const size_t j = uni(0, to_release.size() - 1);
        CHECK(rmat_server_release(s, to_release[j]) == RMAT_OK, "scenario %d: release", sc);
        to_release[j] = to_release.back();
        to_release.pop_back();
      }
      if (next == trace.size() && uni(0, 30) == 0) {
        // drain: it may only stop early while delivered outputs block admission
        const int rc = rmat_server_drain(s);
        rmat_server_stats ds;
        rmat_server_get_stats(s, &ds);
        CHECK(rc == RMAT_OK || (rc == RMAT_EINVAL && ds.active == 0 && ds.pending > 0 && ds.arena_bytes > 0),
              "scenario %d: drain: %s", sc, rmat_last_error());
      }
    }
    CHECK(guard < 10000000, "scenario %d: no progress", sc);
    for (uint64_t t : to_release) CHECK(rmat_server_release(s, t) == RMAT_OK, "scenario %d: late release", sc);
    CHECK(rmat_server_release(s, 0xFFFFFFFFull) == RMAT_EINVAL, "scenario %d: bogus release", sc);
  }
  for (auto& kv : want) CHECK(kv.second.seen, "scenario %d: request %" PRIu64 " never completed", sc, kv.first);
  rmat_server_stats st;
  rmat_server_get_stats(s, &st);
  CHECK(st.arena_bytes == 0, "scenario %d: arena not empty at the end (%" PRIu64 ")", sc, st.arena_bytes);
  CHECK(st.arena_peak <= c.hbm_budget_bytes, "scenario %d: arena over budget", sc);
  CHECK(st.active == 0 && st.pending == 0, "scenario %d: requests left", sc);
  CHECK(st.completed == trace.size(), "scenario %d: completed %" PRIu64 " of %zu", sc, st.completed, trace.size());
  rmat_server_free(s);
}

}  // namespace

int main(int argc, char** argv) {
  const int scenarios = argc > 1 ? std::atoi(argv[1]) : 200;
  std::mt19937_64 rng(argc > 2 ? std::strtoull(argv[2], nullptr, 10) : 7);
  for (int sc = 0; sc < scenarios; ++sc) run_scenario(sc, rng);
  if (sim_failed()) ++g_errors;
  std::printf("%d scenarios, %d errors\n", scenarios, g_errors);
  return g_errors ? 1 : 0;
}
