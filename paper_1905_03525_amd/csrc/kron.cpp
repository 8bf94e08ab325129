// kron.cpp -- tables for K x K stochastic Kronecker initiators (Sec. 3).
//
// The letters are the K^2 cells of the initiator, cell (i, j) being letter
// K i + j (row digit i, column digit j); node ids are k-digit base-K numbers.
// The table is the one of Sec. 2 over K^2 letters: the variable-length set
// grows by expanding the most probable path while |A| + K^2 - 1 < bound
// (ties: probability descending, depth ascending, code ascending; a path's
// probability is 1.0 times P_x n_x times for x = 0, 1, ...), or all paths of
// length l = floor(log_{K^2} bound); paths stop at the depth cap, the
// largest L with K^L <= 2^15 (and at most k).  Weights are rounded to 2^32
// by largest remainders and the alias table comes from one deterministic
// sweep, as for R-MAT.  K = 2 is the R-MAT table and is built by the device
// builder; for K > 2 the table (at most a few thousand paths for LDS) is
// built here on the host and copied to the device in the same layout, its
// bucket records holding row and column digit values instead of bit strings.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <queue>
#include <vector>

#include "rmat.h"
#include "rmat_internal.h"

namespace rmat {
int adopt_table(const rmat_info& info, const double q[4], int kron_K, const TableView& host, void* d_mem,
                rmat_table_t* out);
}  // namespace rmat

namespace {

using rmat::set_error;

struct Node {
  double p;
  uint64_t code;  // base-K^2 digits, root-most most significant
  int depth;
  std::vector<uint8_t> counts;
};

// true if u precedes v: probability descending, depth ascending, code ascending
bool precedes(const Node& u, const Node& v) {
  if (u.p != v.p) return u.p > v.p;
  if (u.depth != v.depth) return u.depth < v.depth;
  return u.code < v.code;
}

double product(const double* P, int letters, const std::vector<uint8_t>& counts) {
  double p = 1.0;
  for (int x = 0; x < letters; ++x)
    for (int i = 0; i < counts[x]; ++i) p = p * P[x];
  return p;
}

int depth_cap(int K, int k) {
  int L = 0;
  uint64_t v = 1;
  while (v * static_cast<uint64_t>(K) <= 32768u) {
    v *= static_cast<uint64_t>(K);
    ++L;
  }
  return std::min(L, k);
}

}  // namespace

static int rmat_kron_build_table_body(const double* P, int K, int k, uint64_t table_bound, int path_mode,
                                      rmat_table_t* out) {
  rmat::clear_error();
  if (!out) return set_error(RMAT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!P) return set_error(RMAT_EINVAL, "NULL initiator");
  if (K < 2 || K > 16) return set_error(RMAT_EINVAL, "K %d outside 2..16", K);
  if (K == 2) return rmat_build_table(P[0], P[1], P[2], P[3], k, table_bound, path_mode, out);
  const int letters = K * K;
  double s = 0.0;
  for (int x = 0; x < letters; ++x) {
    if (!(P[x] >= 0.0) || std::isinf(P[x])) return set_error(RMAT_EINVAL, "initiator entry %d is not >= 0", x);
    s += P[x];
  }
  if (std::fabs(s - 1.0) > 1e-9) return set_error(RMAT_EINVAL, "initiator entries sum to %.17g, not 1", s);
  if (k < 1) return set_error(RMAT_EINVAL, "k must be >= 1");
  {
    long double n = 1.0L;  // K^k <= 2^64
    for (int i = 0; i < k; ++i) n *= K;
    if (n > 18446744073709551616.0L) return set_error(RMAT_EINVAL, "K^k exceeds 2^64");
  }
  if (table_bound > rmat::kMaxBound) return set_error(RMAT_EINVAL, "table_bound above 2^24");
  if (path_mode == RMAT_VARIABLE) {
    if (table_bound < static_cast<uint64_t>(letters) + 1)
      return set_error(RMAT_EINVAL, "VARIABLE needs table_bound >= K^2 + 1");
  } else if (path_mode == RMAT_FIXED) {
    if (table_bound < static_cast<uint64_t>(letters)) return set_error(RMAT_EINVAL, "FIXED needs table_bound >= K^2");
  } else {
    return set_error(RMAT_EINVAL, "unknown path mode %d", path_mode);
  }
  int rc = rmat::check_device();
  if (rc) return rc;
  const int cap = depth_cap(K, k);

  // leaves
  std::vector<Node> leaves;
  if (path_mode == RMAT_FIXED) {
    int ell = 0;
    uint64_t size = 1;
    while (size * static_cast<uint64_t>(letters) <= table_bound) {
      size *= static_cast<uint64_t>(letters);
      ++ell;
    }
    if (ell > cap) return set_error(RMAT_EINVAL, "FIXED length %d exceeds the depth cap %d", ell, cap);
    leaves.resize(size);
    for (uint64_t code = 0; code < size; ++code) {
      Node& v = leaves[code];
      v.code = code;
      v.depth = ell;
      v.counts.assign(letters, 0);
      uint64_t c = code;
      for (int pos = 0; pos < ell; ++pos) {
        v.counts[c % letters]++;
        c /= letters;
      }
      v.p = product(P, letters, v.counts);
    }
  } else {
    auto later = [](const Node& u, const Node& v) { return precedes(v, u); };
    std::priority_queue<Node, std::vector<Node>, decltype(later)> queue(later);
    std::vector<Node> final_leaves;  // at the depth cap, never expanded
    Node root;
    root.p = 1.0;
    root.code = 0;
    root.depth = 0;
    root.counts.assign(letters, 0);
    queue.push(root);
    while (!queue.empty() && queue.size() + final_leaves.size() + (letters - 1) < table_bound) {
      const Node v = queue.top();
      queue.pop();
      for (int x = 0; x < letters; ++x) {
        Node c = v;
        c.code = v.code * letters + x;
        c.depth = v.depth + 1;
        c.counts[x]++;
        c.p = product(P, letters, c.counts);
        if (c.depth < cap)
          queue.push(std::move(c));
        else
          final_leaves.push_back(std::move(c));
      }
    }
    while (!queue.empty()) {
      leaves.push_back(queue.top());
      queue.pop();
    }
    for (Node& v : final_leaves) leaves.push_back(std::move(v));
  }
  const uint64_t n = leaves.size();
  if (n > (1ull << 24)) return set_error(RMAT_EINVAL, "table too large");
  // tree order: by left-aligned code
  std::vector<uint64_t> lac(n);
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t v = leaves[i].code;
    for (int d = leaves[i].depth; d < cap; ++d) v *= letters;
    lac[i] = v;
  }
  std::vector<uint32_t> order(n);
  for (uint64_t i = 0; i < n; ++i) order[i] = static_cast<uint32_t>(i);
  std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return lac[a] < lac[b]; });
  int bits = 0;
  uint64_t nb = 1;
  while (nb < n) {
    nb <<= 1;
    ++bits;
  }
  const uint64_t C = 1ull << (32 - bits);
  std::vector<double> p(nb, 0.0);
  std::vector<uint64_t> w(nb, 0);
  std::vector<uint32_t> len(nb, 0), row(nb, 0), col(nb, 0), thr(nb, 0), alias(nb, 0);
  for (uint64_t j = 0; j < n; ++j) {
    const Node& v = leaves[order[j]];
    p[j] = v.p;
    len[j] = static_cast<uint32_t>(v.depth);
    uint64_t digits[16], code = v.code, r = 0, c = 0;
    for (int pos = 0; pos < v.depth; ++pos) {
      digits[pos] = code % letters;
      code /= letters;
    }
    for (int pos = v.depth - 1; pos >= 0; --pos) {
      r = r * K + digits[pos] / K;
      c = c * K + digits[pos] % K;
    }
    row[j] = static_cast<uint32_t>(r);
    col[j] = static_cast<uint32_t>(c);
  }
  // largest remainders: floors, then one unit to the largest fractional parts (ties: lower index)
  {
    std::vector<std::pair<double, uint32_t>> frac(n);
    uint64_t sum = 0;
    for (uint64_t j = 0; j < n; ++j) {
      const double x = p[j] * 4294967296.0;
      const double fl = std::floor(x);
      w[j] = static_cast<uint64_t>(fl);
      sum += w[j];
      frac[j] = {x - fl, static_cast<uint32_t>(j)};
    }
    if (sum > (1ull << 32) || (1ull << 32) - sum > n) return set_error(RMAT_EDEVICE, "weights do not sum to 2^32");
    std::sort(frac.begin(), frac.end(), [](const std::pair<double, uint32_t>& a, const std::pair<double, uint32_t>& b) {
      return a.first != b.first ? a.first > b.first : a.second < b.second;
    });
    const uint64_t residual = (1ull << 32) - sum;
    for (uint64_t r = 0; r < residual; ++r) ++w[frac[r].second];
  }
  // alias sweep: lights and heavies in index order, the current heavy pays each light's deficit
  {
    std::vector<uint32_t> lights, heavies;
    for (uint64_t i = 0; i < nb; ++i) (w[i] < C ? lights : heavies).push_back(static_cast<uint32_t>(i));
    if (heavies.empty()) return set_error(RMAT_EDEVICE, "alias table without a heavy bucket");
    size_t h = 0;
    uint32_t j = heavies[0];
    int64_t rem = static_cast<int64_t>(w[j]);
    for (uint32_t i : lights) {
      thr[i] = static_cast<uint32_t>(w[i]);
      alias[i] = j;
      rem -= static_cast<int64_t>(C - w[i]);
      while (rem < static_cast<int64_t>(C)) {
        if (++h >= heavies.size()) return set_error(RMAT_EDEVICE, "alias sweep ran out of heavy buckets");
        const uint32_t jn = heavies[h];
        thr[j] = static_cast<uint32_t>(rem);
        alias[j] = jn;
        rem = static_cast<int64_t>(w[jn]) - (static_cast<int64_t>(C) - rem);
        j = jn;
      }
    }
    if (rem != static_cast<int64_t>(C)) return set_error(RMAT_EDEVICE, "alias sweep left mass %lld", (long long)rem);
    thr[j] = static_cast<uint32_t>(C);
    alias[j] = j;
    for (size_t hh = h + 1; hh < heavies.size(); ++hh) {
      const uint32_t jj = heavies[hh];
      if (w[jj] != C) return set_error(RMAT_EDEVICE, "a leftover heavy bucket is not full");
      thr[jj] = static_cast<uint32_t>(C);
      alias[jj] = jj;
    }
  }
  // device copy in the layout of a device-built table
  rmat::Shape S;
  std::memset(&S, 0, sizeof(S));
  S.cap = cap;
  S.bucket_bits = bits;
  S.n_items = n;
  S.n_buckets = nb;
  S.capacity = C;
  std::vector<rmat::BucketRecord> rec(nb);
  rmat::BuildStats st;
  std::memset(&st, 0, sizeof(st));
  st.n_items = static_cast<uint32_t>(n);
  st.min_len = 0xFFFFFFFFu;
  for (uint64_t i = 0; i < nb; ++i) {
    rec[i].thr_abs = static_cast<uint32_t>(i * C + thr[i]);
    rec[i].rows = row[i] | (row[alias[i]] << 16);
    rec[i].cols = col[i] | (col[alias[i]] << 16);
    rec[i].lens = len[i] | (len[alias[i]] << 16);
    if (i < n) {
      st.min_len = std::min(st.min_len, len[i]);
      st.max_len = std::max(st.max_len, len[i]);
    }
    st.sum_wl += w[i] * len[i];
    st.len_mass[len[i] & 15u] += w[i];
  }
  const uint64_t tb = rmat::table_bytes(S);
  void* d_mem = nullptr;
  hipError_t e = hipMalloc(&d_mem, tb);
  if (e != hipSuccess) return rmat::hip_fail(e, "hipMalloc(kron table)");
  const rmat::TableView V = rmat::place_table(static_cast<char*>(d_mem), S);
  struct Part {
    void* dst;
    const void* src;
    size_t bytes;
  } parts[] = {{V.records, rec.data(), nb * sizeof(rmat::BucketRecord)},
               {V.p, p.data(), nb * 8},
               {V.w, w.data(), nb * 8},
               {V.len, len.data(), nb * 4},
               {V.row, row.data(), nb * 4},
               {V.col, col.data(), nb * 4},
               {V.thr, thr.data(), nb * 4},
               {V.alias, alias.data(), nb * 4},
               {V.stats, &st, sizeof(st)}};
  for (const Part& pt : parts) {
    e = hipMemcpy(pt.dst, pt.src, pt.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(d_mem);
      return rmat::hip_fail(e, "kron table upload");
    }
  }
  rmat_info info;
  rmat::fill_info(&info, k, path_mode, table_bound, S, st, tb);
  const double q4[4] = {P[0], P[1], P[2], P[3]};
  rc = rmat::adopt_table(info, q4, K, V, d_mem, out);
  if (rc) (void)hipFree(d_mem);
  return rc;
}

extern "C" int rmat_kron_build_table(const double* P, int K, int k, uint64_t table_bound, int path_mode,
                                     rmat_table_t* out) {
  RMAT_GUARD("rmat_kron_build_table", rmat_kron_build_table_body(P, K, k, table_bound, path_mode, out));
}
