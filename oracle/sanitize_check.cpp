// Host-only driver for a sanitizer build of the oracle (test infrastructure,
// like the rest of oracle/): runs every entry point of mce_oracle.cpp on small
// random graphs and cross-checks the answers, so that AddressSanitizer,
// UndefinedBehaviorSanitizer or ThreadSanitizer see each code path.  Exit
// status 0 when every check agrees; the sanitizers abort on their own errors.
//
//   - Algorithm 1 from the root, ParMCE (Algorithm 4) under every rank with
//     one and with two threads, and brute force (small graphs) report the
//     same clique set (count, hash, materialised sets);
//   - the incremental step (Algorithms 5-8, membership cross-checked) and the
//     decremental reduction (Section 5.3) on random batches keep the state
//     equal to a fresh enumeration of the current graph.

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <set>
#include <utility>
#include <vector>

extern "C" {
typedef struct { uint64_t count, set_hash, nodes; } orc_result;
typedef struct {
  uint64_t n_applied, n_skipped, n_new, n_del, hash_new, hash_del, count, set_hash;
} orc_imce_result;
struct CliqueOut {
  uint64_t cap_cliques, cap_verts;
  uint64_t* off;
  uint32_t* vert;
  uint64_t n_cliques, n_verts;
};
int orc_mce_ttt_root(uint64_t n, const uint64_t* rp, const uint32_t* col, orc_result* res, CliqueOut* out);
int orc_mce_parmce(uint64_t n, const uint64_t* rp, const uint32_t* col, int kind, const uint32_t* verts,
                   uint64_t nverts, int nthreads, orc_result* res, uint64_t* nodes_v, uint64_t* count_v,
                   uint64_t* hash_v, CliqueOut* out, uint64_t* size_hist, uint64_t hist_len);
int orc_mce_brute(uint64_t n, const uint64_t* rp, const uint32_t* col, orc_result* res, CliqueOut* out);
int orc_rank_metric(uint64_t n, const uint64_t* rp, const uint32_t* col, int kind, uint64_t* metric);
int orc_csr_valid(uint64_t n, const uint64_t* rp, const uint32_t* col);
void* orc_imce_create(uint64_t n, const uint64_t* rp, const uint32_t* col, int nthreads);
void orc_imce_destroy(void* h);
int orc_imce_snapshot(void* h, orc_result* res, CliqueOut* out);
int orc_imce_add(void* h, const uint32_t* src, const uint32_t* dst, uint64_t rho, orc_imce_result* res,
                 CliqueOut* new_out, CliqueOut* del_out, int check_form);
int orc_imce_remove(void* h, const uint32_t* src, const uint32_t* dst, uint64_t rho, orc_imce_result* res,
                    CliqueOut* added_out, CliqueOut* removed_out);
}

namespace {

uint64_t rng_state = 0x243F6A8885A308D3ULL;
uint64_t next_u64() {  // xorshift64*
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return rng_state * 0x2545F4914F6CDD1DULL;
}
double next_unit() { return (double)(next_u64() >> 11) / 9007199254740992.0; }

struct Csr {
  uint64_t n = 0;
  std::vector<uint64_t> rp;
  std::vector<uint32_t> col;
};

Csr to_csr(uint64_t n, const std::set<std::pair<uint32_t, uint32_t>>& edges) {
  std::vector<std::vector<uint32_t>> adj(n);
  for (auto& e : edges) {
    adj[e.first].push_back(e.second);
    adj[e.second].push_back(e.first);
  }
  Csr g;
  g.n = n;
  g.rp.assign(n + 1, 0);
  for (uint64_t v = 0; v < n; ++v) {
    std::set<uint32_t> s(adj[v].begin(), adj[v].end());
    g.rp[v + 1] = g.rp[v] + s.size();
    g.col.insert(g.col.end(), s.begin(), s.end());
  }
  return g;
}

std::set<std::pair<uint32_t, uint32_t>> random_edges(uint64_t n, double p) {
  std::set<std::pair<uint32_t, uint32_t>> e;
  for (uint32_t i = 0; i < n; ++i)
    for (uint32_t j = i + 1; j < n; ++j)
      if (next_unit() < p) e.insert({i, j});
  return e;
}

// Materialised clique sets, each clique as a sorted vector.
struct Out {
  std::vector<uint64_t> off;
  std::vector<uint32_t> vert;
  CliqueOut co{};
  // cliques of these graphs have at most 40 vertices
  explicit Out(uint64_t cap) : off(cap + 1), vert(cap * 40) {
    co.cap_cliques = cap;
    co.cap_verts = cap * 40;
    co.off = off.data();
    co.vert = vert.data();
  }
  bool fits() const { return co.n_cliques <= co.cap_cliques && co.n_verts <= co.cap_verts; }
  std::set<std::vector<uint32_t>> sets() const {
    std::set<std::vector<uint32_t>> s;
    if (!fits()) {
      std::fprintf(stderr, "clique output larger than the buffer\n");
      std::exit(2);
    }
    for (uint64_t i = 0; i < co.n_cliques; ++i) s.insert(std::vector<uint32_t>(&vert[off[i]], &vert[off[i + 1]]));
    return s;
  }
};

int failures = 0;
void expect(bool ok, const char* what, uint64_t n) {
  if (!ok) {
    std::fprintf(stderr, "mismatch: %s (n = %llu)\n", what, (unsigned long long)n);
    ++failures;
  }
}

void static_paths(const Csr& g) {
  expect(orc_csr_valid(g.n, g.rp.data(), g.col.data()) == 1, "csr valid", g.n);
  orc_result root{};
  Out oroot(100000);
  orc_mce_ttt_root(g.n, g.rp.data(), g.col.data(), &root, &oroot.co);
  const auto want = oroot.sets();
  expect(want.size() == root.count, "root count vs sets", g.n);
  if (g.n <= 20) {
    orc_result br{};
    Out obr(100000);
    orc_mce_brute(g.n, g.rp.data(), g.col.data(), &br, &obr.co);
    expect(br.count == root.count && br.set_hash == root.set_hash && obr.sets() == want, "brute force", g.n);
  }
  std::vector<uint64_t> metric(g.n + 1);
  for (int kind = 0; kind < 4; ++kind) {
    orc_rank_metric(g.n, g.rp.data(), g.col.data(), kind, metric.data());
    for (int threads = 1; threads <= 2; ++threads) {
      orc_result r{};
      Out o(100000);
      std::vector<uint64_t> nodes(g.n + 1), count(g.n + 1), hash(g.n + 1), hist(16);
      orc_mce_parmce(g.n, g.rp.data(), g.col.data(), kind, nullptr, 0, threads, &r, nodes.data(), count.data(),
                     hash.data(), &o.co, hist.data(), hist.size());
      uint64_t c = 0, h = 0, hc = 0;
      for (uint64_t v = 0; v < g.n; ++v) {
        c += count[v];
        h += hash[v];
      }
      for (uint64_t k : hist) hc += k;
      expect(r.count == root.count && r.set_hash == root.set_hash, "parmce totals", g.n);
      expect(c == r.count && h == r.set_hash && hc == r.count, "parmce per vertex", g.n);
      expect(o.sets() == want, "parmce sets", g.n);
    }
  }
}

void incremental_paths(uint64_t n, double p) {
  auto edges = random_edges(n, p);
  Csr g = to_csr(n, edges);
  void* st = orc_imce_create(g.n, g.rp.data(), g.col.data(), 2);
  for (int step = 0; step < 6; ++step) {
    const bool remove = (step % 3 == 2) && !edges.empty();
    std::vector<uint32_t> src, dst;
    const int rho = 1 + (int)(next_u64() % 6);
    for (int i = 0; i < rho; ++i) {
      if (remove) {
        auto it = edges.begin();
        std::advance(it, next_u64() % edges.size());
        src.push_back(it->first);
        dst.push_back(it->second);
      } else {
        uint32_t a = (uint32_t)(next_u64() % n), b = (uint32_t)(next_u64() % n);
        if (a == b) b = (a + 1) % n;
        src.push_back(a);
        dst.push_back(b);
      }
    }
    orc_imce_result res{};
    Out onew(100000), odel(100000);
    int rc = remove ? orc_imce_remove(st, src.data(), dst.data(), src.size(), &res, &onew.co, &odel.co)
                    : orc_imce_add(st, src.data(), dst.data(), src.size(), &res, &onew.co, &odel.co, 1);
    expect(rc == 0, remove ? "remove rc" : "add rc (membership forms agree)", n);
    for (size_t i = 0; i < src.size(); ++i) {
      auto e = std::make_pair(std::min(src[i], dst[i]), std::max(src[i], dst[i]));
      if (remove)
        edges.erase(e);
      else
        edges.insert(e);
    }
    Csr cur = to_csr(n, edges);
    orc_result fresh{}, snap{};
    Out ofresh(100000), osnap(100000);
    orc_mce_ttt_root(cur.n, cur.rp.data(), cur.col.data(), &fresh, &ofresh.co);
    orc_imce_snapshot(st, &snap, &osnap.co);
    expect(snap.count == fresh.count && snap.set_hash == fresh.set_hash && osnap.sets() == ofresh.sets(),
           "incremental state vs fresh enumeration", n);
  }
  orc_imce_destroy(st);
}

}  // namespace

// argv[1] == "quick": fewer graphs (for the slower thread-sanitizer build).
int main(int argc, char** argv) {
  const bool quick = argc > 1 && std::strcmp(argv[1], "quick") == 0;
  const int n_static = quick ? 6 : 24, n_incr = quick ? 2 : 8;
  for (int i = 0; i < n_static; ++i) {
    const uint64_t n = 1 + next_u64() % 40;
    const double p = 0.1 + 0.8 * next_unit();
    static_paths(to_csr(n, random_edges(n, p)));
  }
  static_paths(to_csr(0, {}));
  for (int i = 0; i < n_incr; ++i) incremental_paths(8 + next_u64() % 24, 0.2 + 0.5 * next_unit());
  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("sanitize_check ok\n");
  return 0;
}
