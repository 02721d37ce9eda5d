// CPU oracle for maximal clique enumeration (MCE) and its incremental update
// (IMCE), after Das, Sanei-Mehri and Tirthapura, "Shared-Memory Parallel
// Maximal Clique Enumeration from Static and Dynamic Graphs".
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library may include, link or
// call this file; only the test suite, the smoke check and the benchmark's CPU
// baseline leg use it.  It is deliberately plain and slow: sets are sorted
// std::vector<uint32_t>, intersections are merges or binary searches, and
// every function follows one passage of the paper (cited at the function).
//
// Readings where the paper leaves a choice open (binding for any
// implementation that wants identical recursion-node counts):
//   * pivot tie-break: among the vertices of cand u fini that maximise
//     |cand n Gamma(u)|, the one with the smallest vertex id;
//   * ext is iterated in ascending vertex id;
//   * a "node" is one invocation of the TTT routine (Algorithm 1), the
//     subproblem root included; dead ends (cand empty, fini not) count;
//     branches skipped by the edge exclusion of Algorithm 8 are not nodes;
//   * rank(v) = (metric(v), id(v)) compared lexicographically (Section 4.2);
//   * clique-set hash: z(v) = mix(v), hc(c) = mix(sum z(v) + |c| * G),
//     H = sum hc(c) (all mod 2^64), mix = the splitmix64 finaliser,
//     G = 0x9E3779B97F4A7C15.
//
// Pins: the clique sets, counts and hashes are pinned by brute force, closed
// forms and the paper's worked examples (see the tests).  Search-node counts
// depend on the tie-break reading above; closed forms pin them only for
// complete graphs (2n - 1 under degree rank), stars (2k + 1 under degree and
// degeneracy rank) and edgeless graphs (n); beyond
// those they are parity unpinned (checked oracle against GPU only).  The
// peel-round metric is pinned by closed forms on paths, cycles and stars, by
// its first round (exactly the vertices of minimum degree), by invariance under
// relabelling, and by the bound of later neighbours by the core number.
//
// Build: g++ -O2 -std=c++17 -shared -fPIC -pthread mce_oracle.cpp -o libmce_oracle.so

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

typedef std::vector<uint32_t> VSet;  // sorted ascending, no repeats

const uint64_t kGolden = 0x9E3779B97F4A7C15ULL;

// splitmix64 output function (Steele, Lea, Flood 2014; Vigna's public-domain
// reference): add the golden gamma, then two xor-shift-multiply rounds.
uint64_t mix64(uint64_t x) {
  x += kGolden;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

uint64_t clique_hash(const uint32_t* v, uint64_t k) {
  uint64_t s = 0;
  for (uint64_t i = 0; i < k; ++i) s += mix64(v[i]);
  return mix64(s + k * kGolden);
}

// |A n B| for sorted sets.
uint64_t inter_size(const uint32_t* a, size_t na, const uint32_t* b, size_t nb) {
  if (na > nb) { std::swap(a, b); std::swap(na, nb); }
  uint64_t c = 0;
  if (na * 16 < nb) {
    for (size_t i = 0; i < na; ++i) c += std::binary_search(b, b + nb, a[i]) ? 1 : 0;
    return c;
  }
  size_t i = 0, j = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j]) ++i;
    else if (a[i] > b[j]) ++j;
    else { ++c; ++i; ++j; }
  }
  return c;
}

VSet intersect(const VSet& a, const uint32_t* b, size_t nb) {
  VSet out;
  size_t na = a.size();
  if (na * 16 < nb) {
    for (uint32_t x : a) if (std::binary_search(b, b + nb, x)) out.push_back(x);
    return out;
  }
  if (nb * 16 < na) {
    for (size_t j = 0; j < nb; ++j) if (std::binary_search(a.begin(), a.end(), b[j])) out.push_back(b[j]);
    return out;
  }
  size_t i = 0, j = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j]) ++i;
    else if (a[i] > b[j]) ++j;
    else { out.push_back(a[i]); ++i; ++j; }
  }
  return out;
}

bool contains(const VSet& s, uint32_t x) { return std::binary_search(s.begin(), s.end(), x); }
void erase_sorted(VSet& s, uint32_t x) {
  auto it = std::lower_bound(s.begin(), s.end(), x);
  if (it != s.end() && *it == x) s.erase(it);
}
void insert_sorted(VSet& s, uint32_t x) {
  auto it = std::lower_bound(s.begin(), s.end(), x);
  if (it == s.end() || *it != x) s.insert(it, x);
}

// Adjacency view: Gamma(u) as a sorted array.
struct Adj {
  std::vector<VSet> rows;
  const VSet& row(uint32_t u) const { return rows[u]; }
  const uint32_t* nb(uint32_t u) const { return rows[u].data(); }
  size_t deg(uint32_t u) const { return rows[u].size(); }
  bool has(uint32_t a, uint32_t b) const { return contains(rows[a], b); }
};

Adj adj_from_csr(uint64_t n, const uint64_t* rp, const uint32_t* col) {
  Adj A;
  A.rows.resize(n);
  for (uint64_t v = 0; v < n; ++v) A.rows[v].assign(col + rp[v], col + rp[v + 1]);
  return A;
}

// The subgraph G_v of Algorithm 4, induced by Gamma(v) u {v}: for u in
// Gamma(v), Gamma_{G_v}(u) = Gamma(u) n Gamma(v) (v itself is in K and is
// never looked up).  Rows are addressed by global id.
struct InducedAdj {
  std::vector<VSet> rows;
  std::unordered_map<uint32_t, uint32_t> slot;
  const VSet& row(uint32_t u) const { return rows[slot.at(u)]; }
};

InducedAdj induced_by_neighbourhood(const Adj& A, uint32_t v) {
  InducedAdj g;
  const VSet& nv = A.rows[v];
  g.rows.reserve(nv.size());
  for (uint32_t u : nv) {
    g.slot[u] = (uint32_t)g.rows.size();
    g.rows.push_back(intersect(nv, A.nb(u), A.deg(u)));
  }
  return g;
}

struct Sink {
  uint64_t count = 0, hash = 0, nodes = 0;
  bool keep = false;
  std::vector<VSet> cliques;
  std::vector<uint64_t> sizes;  // sizes[k] = number of maximal cliques with k vertices (Section 6.1, Figure 5)
  void emit(const std::vector<uint32_t>& K) {
    VSet c = K;
    std::sort(c.begin(), c.end());
    count += 1;
    hash += clique_hash(c.data(), c.size());
    if (sizes.size() <= c.size()) sizes.resize(c.size() + 1, 0);
    sizes[c.size()] += 1;
    if (keep) cliques.push_back(std::move(c));
  }
};

// Edge-exclusion test of Algorithm 8: K_q "meets" the excluded edge set when
// K u {q} contains both endpoints of an excluded edge; K itself never does, so
// only the pairs (q, w), w in K, need checking.
struct Exclusion {
  const std::map<std::pair<uint32_t, uint32_t>, uint64_t>* index = nullptr;  // edge -> position in batch
  uint64_t before = 0;  // exclude edges e_j with j < before
  bool active() const { return index != nullptr; }
  bool hits(const std::vector<uint32_t>& K, uint32_t q) const {
    for (uint32_t w : K) {
      auto key = std::make_pair(std::min(q, w), std::max(q, w));
      auto it = index->find(key);
      if (it != index->end() && it->second < before) return true;
    }
    return false;
  }
};

// Algorithm 1 (TTT), and with `ex` active Algorithm 8 (TTTExcludeEdges):
// report every maximal clique that contains K, uses vertices of cand and none
// of fini.  `G.row(u)` is Gamma(u) in the graph the call is made on.
template <class Graph>
void ttt(const Graph& G, std::vector<uint32_t>& K, VSet cand, VSet fini, Sink& out, const Exclusion& ex) {
  out.nodes += 1;
  if (cand.empty() && fini.empty()) {  // K is maximal
    out.emit(K);
    return;
  }
  if (cand.empty()) return;  // ext = cand - Gamma(pivot) is empty for any pivot
  // pivot: u in cand u fini maximising |cand n Gamma(u)|; ties -> smallest id
  uint32_t pivot = 0;
  int64_t best = -1;
  size_t i = 0, j = 0;
  while (i < cand.size() || j < fini.size()) {
    uint32_t u;
    if (j >= fini.size() || (i < cand.size() && cand[i] < fini[j])) u = cand[i++];
    else u = fini[j++];
    const VSet& r = G.row(u);
    int64_t t = (int64_t)inter_size(cand.data(), cand.size(), r.data(), r.size());
    if (t > best) { best = t; pivot = u; }
  }
  // ext = cand - Gamma(pivot), visited in ascending id
  const VSet& rp = G.row(pivot);
  VSet ext;
  for (uint32_t q : cand) if (!contains(rp, q)) ext.push_back(q);
  for (uint32_t q : ext) {
    if (ex.active() && ex.hits(K, q)) {  // Algorithm 8: skip q, move it to fini
      erase_sorted(cand, q);
      insert_sorted(fini, q);
      continue;
    }
    const VSet& rq = G.row(q);
    VSet cq = intersect(cand, rq.data(), rq.size());
    VSet fq = intersect(fini, rq.data(), rq.size());
    K.push_back(q);
    ttt(G, K, std::move(cq), std::move(fq), out, ex);
    K.pop_back();
    erase_sorted(cand, q);
    insert_sorted(fini, q);
  }
}

// Vertex metric behind the rank functions of Section 4.2.
enum { RANK_DEGREE = 0, RANK_DEGENERACY = 1, RANK_TRIANGLE = 2, RANK_PEEL = 3 };

// Core numbers by Batagelj-Zaversnik bucket peeling: repeatedly remove a vertex
// of minimum remaining degree; its core number is the running maximum of the
// degrees at removal time.
std::vector<uint64_t> core_numbers(const Adj& A) {
  uint64_t n = A.rows.size();
  std::vector<uint64_t> deg(n), core(n, 0);
  uint64_t maxd = 0;
  for (uint64_t v = 0; v < n; ++v) { deg[v] = A.deg(v); maxd = std::max(maxd, deg[v]); }
  std::vector<std::vector<uint32_t>> bucket(maxd + 1);
  for (uint64_t v = 0; v < n; ++v) bucket[deg[v]].push_back((uint32_t)v);
  std::vector<char> removed(n, 0);
  uint64_t k = 0;
  uint64_t done = 0;
  uint64_t d = 0;
  while (done < n) {
    while (d <= maxd && bucket[d].empty()) ++d;
    uint32_t v = bucket[d].back();
    bucket[d].pop_back();
    if (removed[v] || deg[v] != d) continue;  // stale entry
    removed[v] = 1;
    ++done;
    k = std::max(k, d);
    core[v] = k;
    for (uint32_t w : A.rows[v]) {
      if (removed[w]) continue;
      deg[w] -= 1;
      bucket[deg[w]].push_back(w);
      if (deg[w] < d) d = deg[w];
    }
  }
  return core;
}

// t(v) = number of triangles through v = half the number of ordered pairs of
// adjacent neighbours = (1/2) sum_{u in Gamma(v)} |Gamma(u) n Gamma(v)|.
std::vector<uint64_t> triangle_counts(const Adj& A) {
  uint64_t n = A.rows.size();
  std::vector<uint64_t> t(n, 0);
  for (uint64_t v = 0; v < n; ++v) {
    uint64_t s = 0;
    for (uint32_t u : A.rows[v]) s += inter_size(A.nb(u), A.deg(u), A.nb(v), A.deg(v));
    t[v] = s / 2;
  }
  return t;
}

// Peel order: the degeneracy ordering of Eppstein, Loeffler and Strash taken
// in synchronous rounds.  Level k starts at 0.  A round removes, all at once,
// every remaining vertex whose degree in the remaining graph is at most k, and
// the vertex's metric is the index of that round.  A round that would remove
// nothing instead raises k to the smallest remaining degree and is not counted.
// A vertex leaving at level k has at most k neighbours that leave in the same
// round or later, so with rank (round, id) its candidate set is no larger than
// its core number.
std::vector<uint64_t> peel_rounds(const Adj& A) {
  uint64_t n = A.rows.size();
  std::vector<uint64_t> deg(n), round(n, ~0ULL);
  for (uint64_t v = 0; v < n; ++v) deg[v] = A.deg(v);
  uint64_t k = 0, r = 0, left = n;
  while (left > 0) {
    std::vector<uint32_t> out;
    uint64_t mind = ~0ULL;
    for (uint64_t v = 0; v < n; ++v) {
      if (round[v] != ~0ULL) continue;
      if (deg[v] <= k) out.push_back((uint32_t)v);
      else mind = std::min(mind, deg[v]);
    }
    if (out.empty()) {
      k = mind;
      continue;
    }
    for (uint32_t v : out) round[v] = r;
    for (uint32_t v : out)
      for (uint32_t w : A.rows[v])
        if (round[w] == ~0ULL) deg[w] -= 1;
    left -= out.size();
    ++r;
  }
  return round;
}

std::vector<uint64_t> metric_of(const Adj& A, int kind) {
  uint64_t n = A.rows.size();
  if (kind == RANK_DEGENERACY) return core_numbers(A);
  if (kind == RANK_PEEL) return peel_rounds(A);
  if (kind == RANK_TRIANGLE) return triangle_counts(A);
  std::vector<uint64_t> d(n);
  for (uint64_t v = 0; v < n; ++v) d[v] = A.deg(v);
  return d;
}

// rank(w) > rank(v) for rank = (metric, id), lexicographic.
inline bool rank_gt(const std::vector<uint64_t>& m, uint32_t w, uint32_t v) {
  return m[w] > m[v] || (m[w] == m[v] && w > v);
}

// One ParMCE subproblem (Algorithm 4 body): K = {v}, cand = neighbours of
// higher rank, fini = the others; TTT on G_v.  (The per-subproblem solver of
// Algorithm 4 is ParTTT, whose unrolled children are exactly TTT's children,
// so the recursion tree and its node count are TTT's.)
void parmce_vertex(const Adj& A, const std::vector<uint64_t>& metric, uint32_t v, Sink& out) {
  InducedAdj Gv = induced_by_neighbourhood(A, v);
  VSet cand, fini;
  for (uint32_t w : A.rows[v]) {
    if (rank_gt(metric, w, v)) cand.push_back(w);
    else fini.push_back(w);
  }
  std::vector<uint32_t> K{v};
  Exclusion none;
  ttt(Gv, K, std::move(cand), std::move(fini), out, none);
}

struct CliqueOut {
  uint64_t cap_cliques, cap_verts;
  uint64_t* off;
  uint32_t* vert;
  uint64_t n_cliques, n_verts;
};

void write_cliques(const std::vector<VSet>& cl, CliqueOut* out) {
  if (!out) return;
  uint64_t nv = 0;
  for (const VSet& c : cl) nv += c.size();
  out->n_cliques = cl.size();
  out->n_verts = nv;
  if (cl.size() > out->cap_cliques || nv > out->cap_verts || !out->off || !out->vert) return;
  uint64_t o = 0;
  out->off[0] = 0;
  for (size_t i = 0; i < cl.size(); ++i) {
    std::memcpy(out->vert + o, cl[i].data(), cl[i].size() * sizeof(uint32_t));
    o += cl[i].size();
    out->off[i + 1] = o;
  }
}

bool csr_ok(uint64_t n, const uint64_t* rp, const uint32_t* col) {
  if (n && (!rp || rp[0] != 0)) return false;
  for (uint64_t v = 0; v < n; ++v) {
    if (rp[v + 1] < rp[v]) return false;
    for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) {
      if (col[e] >= n || col[e] == v) return false;
      if (e > rp[v] && col[e] <= col[e - 1]) return false;
    }
  }
  // symmetry
  for (uint64_t v = 0; v < n; ++v)
    for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) {
      uint32_t w = col[e];
      if (!std::binary_search(col + rp[w], col + rp[w + 1], (uint32_t)v)) return false;
    }
  return true;
}

bool maximal_in(const Adj& G, const VSet& c) {
  if (c.empty()) return false;
  for (uint32_t w : G.rows[c[0]]) {
    if (contains(c, w)) continue;
    bool all = true;
    for (uint32_t y : c) if (!G.has(w, y)) { all = false; break; }
    if (all) return false;
  }
  return true;
}

// Algorithm 7's splitting: the subsets of c that keep no edge of the batch,
// obtained by splitting, for each batch edge (x, y) inside c, every subset
// holding both ends into one without x and one without y.
std::set<VSet> edge_free_subsets(const VSet& c, const std::map<std::pair<uint32_t, uint32_t>, uint64_t>& index) {
  std::set<VSet> S{c};
  for (size_t x = 0; x < c.size(); ++x)
    for (size_t y = x + 1; y < c.size(); ++y) {
      auto key = std::make_pair(c[x], c[y]);
      if (!index.count(key)) continue;
      std::set<VSet> S2;
      for (const VSet& cp : S) {
        if (contains(cp, key.first) && contains(cp, key.second)) {
          VSet c1 = cp, c2 = cp;
          erase_sorted(c1, key.first);
          erase_sorted(c2, key.second);
          S2.insert(std::move(c1));
          S2.insert(std::move(c2));
        } else {
          S2.insert(cp);
        }
      }
      S.swap(S2);
    }
  return S;
}

// ---------------------------------------------------------------------------
// IMCE state: the graph G and the set C of its maximal cliques (Section 5).
struct ImceState {
  uint64_t n;
  Adj A;
  std::set<VSet> C;
  uint64_t count = 0, hash = 0;
};

}  // namespace

extern "C" {

typedef struct { uint64_t count, set_hash, nodes; } orc_result;
typedef struct {
  uint64_t n_applied, n_skipped, n_new, n_del, hash_new, hash_del, count, set_hash;
} orc_imce_result;

uint64_t orc_mix64(uint64_t x) { return mix64(x); }
uint64_t orc_clique_hash(const uint32_t* v, uint64_t k) { return clique_hash(v, k); }

int orc_csr_valid(uint64_t n, const uint64_t* rp, const uint32_t* col) { return csr_ok(n, rp, col) ? 1 : 0; }

// Per-vertex metric for the rank functions of Section 4.2 (degree, core
// number, triangle count).
int orc_rank_metric(uint64_t n, const uint64_t* rp, const uint32_t* col, int kind, uint64_t* metric) {
  Adj A = adj_from_csr(n, rp, col);
  std::vector<uint64_t> m = metric_of(A, kind);
  if (n) std::memcpy(metric, m.data(), n * sizeof(uint64_t));  // an empty graph has no metric (and m.data() may be null)
  return 0;
}

// Definition path: Algorithm 1 from the root, K = {}, cand = V, fini = {}.
// For n = 0 no clique is reported (there are no per-vertex subproblems).
int orc_mce_ttt_root(uint64_t n, const uint64_t* rp, const uint32_t* col, orc_result* res, CliqueOut* out) {
  Sink s;
  s.keep = out != nullptr;
  if (n > 0) {
    Adj A = adj_from_csr(n, rp, col);
    VSet cand(n);
    for (uint64_t v = 0; v < n; ++v) cand[v] = (uint32_t)v;
    std::vector<uint32_t> K;
    Exclusion none;
    ttt(A, K, std::move(cand), VSet(), s, none);
  }
  res->count = s.count;
  res->set_hash = s.hash;
  res->nodes = s.nodes;
  write_cliques(s.cliques, out);
  return 0;
}

// Decomposed path: Algorithm 4, one subproblem per vertex, solved
// sequentially (optionally by `nthreads` threads that pull vertices from a
// shared counter; sums are commutative so the merge is exact).  `verts`
// restricts the run to a subset of the subproblems (NULL = all n).
//
// `size_hist` (nullable, `hist_len` entries): size_hist[k] = number of maximal
// cliques with k vertices (sizes >= hist_len are added to the last entry), the
// distribution the paper plots per input graph (Section 6.1).
int orc_mce_parmce(uint64_t n, const uint64_t* rp, const uint32_t* col, int kind, const uint32_t* verts,
                   uint64_t nverts, int nthreads, orc_result* res, uint64_t* nodes_v, uint64_t* count_v,
                   uint64_t* hash_v, CliqueOut* out, uint64_t* size_hist, uint64_t hist_len) {
  Adj A = adj_from_csr(n, rp, col);
  std::vector<uint64_t> metric = metric_of(A, kind);
  uint64_t total = verts ? nverts : n;
  if (nthreads < 1) nthreads = 1;
  std::atomic<uint64_t> next(0);
  std::vector<Sink> sinks(nthreads);
  auto work = [&](int t) {
    Sink& s = sinks[t];
    s.keep = out != nullptr;
    for (;;) {
      uint64_t i = next.fetch_add(1);
      if (i >= total) break;
      uint32_t v = verts ? verts[i] : (uint32_t)i;
      uint64_t c0 = s.count, h0 = s.hash, n0 = s.nodes;
      parmce_vertex(A, metric, v, s);
      if (nodes_v) nodes_v[i] = s.nodes - n0;
      if (count_v) count_v[i] = s.count - c0;
      if (hash_v) hash_v[i] = s.hash - h0;
    }
  };
  if (nthreads == 1) {
    work(0);
  } else {
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) th.emplace_back(work, t);
    for (auto& x : th) x.join();
  }
  orc_result r{0, 0, 0};
  std::vector<VSet> all;
  if (size_hist)
    for (uint64_t k = 0; k < hist_len; ++k) size_hist[k] = 0;
  for (Sink& s : sinks) {
    r.count += s.count;
    r.set_hash += s.hash;
    r.nodes += s.nodes;
    if (size_hist && hist_len)
      for (uint64_t k = 0; k < s.sizes.size(); ++k) size_hist[std::min(k, hist_len - 1)] += s.sizes[k];
    if (out) for (auto& c : s.cliques) all.push_back(std::move(c));
  }
  *res = r;
  if (out) {
    std::sort(all.begin(), all.end());
    write_cliques(all, out);
  }
  return 0;
}

// Brute force from the definition (Section 1): every vertex subset S that is a
// clique and that no outside vertex is adjacent to all of.  n <= 24.
int orc_mce_brute(uint64_t n, const uint64_t* rp, const uint32_t* col, orc_result* res, CliqueOut* out) {
  if (n > 24) return -1;
  std::vector<uint32_t> nbmask(n, 0);
  for (uint64_t v = 0; v < n; ++v)
    for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) nbmask[v] |= 1u << col[e];
  Sink s;
  s.keep = out != nullptr;
  for (uint64_t S = 1; S < (1ull << n); ++S) {
    bool clique = true;
    for (uint64_t v = 0; v < n && clique; ++v)
      if ((S >> v) & 1) clique = ((S & ~(1ull << v)) & ~(uint64_t)nbmask[v]) == 0;
    if (!clique) continue;
    bool maximal = true;
    for (uint64_t w = 0; w < n && maximal; ++w)
      if (!((S >> w) & 1) && (S & ~(uint64_t)nbmask[w]) == 0) maximal = false;
    if (!maximal) continue;
    std::vector<uint32_t> K;
    for (uint64_t v = 0; v < n; ++v) if ((S >> v) & 1) K.push_back((uint32_t)v);
    s.emit(K);
  }
  res->count = s.count;
  res->set_hash = s.hash;
  res->nodes = 0;
  write_cliques(s.cliques, out);
  return 0;
}

// ---------------------------------------------------------------------------
// IMCE (Section 5).

void* orc_imce_create(uint64_t n, const uint64_t* rp, const uint32_t* col, int nthreads) {
  ImceState* st = new ImceState();
  st->n = n;
  st->A = adj_from_csr(n, rp, col);
  std::vector<uint64_t> metric = metric_of(st->A, RANK_DEGREE);
  if (nthreads < 1) nthreads = 1;
  std::atomic<uint64_t> next(0);
  std::vector<Sink> sinks(nthreads);
  auto work = [&](int t) {
    Sink& s = sinks[t];
    s.keep = true;
    for (;;) {
      uint64_t v = next.fetch_add(1);
      if (v >= n) break;
      parmce_vertex(st->A, metric, (uint32_t)v, s);
    }
  };
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t) th.emplace_back(work, t);
  for (auto& x : th) x.join();
  for (Sink& s : sinks) {
    st->count += s.count;
    st->hash += s.hash;
    for (auto& c : s.cliques) st->C.insert(std::move(c));
  }
  return st;
}

void orc_imce_destroy(void* h) { delete (ImceState*)h; }

int orc_imce_snapshot(void* h, orc_result* res, CliqueOut* out) {
  ImceState* st = (ImceState*)h;
  res->count = st->count;
  res->set_hash = st->hash;
  res->nodes = 0;
  if (out) {
    std::vector<VSet> all(st->C.begin(), st->C.end());
    write_cliques(all, out);
  }
  return 0;
}

// One batch H of edge additions.  Canonicalisation: every pair must be two
// distinct ids < n (else the whole batch is rejected with -1 and the state is
// untouched); pairs already in G or repeated in the batch are skipped; the
// survivors, in input order, are e_1..e_rho.
//  * new cliques: Algorithm 5, each e_i = (u,v) searched by Algorithm 8 on
//    G'[{u,v} u (Gamma'(u) n Gamma'(v))] with K = {u,v}, cand = the common
//    neighbours, fini = {}, excluding e_1..e_{i-1};
//  * subsumed cliques: Algorithm 7 run serially against the stored set C;
//    with `check_form` set, every membership answer is cross-checked against
//    the equivalent test "c' is a maximal clique of G" (returns -2 on a
//    mismatch).
int orc_imce_add(void* h, const uint32_t* src, const uint32_t* dst, uint64_t rho, orc_imce_result* res,
                 CliqueOut* new_out, CliqueOut* del_out, int check_form) {
  ImceState* st = (ImceState*)h;
  const uint64_t n = st->n;
  for (uint64_t i = 0; i < rho; ++i)
    if (src[i] >= n || dst[i] >= n || src[i] == dst[i]) return -1;
  std::map<std::pair<uint32_t, uint32_t>, uint64_t> index;
  std::vector<std::pair<uint32_t, uint32_t>> H;
  uint64_t skipped = 0;
  for (uint64_t i = 0; i < rho; ++i) {
    uint32_t a = std::min(src[i], dst[i]), b = std::max(src[i], dst[i]);
    if (st->A.has(a, b) || index.count({a, b})) { ++skipped; continue; }
    index[{a, b}] = H.size();
    H.push_back({a, b});
  }
  // Snapshot of G, needed by the cross-check of the subsumed test.
  Adj G_old;
  if (check_form) G_old = st->A;
  // G' = G + H
  for (auto& e : H) {
    insert_sorted(st->A.rows[e.first], e.second);
    insert_sorted(st->A.rows[e.second], e.first);
  }
  // Lambda_new
  Sink news;
  news.keep = true;
  for (uint64_t i = 0; i < H.size(); ++i) {
    uint32_t u = H[i].first, v = H[i].second;
    VSet common = intersect(st->A.rows[u], st->A.nb(v), st->A.deg(v));
    std::vector<uint32_t> K{u, v};
    Exclusion ex;
    ex.index = &index;
    ex.before = i;
    // Gamma_{G''}(w) n cand = Gamma_{G'}(w) n cand since cand, fini stay
    // inside V_e; the TTT routine reads G' directly.
    ttt(st->A, K, common, VSet(), news, ex);
  }
  // Lambda_del (Algorithm 7, serial)
  std::set<VSet> del;
  for (const VSet& c : news.cliques) {
    std::set<VSet> S{c};
    for (size_t x = 0; x < c.size(); ++x)
      for (size_t y = x + 1; y < c.size(); ++y) {
        auto key = std::make_pair(c[x], c[y]);
        if (!index.count(key)) continue;  // (c[x], c[y]) is not a new edge
        std::set<VSet> S2;
        for (const VSet& cp : S) {
          if (contains(cp, key.first) && contains(cp, key.second)) {
            VSet c1 = cp, c2 = cp;
            erase_sorted(c1, key.first);
            erase_sorted(c2, key.second);
            S2.insert(std::move(c1));
            S2.insert(std::move(c2));
          } else {
            S2.insert(cp);
          }
        }
        S.swap(S2);
      }
    for (const VSet& cp : S) {
      bool inC = st->C.count(cp) > 0;
      if (check_form) {
        // c' is a clique of G (a subset of a clique of G' with no new edge);
        // it is maximal in G iff no outside vertex is G-adjacent to all of it.
        bool maximal = !cp.empty();
        if (maximal) {
          uint32_t a = cp[0];
          for (uint32_t w : G_old.rows[a]) {
            if (contains(cp, w)) continue;
            bool all = true;
            for (uint32_t y : cp) if (!G_old.has(w, y)) { all = false; break; }
            if (all) { maximal = false; break; }
          }
        }
        // an earlier new clique of this batch may already have claimed c'
        if (maximal != (inC || del.count(cp) > 0)) return -2;
      }
      if (inC) {
        del.insert(cp);
        st->C.erase(cp);
      }
    }
  }
  orc_imce_result r{};
  r.n_applied = H.size();
  r.n_skipped = skipped;
  r.n_new = news.count;
  r.hash_new = news.hash;
  r.n_del = del.size();
  for (const VSet& c : del) r.hash_del += clique_hash(c.data(), c.size());
  for (const VSet& c : news.cliques) st->C.insert(c);
  st->count = st->count + r.n_new - r.n_del;
  st->hash = st->hash + r.hash_new - r.hash_del;
  r.count = st->count;
  r.set_hash = st->hash;
  *res = r;
  if (new_out) {
    std::vector<VSet> v = news.cliques;
    std::sort(v.begin(), v.end());
    write_cliques(v, new_out);
  }
  if (del_out) {
    std::vector<VSet> v(del.begin(), del.end());
    write_cliques(v, del_out);
  }
  return 0;
}

// Decremental step (Section 5.3): deleting a batch H from G reduces to the
// incremental case on G' = G - H with the same batch, because G = G' + H:
//  * C(G) \ C(G') = Lambda_new(G', H), the maximal cliques of G that hold an
//    edge of H: Algorithm 5 with the exclusion of Algorithm 8, run on G;
//  * C(G') \ C(G) = Lambda_del(G', H): Algorithm 7 over those cliques, whose
//    stored-set test "c' in C(G')" takes its equivalent form (c' is a clique
//    of G' that no outside vertex is G'-adjacent to all of), since C(G') is
//    what is being computed.
// Canonicalisation as for additions, except that pairs not in G (instead of
// pairs already in G) are skipped.  Returns -1 for a self-loop or id >= n
// (state untouched) and -2 if a removed clique is missing from the stored set
// or an added one is already in it.  In `res`, n_new / hash_new describe the
// cliques that become maximal (added) and n_del / hash_del those that stop
// being maximal (removed).
int orc_imce_remove(void* h, const uint32_t* src, const uint32_t* dst, uint64_t rho, orc_imce_result* res,
                    CliqueOut* added_out, CliqueOut* removed_out) {
  ImceState* st = (ImceState*)h;
  const uint64_t n = st->n;
  for (uint64_t i = 0; i < rho; ++i)
    if (src[i] >= n || dst[i] >= n || src[i] == dst[i]) return -1;
  std::map<std::pair<uint32_t, uint32_t>, uint64_t> index;
  std::vector<std::pair<uint32_t, uint32_t>> H;
  uint64_t skipped = 0;
  for (uint64_t i = 0; i < rho; ++i) {
    uint32_t a = std::min(src[i], dst[i]), b = std::max(src[i], dst[i]);
    if (!st->A.has(a, b) || index.count({a, b})) { ++skipped; continue; }
    index[{a, b}] = H.size();
    H.push_back({a, b});
  }
  // Lambda_new(G', H) on G = G' + H: the cliques that stop being maximal
  Sink gone;
  gone.keep = true;
  for (uint64_t i = 0; i < H.size(); ++i) {
    uint32_t u = H[i].first, v = H[i].second;
    VSet common = intersect(st->A.rows[u], st->A.nb(v), st->A.deg(v));
    std::vector<uint32_t> K{u, v};
    Exclusion ex;
    ex.index = &index;
    ex.before = i;
    ttt(st->A, K, common, VSet(), gone, ex);
  }
  for (const VSet& c : gone.cliques)
    if (!st->C.count(c)) return -2;
  // G' = G - H
  for (auto& e : H) {
    erase_sorted(st->A.rows[e.first], e.second);
    erase_sorted(st->A.rows[e.second], e.first);
  }
  // Lambda_del(G', H): edge-free subsets of the removed cliques, maximal in G'
  std::set<VSet> added;
  for (const VSet& c : gone.cliques)
    for (const VSet& cp : edge_free_subsets(c, index))
      if (maximal_in(st->A, cp)) added.insert(cp);
  for (const VSet& c : added)
    if (st->C.count(c)) return -2;
  orc_imce_result r{};
  r.n_applied = H.size();
  r.n_skipped = skipped;
  r.n_del = gone.count;
  r.hash_del = gone.hash;
  r.n_new = added.size();
  for (const VSet& c : added) r.hash_new += clique_hash(c.data(), c.size());
  for (const VSet& c : gone.cliques) st->C.erase(c);
  for (const VSet& c : added) st->C.insert(c);
  st->count = st->count + r.n_new - r.n_del;
  st->hash = st->hash + r.hash_new - r.hash_del;
  r.count = st->count;
  r.set_hash = st->hash;
  *res = r;
  if (added_out) {
    std::vector<VSet> v(added.begin(), added.end());
    write_cliques(v, added_out);
  }
  if (removed_out) {
    std::vector<VSet> v = gone.cliques;
    std::sort(v.begin(), v.end());
    write_cliques(v, removed_out);
  }
  return 0;
}

}  // extern "C"
