// Incremental maintenance of the maximal cliques under edge additions
// (Section 5).  One batch H:
//   1. canonicalise: reject self-loops / ids >= n; normalise (min, max); drop
//      pairs already in G and repeats (first occurrence wins); survivors in
//      input order are e_1..e_rho (Algorithm 5 takes them in any fixed order);
//   2. G' = G + H into a second CSR buffer (G stays intact until commit);
//   3. new cliques (Algorithms 5, 6, 8): one edge subproblem per e_i = (u, v)
//      with K = {u, v}, cand = Gamma'(u) n Gamma'(v), fini = {}; a child q is
//      skipped (and moved to fini) when K u {q} contains e_j, j < i.  The
//      persistent search kernel runs these subproblems in exclusion mode and
//      writes the new cliques to a device buffer;
//   4. subsumed cliques (Algorithm 7): each new clique c is split along its
//      batch edges into edge-free subsets; such a subset c' is a clique of G,
//      and c' is in C(G) iff no vertex outside c' is adjacent in G to all of
//      it (the stored-set test of Algorithm 7 in its equivalent form, checked
//      against the stored set by the oracle).  Candidates are de-duplicated
//      exactly, so each subsumed clique is reported once;
//   5. commit: G <- G', count += |new| - |del|, hash += H(new) - H(del).
// Any error before step 5 leaves the state unchanged.
//
// Deletions (Section 5.3) reduce to the same steps: G' = G - H is built in
// step 2, the edge subproblems of step 3 run on G (= G' + H) and give the
// cliques that stop being maximal, and step 4 tests maximality in G' and gives
// the cliques that become maximal.

#include <hipcub/hipcub.hpp>

#include <cstring>
#include <thread>
#include <vector>

#include "dev.h"
#include "internal.h"

using namespace mce;

// One batch between its search (phase A) and the collection of its result.
struct BatchSlot {
  DevBuf new_off, new_vert;  // cliques of the edge subproblems (the search's output)
  DevBuf dk, hk;             // the batch's sorted directed keys (u*n + v, both orientations) and edge keys
  DevBuf hoff;               // hoff[x]: first of vertex x's keys in dk (x = 0..n)
  DevBuf del_off, del_vert;  // the subsumed pass's de-duplicated cliques
  uint64_t cap_nc = 0, cap_nv = 0;
  bool remove = false;
  int prev = -1, next = -1;  // CSR buffer before and after the batch
  uint64_t m = 0, nd = 0, nnz_prev = 0, nnz_next = 0, nc_new = 0, nv_new = 0, dnc = 0, dnv = 0;
  uint64_t n_srch = 0, h_srch = 0, n_sub = 0, h_sub = 0;
  imce_result res;
  int rc = MCE_OK;           // of the subsumed pass
  char err[256] = "";
};

struct imce_state {
  uint64_t n = 0, nnz = 0;      // the graph the next batch applies to
  DevBuf rp[3], col[3];         // three CSR buffers: a batch's graph before, after, and the next batch's after
  int cur = 0;
  uint64_t count = 0, hash = 0; // clique count and set hash after the last batch whose subsumed pass finished
  mce_opts opts;
  // phase A (canonicalise, G +/- H, search)
  DevBuf bsrc, bdst, keys, idx, keys2, idx2, keep, pos, eu, ev, hkeys, hidx, hkeys2, hidx2, dkeys, didx, dkeys2, didx2,
      degw, p, x, words, gwords, off, goff, stats, arena, gids, order, bad;
  EnumWork ew;
  void* scan_tmp = nullptr;
  size_t scan_bytes = 0;
  void* sort_tmp = nullptr;
  size_t sort_bytes = 0;
  // phase B (subsumed pass), one batch at a time
  DevBuf cand_off, cand_vert, cand_hash, cand_id, chash2, chash3, cid2, uniq, sctl, sdefer, sbig;
  uint64_t cap_cc = 0, cap_cv = 0;
  uint64_t arena_per_edge = 0;  // largest edge-subproblem arena bytes per applied edge seen
  void* sort_tmp_b = nullptr;
  size_t sort_bytes_b = 0;
  // pipelined use (imce_submit / imce_collect): two slots, a FIFO of the
  // batches not yet collected, and the helper thread running a subsumed pass
  BatchSlot slot[2];
  int fifo[2] = {-1, -1};
  int nfifo = 0;
  hipStream_t sub_stream = nullptr;
  std::thread sub_thread;
  int sub_slot = -1;            // slot whose subsumed pass runs on sub_thread
};

namespace {

inline uint32_t blocks_for(uint64_t n, uint32_t bs) { return (uint32_t)((n + bs - 1) / bs); }

constexpr uint32_t kSubMaxK = 64;     // largest new clique the bitmask subsumed kernel takes
// common neighbours of a batch edge (an edge subproblem's cand): below the
// static search's limit, which keeps the large-clique subsumed kernel's LDS
// table within one workgroup's share
constexpr uint32_t kMaxCandEdge = 4096;
constexpr uint32_t kBigK = kMaxCandEdge + 2;  // largest new clique of any edge subproblem (|K| = 2 + |cand|)
constexpr uint32_t kBigInvolved = 64;     // batch-edge endpoints inside one large new clique
constexpr uint32_t kSubMaxS = 1024;   // candidate subsets per new clique
constexpr uint32_t kSubMaxPairs = 256;
constexpr uint32_t kEdgeRowsPerWave = 16;
constexpr uint64_t kStateHandUnits = 1ULL << 24;  // first handoff arena of a state: 1 GiB  // candidate rows one wave of k_edge_rows builds
constexpr uint32_t kSubFastS = 32;      // the first pass: subsets and batch edges per clique
constexpr uint32_t kSubFastPairs = 16;

// -- 1. canonicalisation -------------------------------------------------------

__global__ void k_canon(uint64_t rho, const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst, uint64_t n,
                        uint64_t* keys, uint32_t* idx, uint32_t* bad) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= rho) return;
  uint32_t a = src[i], b = dst[i];
  if (a >= n || b >= n || a == b) {
    atomicOr(bad, 1u);
    keys[i] = 0;
  } else {
    uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    keys[i] = lo * n + hi;
  }
  idx[i] = (uint32_t)i;
}

// After a stable sort by key: the first occurrence of each key survives
// unless the edge is already in G (additions) or is not in G (deletions).
__global__ void k_keep(uint64_t rho, const uint64_t* __restrict__ skeys, const uint32_t* __restrict__ sidx, uint64_t n,
                       const uint64_t* __restrict__ rp, const uint32_t* __restrict__ col, int remove, uint64_t* keep) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= rho) return;
  const uint64_t key = skeys[i];
  bool first = i == 0 || skeys[i - 1] != key;
  const uint32_t a = (uint32_t)(key / n), b = (uint32_t)(key % n);
  bool exists = bsearch_u32(col + rp[a], rp[a + 1] - rp[a], b) >= 0;
  keep[sidx[i]] = (first && exists == (remove != 0)) ? 1 : 0;
}

__global__ void k_scatter(uint64_t rho, const uint64_t* __restrict__ keep, const uint64_t* __restrict__ pos,
                          const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst, uint64_t n, uint32_t* eu,
                          uint32_t* ev, uint64_t* hkeys, uint32_t* hidx, uint64_t* dkeys, uint32_t* didx) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= rho || !keep[i]) return;
  const uint64_t j = pos[i];
  const uint32_t a = src[i], b = dst[i];
  const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
  eu[j] = lo;
  ev[j] = hi;
  hkeys[j] = (uint64_t)lo * n + hi;
  hidx[j] = (uint32_t)j;
  dkeys[2 * j] = (uint64_t)lo * n + hi;
  didx[2 * j] = (uint32_t)j;
  dkeys[2 * j + 1] = (uint64_t)hi * n + lo;
  didx[2 * j + 1] = (uint32_t)j;
}

// -- 2. G' = G + H ------------------------------------------------------------

__device__ __forceinline__ uint64_t lower_bound_u64(const uint64_t* a, uint64_t n, uint64_t x) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t lower_bound_u32(const uint32_t* a, uint64_t n, uint32_t x) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Start of every vertex's keys in the sorted directed batch keys (x * n + w):
// hoff[x] = the first key >= x * n, for x = 0..n (hoff[n] = nd).  Built once
// per batch, it replaces two binary searches per lookup in the kernels below.
__global__ void k_hoff(uint64_t n, const uint64_t* __restrict__ dkeys, uint64_t nd, uint64_t* hoff) {
  const uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (x <= n) hoff[x] = lower_bound_u64(dkeys, nd, x * n);
}

__global__ void k_newdeg(uint64_t n, const uint64_t* __restrict__ rp, const uint64_t* __restrict__ hoff,
                         uint64_t* degw) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint64_t lo = hoff[v], hi = hoff[v + 1];
  degw[v] = rp[v + 1] - rp[v] + (hi - lo);
}

__global__ void k_rp_tail(uint64_t n, uint64_t* rpn, const uint64_t* degw) { rpn[n] = rpn[n - 1] + degw[n - 1]; }

// G - H: degrees after the deletions (every batch pair is an edge of G).
__global__ void k_deldeg(uint64_t n, const uint64_t* __restrict__ rp, const uint64_t* __restrict__ hoff,
                         uint64_t* degw) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint64_t lo = hoff[v], hi = hoff[v + 1];
  degw[v] = rp[v + 1] - rp[v] - (hi - lo);
}

// One wave per vertex: its row without the deleted neighbours, order kept.
__global__ void __launch_bounds__(256) k_remove_rows(uint64_t n, const uint64_t* __restrict__ rp,
                                                     const uint32_t* __restrict__ col, const uint64_t* __restrict__ dkeys,
                                                     const uint64_t* __restrict__ hoff, const uint64_t* __restrict__ rpn,
                                                     uint32_t* coln) {
  const uint64_t v = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = lane_id();
  if (v >= n) return;
  const uint64_t lo = hoff[v], hi = hoff[v + 1];
  const uint32_t* row = col + rp[v];
  const uint64_t d = rp[v + 1] - rp[v];
  uint32_t* out = coln + rpn[v];
  uint64_t kept = 0;
  for (uint64_t j0 = 0; j0 < d; j0 += kWave) {
    const uint64_t j = j0 + lane;
    bool keep = j < d;
    const uint32_t w = keep ? row[j] : 0;
    if (keep && hi > lo) {
      const uint64_t k = lower_bound_u64(dkeys + lo, hi - lo, v * n + w);
      keep = !(k < hi - lo && dkeys[lo + k] == v * n + w);
    }
    const uint64_t bm = ballot(keep);
    if (keep) out[kept + mask_prefix(bm, lane)] = w;
    kept += (uint64_t)__popcll(bm);
  }
}

// One wave per vertex: merge the old row with the vertex's new neighbours.
__global__ void __launch_bounds__(256) k_merge_rows(uint64_t n, const uint64_t* __restrict__ rp,
                                                    const uint32_t* __restrict__ col, const uint64_t* __restrict__ dkeys,
                                                    const uint64_t* __restrict__ hoff, const uint64_t* __restrict__ rpn,
                                                    uint32_t* coln) {
  const uint64_t v = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = lane_id();
  if (v >= n) return;
  const uint64_t lo = hoff[v], hi = hoff[v + 1];
  const uint64_t t = hi - lo;
  const uint32_t* row = col + rp[v];
  const uint64_t d = rp[v + 1] - rp[v];
  uint32_t* out = coln + rpn[v];
  for (uint64_t j = lane; j < d; j += kWave) {
    const uint32_t w = row[j];
    // new neighbours smaller than w
    uint64_t a = 0, b = t;
    while (a < b) {
      uint64_t mid = (a + b) >> 1;
      if ((uint32_t)(dkeys[lo + mid] % n) < w) a = mid + 1;
      else b = mid;
    }
    out[j + a] = w;
  }
  for (uint64_t k = lane; k < t; k += kWave) {
    const uint32_t w = (uint32_t)(dkeys[lo + k] % n);
    out[k + lower_bound_u32(row, d, w)] = w;
  }
}

// -- 3. edge subproblems ------------------------------------------------------

// |Gamma'(u) n Gamma'(v)| for every batch edge (one wave per edge).
__global__ void __launch_bounds__(256) k_edge_sizes(uint64_t m, const uint32_t* __restrict__ eu,
                                                    const uint32_t* __restrict__ ev, const uint64_t* __restrict__ rp,
                                                    const uint32_t* __restrict__ col, uint32_t* P, uint32_t* X,
                                                    uint64_t* words, uint64_t* gwords, uint64_t* stats) {
  const uint64_t e = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = lane_id();
  if (e >= m) return;
  uint32_t a = eu[e], b = ev[e];
  uint64_t da = rp[a + 1] - rp[a], db = rp[b + 1] - rp[b];
  if (da > db) {
    uint32_t t = a; a = b; b = t;
    uint64_t tt = da; da = db; db = tt;
  }
  uint32_t c = 0;
  for (uint64_t j = lane; j < da; j += kWave) c += bsearch_u32(col + rp[b], db, col[rp[a] + j]) >= 0 ? 1u : 0u;
  c = (uint32_t)wave_sum_u64(c);
  if (lane == 0) {
    const uint64_t wp = (c + 63) / 64;
    P[e] = c;
    X[e] = 0;
    words[e] = wp * (2ULL * c + 1);
    gwords[e] = c;
    atomicMax((unsigned long long*)&stats[0], (unsigned long long)c);
    atomicMax((unsigned long long*)&stats[1], (unsigned long long)(4 * wp + 1));
  }
}

// Vertex-id table of each edge subproblem: the common neighbours, ascending.
__global__ void __launch_bounds__(256) k_edge_gids(uint64_t m, const uint32_t* __restrict__ eu,
                                                   const uint32_t* __restrict__ ev, const uint64_t* __restrict__ rp,
                                                   const uint32_t* __restrict__ col, const uint64_t* __restrict__ goff,
                                                   uint32_t* gids) {
  const uint64_t e = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = lane_id();
  if (e >= m) return;
  uint32_t a = eu[e], b = ev[e];
  uint64_t da = rp[a + 1] - rp[a], db = rp[b + 1] - rp[b];
  if (da > db) {
    uint32_t t = a; a = b; b = t;
    uint64_t tt = da; da = db; db = tt;
  }
  uint32_t* g = gids + goff[e];
  uint32_t cnt = 0;
  for (uint64_t c0 = 0; c0 < da; c0 += kWave) {
    const uint64_t j = c0 + lane;
    const uint32_t w = j < da ? col[rp[a] + j] : 0;
    const bool in = j < da && bsearch_u32(col + rp[b], db, w) >= 0;
    const uint64_t bm = ballot(in);
    if (in) g[cnt + mask_prefix(bm, lane)] = w;
    cnt += (uint32_t)__popcll(bm);
  }
}

// Bit rows of each edge subproblem: adjacency among the common neighbours
// (word-major), exclusion rows excl[a] = {b : (g[a], g[b]) = e_j, j < i} and
// the root exclusion set F0 = {a : (g[a], u) or (g[a], v) = e_j, j < i}.
__global__ void __launch_bounds__(256) k_edge_rows(uint64_t m, const uint32_t* __restrict__ eu,
                                                   const uint32_t* __restrict__ ev, const uint64_t* __restrict__ rp,
                                                   const uint32_t* __restrict__ col, const uint32_t* __restrict__ P,
                                                   const uint64_t* __restrict__ off, const uint64_t* __restrict__ goff,
                                                   const uint32_t* __restrict__ gids, const uint64_t* __restrict__ dkeys,
                                                   const uint32_t* __restrict__ didx, const uint64_t* __restrict__ hoff,
                                                   uint64_t n, uint64_t* arena) {
  // wave (edge e, blockIdx.y): candidates [y * kEdgeRowsPerWave, ...)
  const uint64_t e = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = lane_id();
  if (e >= m) return;
  const uint32_t p = P[e];
  const uint32_t a0 = blockIdx.y * kEdgeRowsPerWave;
  if (a0 >= p) return;
  const uint32_t a1 = a0 + kEdgeRowsPerWave < p ? a0 + kEdgeRowsPerWave : p;
  const uint64_t wp = (p + 63) / 64;
  uint64_t* rowP = arena + off[e];
  uint64_t* excl = rowP + wp * p;
  uint64_t* F0 = excl + (uint64_t)p * wp;
  const uint32_t* g = gids + goff[e];
  const uint32_t u = eu[e], v = ev[e];
  for (uint32_t a = a0; a < a1; ++a) {
    const uint32_t q = g[a];
    for (uint64_t j = rp[q] + lane; j < rp[q + 1]; j += kWave) {
      const int64_t b = bsearch_u32(g, p, col[j]);
      if (b >= 0) atomicOr((unsigned long long*)&rowP[(uint64_t)(b >> 6) * p + a], 1ULL << (b & 63));
    }
    const uint64_t lo = hoff[q], hi = hoff[q + 1];
    for (uint64_t k = lo + lane; k < hi; k += kWave) {
      if (didx[k] >= e) continue;  // only e_j with j < i are excluded
      const uint32_t w = (uint32_t)(dkeys[k] % n);
      if (w == u || w == v) {
        atomicOr((unsigned long long*)&F0[a >> 6], 1ULL << (a & 63));
      } else {
        const int64_t b = bsearch_u32(g, p, w);
        if (b >= 0) atomicOr((unsigned long long*)&excl[(uint64_t)a * wp + (b >> 6)], 1ULL << (b & 63));
      }
    }
  }
}

__global__ void k_iota32(uint64_t n, uint32_t* a) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = (uint32_t)i;
}

// -- 4. subsumed cliques --------------------------------------------------------

// Candidates found by one wave are staged here and reserved in the output
// with one atomic per kStageN (instead of one per candidate: a single counter
// hit by every wave of the GPU is what bounds the pass otherwise).
constexpr uint32_t kStageN = 32, kStageV = 512;

template <uint32_t MAXS, uint32_t MAXP>
struct SubLds {
  uint32_t c[kSubMaxK];
  uint64_t rb[kSubMaxK], re[kSubMaxK];  // row range of c[j] in the graph without H
  uint32_t ord[kSubMaxK];               // members by ascending degree (ties by index)
  uint64_t pairs[MAXP];
  uint64_t S[2][MAXS];
  uint32_t np, ns;
  uint32_t sv[kStageV];  // staged candidates' vertices, back to back
  uint32_t sk[kStageN];  // their sizes
  uint64_t sh[kStageN];  // their clique hash terms
  uint32_t snn, snv;     // staged candidates and vertices
};

// Writes the staged candidates out (one reservation for all of them) and
// empties the stage.  Every lane calls it.
template <class SL>
__device__ void stage_flush(SL& L, uint64_t* sctl, uint64_t* cand_off, uint32_t* cand_vert, uint64_t* cand_hash,
                            uint64_t cap_c, uint64_t cap_v) {
  const int lane = lane_id();
  __syncthreads();
  const uint32_t nn = L.snn, nv = L.snv;
  if (nn == 0) return;
  uint64_t old = 0;
  if (lane == 0) old = atomicAdd((unsigned long long*)&sctl[0], (unsigned long long)(((uint64_t)nn << 32) | nv));
  old = readlane64(old, 0);
  const uint64_t id = old >> 32, pos = old & 0xFFFFFFFFULL;
  if (id + nn > cap_c || pos + nv > cap_v) {
    if (lane == 0) atomicOr((unsigned long long*)&sctl[1], 4ULL);
  } else {
    for (uint32_t j = lane; j < nv; j += kWave) cand_vert[pos + j] = L.sv[j];
    const uint32_t kk = lane < (int)nn ? L.sk[lane] : 0u;
    const uint32_t incl = wave_incl_scan_u32(kk);
    if (lane < (int)nn) {
      cand_off[id + lane] = pos + incl - kk;
      cand_hash[id + lane] = L.sh[lane];
    }
  }
  __syncthreads();
  if (lane == 0) {
    L.snn = 0;
    L.snv = 0;
  }
  __syncthreads();
}

// Subsumed-clique candidates of the new cliques (or of those listed in
// `list`, `*nlist` of them).  A clique whose batch edges or subsets exceed
// this instance's LDS capacities is appended to `defer` (when given) for the
// large-capacity instance; without `defer` that is an error (flag 2).  A
// clique of more than kSubMaxK vertices goes to `big` for k_subsumed_big.
// sctl: [0] packed candidate counter (cands << 32 | verts), [1] flags
// (1: clique too large, 2: too many subsets or pairs, 4: candidate overflow),
// [2] deferred cliques, [3] cliques for k_subsumed_big
template <uint32_t MAXS, uint32_t MAXP>
__global__ void __launch_bounds__(64) k_subsumed(uint64_t nnew, const uint32_t* __restrict__ list,
                                                 const uint64_t* __restrict__ nlist, uint32_t* defer,
                                                 uint32_t* big, const uint64_t* __restrict__ noff,
                                                 const uint32_t* __restrict__ nvert, uint64_t n,
                                                 const uint64_t* __restrict__ rp, const uint32_t* __restrict__ col,
                                                 const uint64_t* __restrict__ hkeys, uint64_t nh,
                                                 const uint64_t* __restrict__ dkeys, const uint64_t* __restrict__ hoff, uint64_t* sctl,
                                                 uint64_t* cand_off, uint32_t* cand_vert, uint64_t* cand_hash,
                                                 uint64_t cap_c, uint64_t cap_v) {
  __shared__ SubLds<MAXS, MAXP> L;
  const int lane = threadIdx.x;
  const uint64_t items = list ? *nlist : nnew;
  if (lane == 0) {
    L.snn = 0;
    L.snv = 0;
  }
  __syncthreads();
  for (uint64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const uint64_t ci = list ? list[it] : it;
    const uint64_t b0 = noff[ci];
    const uint32_t k = (uint32_t)(noff[ci + 1] - b0);
    if (k > kSubMaxK) {
      if (lane == 0) {
        if (big)
          big[atomicAdd((unsigned long long*)&sctl[3], 1ULL)] = (uint32_t)ci;
        else
          atomicOr((unsigned long long*)&sctl[1], 1ULL);
      }
      continue;
    }
    if (lane < (int)k) L.c[lane] = nvert[b0 + lane];
    if (lane == 0) L.np = 0;
    __syncthreads();
    // the members' rows, loaded once for all the subset tests below, and the
    // members in ascending degree (the order in which a candidate extension is
    // checked: shorter searches, and a non-neighbour found sooner)
    {
      const uint32_t x = lane < (int)k ? L.c[lane] : 0;
      const uint64_t b = lane < (int)k ? rp[x] : 0, e = lane < (int)k ? rp[x + 1] : 0;
      if (lane < (int)k) {
        L.rb[lane] = b;
        L.re[lane] = e;
      }
      const uint64_t key = lane < (int)k ? (((e - b) << 7) | (uint64_t)lane) : ~0ULL;
      uint32_t rank = 0;
      for (uint32_t j = 0; j < k; ++j) rank += readlane64(key, j) < key ? 1u : 0u;
      if (lane < (int)k) L.ord[rank] = (uint32_t)lane;
    }
    __syncthreads();
    // batch edges inside c: lane j walks the new neighbours of c[j]
    if (lane < (int)k) {
      const uint32_t x = L.c[lane];
      const uint64_t lo = hoff[x], hi = hoff[x + 1];
      for (uint64_t t = lo; t < hi; ++t) {
        const uint32_t w = (uint32_t)(dkeys[t] % n);
        if (w <= x) continue;  // each pair once
        const int64_t j2 = bsearch_u32(L.c, k, w);
        if (j2 >= 0) {
          uint32_t slot = atomicAdd(&L.np, 1u);
          if (slot < MAXP) L.pairs[slot] = (1ULL << lane) | (1ULL << j2);
        }
      }
    }
    __syncthreads();
    const uint32_t npairs = L.np;
    if (npairs > MAXP) {
      if (lane == 0) {
        if (defer)
          defer[atomicAdd((unsigned long long*)&sctl[2], 1ULL)] = (uint32_t)ci;
        else
          atomicOr((unsigned long long*)&sctl[1], 2ULL);
      }
      __syncthreads();
      continue;
    }
    // Algorithm 7: split every subset that holds both ends of a batch edge
    int cur = 0;
    uint32_t ns = 1;
    if (lane == 0) L.S[0][0] = k == 64 ? ~0ULL : ((1ULL << k) - 1);
    bool overflow = false;
    for (uint32_t e = 0; e < npairs && !overflow; ++e) {
      __syncthreads();
      const uint64_t pm = L.pairs[e];
      const uint64_t bx = pm & (~pm + 1), by = pm & ~bx;
      uint32_t nout = 0;
      for (uint32_t base = 0; base < ns; base += kWave) {
        const uint32_t i = base + lane;
        const uint64_t sm = i < ns ? L.S[cur][i] : 0;
        const bool split = i < ns && (sm & pm) == pm;
        const bool keep1 = i < ns && !split;
        const uint32_t cnt = split ? 2u : (keep1 ? 1u : 0u);
        const uint32_t incl = wave_incl_scan_u32(cnt);
        const uint32_t total = readlane32(incl, 63);
        if (nout + total > MAXS) {
          overflow = true;
          break;
        }
        const uint32_t o = nout + incl - cnt;
        if (split) {
          L.S[cur ^ 1][o] = sm & ~bx;
          L.S[cur ^ 1][o + 1] = sm & ~by;
        } else if (keep1) {
          L.S[cur ^ 1][o] = sm;
        }
        nout += total;
      }
      cur ^= 1;
      ns = nout;
    }
    __syncthreads();
    if (overflow) {
      if (lane == 0) {
        if (defer)
          defer[atomicAdd((unsigned long long*)&sctl[2], 1ULL)] = (uint32_t)ci;
        else
          atomicOr((unsigned long long*)&sctl[1], 2ULL);
      }
      continue;
    }
    // each distinct subset once (first occurrence), then the maximality test in G
    for (uint32_t i = 0; i < ns; ++i) {
      const uint64_t sm = L.S[cur][i];
      bool dup = false;
      for (uint32_t j = lane; j < i && !dup; j += kWave) dup = L.S[cur][j] == sm;
      if (ballot(dup)) continue;
      // the member of c' with the smallest degree in G (the first in degree order)
      const bool mem = lane < (int)k && ((sm >> lane) & 1ULL);
      const uint32_t x = mem ? L.c[lane] : 0;
      uint32_t first = 0;
      while (first < k && !((sm >> L.ord[first]) & 1ULL)) ++first;
      if (first >= k) continue;  // an empty subset (cannot occur: a split keeps one end of each pair)
      const int la = (int)L.ord[first];
      // is some w outside c' adjacent in G to every vertex of c'?  Each lane
      // takes a neighbour w of c'[la] and checks the other members in degree order
      bool extends = false;
      const uint64_t ab = L.rb[la], ae = L.re[la];
      for (uint64_t j0 = ab; j0 < ae; j0 += kWave) {
        const uint64_t j = j0 + lane;
        bool ok = j < ae;
        uint32_t w = ok ? col[j] : 0;
        if (ok) {
          const int64_t pos = bsearch_u32(L.c, k, w);
          if (pos >= 0 && ((sm >> pos) & 1ULL)) ok = false;
        }
        for (uint32_t t = first + 1; ok && t < k; ++t) {
          const uint32_t y = L.ord[t];
          if (!((sm >> y) & 1ULL)) continue;
          ok = bsearch_u32(col + L.rb[y], L.re[y] - L.rb[y], w) >= 0;
        }
        if (ballot(ok)) {
          extends = true;
          break;
        }
      }
      if (extends) continue;
      // c' is a maximal clique of G: a subsumed-clique candidate, staged
      const uint32_t kk = (uint32_t)__popcll(sm);
      if (L.snn == kStageN || L.snv + kk > kStageV)
        stage_flush(L, sctl, cand_off, cand_vert, cand_hash, cap_c, cap_v);
      const uint32_t at = L.snv;
      const uint64_t below = mem ? __popcll(sm & ((1ULL << lane) - 1)) : 0;
      if (mem) L.sv[at + below] = x;
      const uint64_t z = wave_sum_u64(mem ? mix64(x) : 0);
      __syncthreads();
      if (lane == 0) {
        L.sk[L.snn] = kk;
        L.sh[L.snn] = clique_term(z, kk);
        L.snn += 1;
        L.snv = at + kk;
      }
      __syncthreads();
    }
    __syncthreads();
  }
  stage_flush(L, sctl, cand_off, cand_vert, cand_hash, cap_c, cap_v);
}

// Subsumed-clique candidates of new cliques with more than kSubMaxK vertices
// (Algorithm 7 as in k_subsumed).  Only the endpoints of batch edges inside c
// can leave a subset, so subsets are bitmasks over those "involved" vertices
// (at most kBigInvolved of them); every other vertex of c belongs to every
// subset.  One wave per listed clique.  Flags as in k_subsumed (2: more than
// kBigInvolved involved vertices, kSubMaxPairs batch edges or kSubMaxS subsets).
struct BigLds {
  uint32_t c[kBigK];
  uint16_t invof[kBigK];  // involved index of each position of c, or 0xFFFF
  uint32_t ipos[kBigInvolved];
  uint64_t pairs[kSubMaxPairs];  // batch edges inside c as (position, position), then as involved-index masks
  uint64_t S[2][kSubMaxS];
  uint32_t np, ni, bad;
};

__global__ void __launch_bounds__(64) k_subsumed_big(const uint32_t* __restrict__ list, const uint64_t* __restrict__ nlist,
                                                     const uint64_t* __restrict__ noff,
                                                     const uint32_t* __restrict__ nvert, uint64_t n,
                                                     const uint64_t* __restrict__ rp, const uint32_t* __restrict__ col,
                                                     const uint64_t* __restrict__ dkeys, const uint64_t* __restrict__ hoff, uint64_t* sctl,
                                                     uint64_t* cand_off, uint32_t* cand_vert, uint64_t* cand_hash,
                                                     uint64_t cap_c, uint64_t cap_v) {
  __shared__ BigLds L;
  const int lane = threadIdx.x;
  const uint64_t items = *nlist;
  for (uint64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const uint64_t ci = list[it];
    const uint64_t b0 = noff[ci];
    const uint32_t k = (uint32_t)(noff[ci + 1] - b0);
    if (k > kBigK) {
      if (lane == 0) atomicOr((unsigned long long*)&sctl[1], 1ULL);
      continue;
    }
    for (uint32_t j = lane; j < k; j += kWave) {
      L.c[j] = nvert[b0 + j];
      L.invof[j] = 0xFFFF;
    }
    if (lane == 0) {
      L.np = 0;
      L.ni = 0;
      L.bad = 0;
    }
    __syncthreads();
    // batch edges inside c (each pair once, from its smaller vertex)
    for (uint32_t j = lane; j < k; j += kWave) {
      const uint32_t x = L.c[j];
      const uint64_t lo = hoff[x], hi = hoff[x + 1];
      for (uint64_t t = lo; t < hi; ++t) {
        const uint32_t w = (uint32_t)(dkeys[t] % n);
        if (w <= x) continue;
        const int64_t j2 = bsearch_u32(L.c, k, w);
        if (j2 >= 0) {
          const uint32_t slot = atomicAdd(&L.np, 1u);
          if (slot < kSubMaxPairs) L.pairs[slot] = (uint64_t)j | ((uint64_t)j2 << 32);
        }
      }
    }
    __syncthreads();
    const uint32_t npairs = L.np;
    if (npairs > kSubMaxPairs) {
      if (lane == 0) atomicOr((unsigned long long*)&sctl[1], 2ULL);
      __syncthreads();
      continue;
    }
    // involved vertices: the distinct endpoints, numbered in order of appearance
    if (lane == 0) {
      for (uint32_t e = 0; e < npairs && !L.bad; ++e) {
        const uint32_t ends[2] = {(uint32_t)L.pairs[e], (uint32_t)(L.pairs[e] >> 32)};
        uint64_t m = 0;
        for (uint32_t z = 0; z < 2; ++z) {
          uint32_t ix = L.invof[ends[z]];
          if (ix == 0xFFFF) {
            if (L.ni >= kBigInvolved) {
              L.bad = 1;
              break;
            }
            ix = L.ni++;
            L.invof[ends[z]] = (uint16_t)ix;
            L.ipos[ix] = ends[z];
          }
          m |= 1ULL << ix;
        }
        L.pairs[e] = m;
      }
    }
    __syncthreads();
    if (L.bad) {
      if (lane == 0) atomicOr((unsigned long long*)&sctl[1], 2ULL);
      __syncthreads();
      continue;
    }
    const uint32_t ni = L.ni;
    // Algorithm 7: split every subset that holds both ends of a batch edge
    int cur = 0;
    uint32_t ns = 1;
    if (lane == 0) L.S[0][0] = ni == 64 ? ~0ULL : ((1ULL << ni) - 1);
    bool overflow = false;
    for (uint32_t e = 0; e < npairs && !overflow; ++e) {
      __syncthreads();
      const uint64_t pm = L.pairs[e];
      const uint64_t bx = pm & (~pm + 1), by = pm & ~bx;
      uint32_t nout = 0;
      for (uint32_t base = 0; base < ns; base += kWave) {
        const uint32_t i = base + lane;
        const uint64_t sm = i < ns ? L.S[cur][i] : 0;
        const bool split = i < ns && (sm & pm) == pm;
        const bool keep1 = i < ns && !split;
        const uint32_t cnt = split ? 2u : (keep1 ? 1u : 0u);
        const uint32_t incl = wave_incl_scan_u32(cnt);
        const uint32_t total = readlane32(incl, 63);
        if (nout + total > kSubMaxS) {
          overflow = true;
          break;
        }
        const uint32_t o = nout + incl - cnt;
        if (split) {
          L.S[cur ^ 1][o] = sm & ~bx;
          L.S[cur ^ 1][o + 1] = sm & ~by;
        } else if (keep1) {
          L.S[cur ^ 1][o] = sm;
        }
        nout += total;
      }
      cur ^= 1;
      ns = nout;
    }
    __syncthreads();
    if (overflow) {
      if (lane == 0) atomicOr((unsigned long long*)&sctl[1], 2ULL);
      continue;
    }
    for (uint32_t i = 0; i < ns; ++i) {
      const uint64_t sm = L.S[cur][i];
      bool dup = false;
      for (uint32_t j = lane; j < i && !dup; j += kWave) dup = L.S[cur][j] == sm;
      if (ballot(dup)) continue;
      // position j of c is in c' unless it is an involved vertex left out
      auto member = [&](uint32_t j) {
        const uint32_t ix = L.invof[j];
        return ix == 0xFFFF || ((sm >> ix) & 1ULL);
      };
      // the member of c' with the smallest degree in G
      uint64_t mn = ~0ULL;
      for (uint32_t j = lane; j < k; j += kWave) {
        if (!member(j)) continue;
        const uint32_t x = L.c[j];
        const uint64_t key = ((rp[x + 1] - rp[x]) << 13) | j;
        mn = key < mn ? key : mn;
      }
      for (int o = 32; o >= 1; o >>= 1) {
        uint64_t t = __shfl_xor(mn, o, kWave);
        mn = t < mn ? t : mn;
      }
      const uint32_t la = (uint32_t)(mn & 8191);
      const uint32_t a = L.c[la];
      // is some w outside c' adjacent in G to every vertex of c'?
      bool extends = false;
      const uint64_t ab = rp[a], ae = rp[a + 1];
      for (uint64_t j0 = ab; j0 < ae && !extends; j0 += kWave) {
        const uint64_t j = j0 + lane;
        bool ok = j < ae;
        const uint32_t w = ok ? col[j] : 0;
        if (ok) {
          const int64_t pos = bsearch_u32(L.c, k, w);
          if (pos >= 0 && member((uint32_t)pos)) ok = false;
        }
        for (uint32_t y = 0; ok && y < k; ++y) {
          if (y == la || !member(y)) continue;
          const uint32_t yy = L.c[y];
          ok = bsearch_u32(col + rp[yy], rp[yy + 1] - rp[yy], w) >= 0;
        }
        extends = ballot(ok) != 0;
      }
      if (extends) continue;
      // c' is a maximal clique of G: a subsumed-clique candidate
      const uint32_t kk = k - (ni - (uint32_t)__popcll(sm));
      uint64_t old = 0;
      if (lane == 0) old = atomicAdd((unsigned long long*)&sctl[0], (unsigned long long)((1ULL << 32) | kk));
      old = readlane64(old, 0);
      const uint64_t id = old >> 32, pos = old & 0xFFFFFFFFULL;
      if (id >= cap_c || pos + kk > cap_v) {
        if (lane == 0) atomicOr((unsigned long long*)&sctl[1], 4ULL);
        continue;
      }
      uint64_t z = 0;
      uint32_t written = 0;
      for (uint32_t j0 = 0; j0 < k; j0 += kWave) {
        const uint32_t j = j0 + lane;
        const bool mem = j < k && member(j);
        const uint64_t bm = ballot(mem);
        if (mem) {
          const uint32_t x = L.c[j];
          cand_vert[pos + written + mask_prefix(bm, lane)] = x;
          z += mix64(x);
        }
        written += (uint32_t)__popcll(bm);
      }
      z = wave_sum_u64(z);
      if (lane == 0) {
        cand_off[id] = pos;
        cand_hash[id] = clique_term(z, kk);
      }
    }
    __syncthreads();
  }
}

// After sorting candidates by hash: a candidate is kept unless an earlier one
// of the same hash run has the same vertex list.  Kept ones are counted,
// hashed and (optionally) written out.
__global__ void k_dedup(uint64_t nc, const uint64_t* __restrict__ shash, const uint32_t* __restrict__ sid,
                        const uint64_t* __restrict__ cand_off, const uint32_t* __restrict__ cand_vert,
                        uint64_t total_verts, uint64_t* uniq_ctl,
                        uint64_t* out_off, uint32_t* out_vert, uint64_t cap_c, uint64_t cap_v) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const uint32_t me = sid[i];
  const uint64_t b = cand_off[me];
  const uint64_t e = (uint64_t)me + 1 < nc ? cand_off[me + 1] : total_verts;
  const uint64_t len = e - b;
  bool dup = false;
  for (uint64_t j = i; j > 0 && !dup;) {
    --j;
    if (shash[j] != shash[i]) break;
    const uint32_t o = sid[j];
    const uint64_t ob = cand_off[o];
    const uint64_t oe = (uint64_t)o + 1 < nc ? cand_off[o + 1] : total_verts;
    if (oe - ob != len) continue;
    bool same = true;
    for (uint64_t t = 0; t < len && same; ++t) same = cand_vert[ob + t] == cand_vert[b + t];
    dup = same;
  }
  if (dup) return;
  atomicAdd((unsigned long long*)&uniq_ctl[0], 1ULL);
  atomicAdd((unsigned long long*)&uniq_ctl[1], (unsigned long long)shash[i]);
  if (out_vert) {
    uint64_t old = atomicAdd((unsigned long long*)&uniq_ctl[2], (unsigned long long)((1ULL << 32) | len));
    uint64_t id = old >> 32, pos = old & 0xFFFFFFFFULL;
    if (id < cap_c && pos + len <= cap_v) {
      out_off[id] = pos;
      for (uint64_t t = 0; t < len; ++t) out_vert[pos + t] = cand_vert[b + t];
    }
  }
}

__global__ void k_set_u64(uint64_t* p, uint64_t v) { *p = v; }

int sort_pairs_u64_u32(void*& tmp, size_t& tmp_bytes, uint64_t* k, uint32_t* v, uint64_t* k2, uint32_t* v2,
                       uint64_t nitems, hipStream_t s, uint64_t** ko, uint32_t** vo) {
  hipcub::DoubleBuffer<uint64_t> kb(k, k2);
  hipcub::DoubleBuffer<uint32_t> vb(v, v2);
  size_t need = 0;
  MCE_TRY_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, need, kb, vb, (int)nitems, 0, 64, s));
  MCE_TRY(ensure_temp(tmp, tmp_bytes, need));
  MCE_TRY_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, need, kb, vb, (int)nitems, 0, 64, s));
  *ko = kb.Current();
  *vo = vb.Current();
  return MCE_OK;
}

int copy_cliques_out(mce_clique_buf* out, const uint64_t* off, const uint32_t* vert, uint64_t nc, uint64_t nv,
                     hipStream_t s) {
  out->n_cliques = nc;
  out->n_verts = nv;
  if (nc > out->cap_cliques || nv > out->cap_verts || (nc && !out->off) || (nv && !out->vert)) return MCE_ENOSPC;
  const hipMemcpyKind kind = out->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (out->off) {
    if (nc) MCE_TRY_HIP(hipMemcpyAsync(out->off, off, nc * sizeof(uint64_t), kind, s));
    if (out->on_device) {
      hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, out->off + nc, nv);
      MCE_TRY_HIP(hipGetLastError());
    } else {
      MCE_TRY_HIP(hipStreamSynchronize(s));
      out->off[nc] = nv;
    }
  }
  if (nv) MCE_TRY_HIP(hipMemcpyAsync(out->vert, vert, nv * sizeof(uint32_t), kind, s));
  return MCE_OK;
}

// Device time between two events (0 when either is missing).
double event_ms(hipEvent_t a, hipEvent_t b) {
  float t = 0;
  if (!a || !b || hipEventElapsedTime(&t, a, b) != hipSuccess) return 0;
  return t;
}

struct Events {
  hipEvent_t e[2] = {nullptr, nullptr};
  ~Events() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
  int init() {
    for (auto& x : e) MCE_TRY_HIP(hipEventCreate(&x));
    return MCE_OK;
  }
};

// A CSR buffer for a batch's graph after the batch: neither the current one
// nor `keep` (the graph a pending subsumed pass still reads).
int free_buffer(const imce_state* st, int keep) {
  for (int b = 0; b < 3; ++b)
    if (b != st->cur && b != keep) return b;
  return -1;
}

// Phase A of one batch of edge additions (remove = false) or deletions
// (remove = true) into slot `si`: canonicalise, build the graph after the
// batch into a free CSR buffer (`keep` is protected), run the edge
// subproblems (new cliques).  On success the state's current graph is the
// one after the batch; on error the state is as it was.
//
// A deletion is the reduction of Section 5.3: with G' = G - H, G = G' + H, so
// the edge-subproblem search over G finds Lambda_new(G', H) = the cliques that
// stop being maximal, and the subsumed pass over G' finds Lambda_del(G', H) =
// the cliques that become maximal.  The same kernels run with the roles of
// the two graphs swapped: the search always runs on the graph that holds H,
// the maximality test on the graph without it.
int phase_a(imce_state* st, const uint32_t* src, const uint32_t* dst, uint64_t rho, int on_device, bool remove,
            int si, int keep) {
  BatchSlot& b = st->slot[si];
  hipStream_t s = (hipStream_t)st->opts.hip_stream;
  const uint64_t n = st->n;
  std::memset(&b.res, 0, sizeof(b.res));
  b.remove = remove;
  b.rc = MCE_OK;
  b.err[0] = 0;
  b.m = b.nd = b.nc_new = b.nv_new = b.dnc = b.dnv = 0;
  b.n_srch = b.h_srch = b.n_sub = b.h_sub = 0;
  b.prev = b.next = st->cur;
  b.nnz_prev = b.nnz_next = st->nnz;
  if (rho == 0) return MCE_OK;
  if (!src || !dst) {
    set_error("NULL batch arrays");
    return MCE_EINVAL;
  }
  Events evs;
  MCE_TRY(evs.init());
  MCE_TRY_HIP(hipEventRecord(evs.e[0], s));

  const uint64_t* rp = st->rp[st->cur].as<uint64_t>();
  const uint32_t* col = st->col[st->cur].as<uint32_t>();
  const uint32_t* dsrc = src;
  const uint32_t* ddst = dst;
  if (!on_device) {
    MCE_TRY(st->bsrc.ensure(rho * sizeof(uint32_t)));
    MCE_TRY(st->bdst.ensure(rho * sizeof(uint32_t)));
    MCE_TRY_HIP(hipMemcpyAsync(st->bsrc.p, src, rho * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    MCE_TRY_HIP(hipMemcpyAsync(st->bdst.p, dst, rho * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    dsrc = st->bsrc.as<uint32_t>();
    ddst = st->bdst.as<uint32_t>();
  }

  // 1. canonicalise
  MCE_TRY(st->keys.ensure(rho * 8));
  MCE_TRY(st->keys2.ensure(rho * 8));
  MCE_TRY(st->idx.ensure(rho * 4));
  MCE_TRY(st->idx2.ensure(rho * 4));
  MCE_TRY(st->keep.ensure(rho * 8));
  MCE_TRY(st->pos.ensure(rho * 8));
  MCE_TRY(st->bad.ensure(8));
  MCE_TRY_HIP(dev_zero(st->bad.p, 4, s));
  hipLaunchKernelGGL(k_canon, dim3(blocks_for(rho, 256)), dim3(256), 0, s, rho, dsrc, ddst, n, st->keys.as<uint64_t>(),
                     st->idx.as<uint32_t>(), st->bad.as<uint32_t>());
  MCE_TRY_HIP(hipGetLastError());
  uint32_t bad = 0;
  MCE_TRY_HIP(hipMemcpyAsync(&bad, st->bad.p, 4, hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipStreamSynchronize(s));
  if (bad) {
    set_error("batch has a self-loop or a vertex id >= n");
    return MCE_EINVAL;
  }
  uint64_t* skeys;
  uint32_t* sidx;
  MCE_TRY(sort_pairs_u64_u32(st->sort_tmp, st->sort_bytes, st->keys.as<uint64_t>(), st->idx.as<uint32_t>(),
                             st->keys2.as<uint64_t>(), st->idx2.as<uint32_t>(), rho, s, &skeys, &sidx));
  hipLaunchKernelGGL(k_keep, dim3(blocks_for(rho, 256)), dim3(256), 0, s, rho, skeys, sidx, n, rp, col,
                     remove ? 1 : 0, st->keep.as<uint64_t>());
  MCE_TRY_HIP(hipGetLastError());
  MCE_TRY(device_exclusive_scan(st->keep.as<uint64_t>(), st->pos.as<uint64_t>(), rho, st->scan_tmp, st->scan_bytes, s));
  uint64_t lastpos = 0, lastkeep = 0;
  MCE_TRY_HIP(hipMemcpyAsync(&lastpos, st->pos.as<uint64_t>() + rho - 1, 8, hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipMemcpyAsync(&lastkeep, st->keep.as<uint64_t>() + rho - 1, 8, hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipStreamSynchronize(s));
  const uint64_t m = lastpos + lastkeep;  // applied edges
  b.res.n_applied = m;
  b.res.n_skipped = rho - m;
  if (m == 0) {
    MCE_TRY_HIP(hipEventRecord(evs.e[1], s));
    MCE_TRY_HIP(hipStreamSynchronize(s));
    b.res.new_ms = event_ms(evs.e[0], evs.e[1]);
    return MCE_OK;
  }
  const uint64_t nd = 2 * m;
  MCE_TRY(st->eu.ensure(m * 4));
  MCE_TRY(st->ev.ensure(m * 4));
  MCE_TRY(st->hkeys.ensure(m * 8));
  MCE_TRY(st->hidx.ensure(m * 4));
  MCE_TRY(st->hkeys2.ensure(m * 8));
  MCE_TRY(st->hidx2.ensure(m * 4));
  MCE_TRY(st->dkeys.ensure(nd * 8));
  MCE_TRY(st->didx.ensure(nd * 4));
  MCE_TRY(st->dkeys2.ensure(nd * 8));
  MCE_TRY(st->didx2.ensure(nd * 4));
  hipLaunchKernelGGL(k_scatter, dim3(blocks_for(rho, 256)), dim3(256), 0, s, rho, st->keep.as<uint64_t>(),
                     st->pos.as<uint64_t>(), dsrc, ddst, n, st->eu.as<uint32_t>(), st->ev.as<uint32_t>(),
                     st->hkeys.as<uint64_t>(), st->hidx.as<uint32_t>(), st->dkeys.as<uint64_t>(), st->didx.as<uint32_t>());
  MCE_TRY_HIP(hipGetLastError());
  uint64_t* hk;
  uint32_t* hi;
  MCE_TRY(sort_pairs_u64_u32(st->sort_tmp, st->sort_bytes, st->hkeys.as<uint64_t>(), st->hidx.as<uint32_t>(),
                             st->hkeys2.as<uint64_t>(), st->hidx2.as<uint32_t>(), m, s, &hk, &hi));
  uint64_t* dk;
  uint32_t* di;
  MCE_TRY(sort_pairs_u64_u32(st->sort_tmp, st->sort_bytes, st->dkeys.as<uint64_t>(), st->didx.as<uint32_t>(),
                             st->dkeys2.as<uint64_t>(), st->didx2.as<uint32_t>(), nd, s, &dk, &di));
  // the subsumed pass reads the sorted keys after the next batch has reused
  // these buffers: keep a copy in the slot
  MCE_TRY(b.dk.ensure(nd * 8));
  MCE_TRY(b.hk.ensure(m * 8));
  MCE_TRY_HIP(hipMemcpyAsync(b.dk.p, dk, nd * 8, hipMemcpyDeviceToDevice, s));
  MCE_TRY_HIP(hipMemcpyAsync(b.hk.p, hk, m * 8, hipMemcpyDeviceToDevice, s));
  MCE_TRY(b.hoff.ensure((n + 1) * 8));
  hipLaunchKernelGGL(k_hoff, dim3(blocks_for(n + 1, 256)), dim3(256), 0, s, n, dk, nd, b.hoff.as<uint64_t>());
  MCE_TRY_HIP(hipGetLastError());
  const uint64_t* hof = b.hoff.as<uint64_t>();

  // 2. the graph after the batch, G + H or G - H, into a free buffer
  const int nxt = free_buffer(st, keep);
  const uint64_t nnz2 = remove ? st->nnz - nd : st->nnz + nd;
  MCE_TRY(st->degw.ensure(n * 8));
  MCE_TRY(st->rp[nxt].ensure((n + 1) * 8));
  MCE_TRY(st->col[nxt].ensure(std::max<uint64_t>(nnz2, 1) * 4));
  uint64_t* rpn = st->rp[nxt].as<uint64_t>();
  uint32_t* coln = st->col[nxt].as<uint32_t>();
  if (remove)
    hipLaunchKernelGGL(k_deldeg, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, hof, st->degw.as<uint64_t>());
  else
    hipLaunchKernelGGL(k_newdeg, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, hof, st->degw.as<uint64_t>());
  MCE_TRY_HIP(hipGetLastError());
  MCE_TRY(device_exclusive_scan(st->degw.as<uint64_t>(), rpn, n, st->scan_tmp, st->scan_bytes, s));
  hipLaunchKernelGGL(k_rp_tail, dim3(1), dim3(1), 0, s, n, rpn, st->degw.as<uint64_t>());
  if (remove)
    hipLaunchKernelGGL(k_remove_rows, dim3(blocks_for(n * 64, 256)), dim3(256), 0, s, n, rp, col, dk, hof, rpn, coln);
  else
    hipLaunchKernelGGL(k_merge_rows, dim3(blocks_for(n * 64, 256)), dim3(256), 0, s, n, rp, col, dk, hof, rpn, coln);
  MCE_TRY_HIP(hipGetLastError());
  // the search runs on the graph that holds H
  const uint64_t* srp = remove ? rp : rpn;
  const uint32_t* scol = remove ? col : coln;

  // 3. new cliques: one edge subproblem per applied edge
  MCE_TRY(st->p.ensure(m * 4));
  MCE_TRY(st->x.ensure(m * 4));
  MCE_TRY(st->words.ensure(m * 8));
  MCE_TRY(st->gwords.ensure(m * 8));
  MCE_TRY(st->off.ensure(m * 8));
  MCE_TRY(st->goff.ensure(m * 8));
  MCE_TRY(st->order.ensure(m * 4));
  MCE_TRY(st->stats.ensure(8 * 8));
  MCE_TRY_HIP(dev_zero(st->stats.p, 64, s));
  hipLaunchKernelGGL(k_edge_sizes, dim3(blocks_for(m * 64, 256)), dim3(256), 0, s, m, st->eu.as<uint32_t>(),
                     st->ev.as<uint32_t>(), srp, scol, st->p.as<uint32_t>(), st->x.as<uint32_t>(),
                     st->words.as<uint64_t>(), st->gwords.as<uint64_t>(), st->stats.as<uint64_t>());
  MCE_TRY_HIP(hipGetLastError());
  MCE_TRY(device_exclusive_scan(st->words.as<uint64_t>(), st->off.as<uint64_t>(), m, st->scan_tmp, st->scan_bytes, s));
  MCE_TRY(device_exclusive_scan(st->gwords.as<uint64_t>(), st->goff.as<uint64_t>(), m, st->scan_tmp, st->scan_bytes, s));
  uint64_t stats[8], tl[4];
  MCE_TRY_HIP(hipMemcpyAsync(stats, st->stats.p, 64, hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipMemcpyAsync(&tl[0], st->off.as<uint64_t>() + m - 1, 8, hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipMemcpyAsync(&tl[1], st->words.as<uint64_t>() + m - 1, 8, hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipMemcpyAsync(&tl[2], st->goff.as<uint64_t>() + m - 1, 8, hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipMemcpyAsync(&tl[3], st->gwords.as<uint64_t>() + m - 1, 8, hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipStreamSynchronize(s));
  if (stats[0] > kMaxCandEdge) {
    set_error("an edge subproblem has %llu common neighbours; at most %u are supported",
              (unsigned long long)stats[0], kMaxCandEdge);
    return MCE_ENOTSUP;
  }
  const uint64_t aw = std::max<uint64_t>(tl[0] + tl[1], 1), gw = std::max<uint64_t>(tl[2] + tl[3], 1);
  st->arena_per_edge = std::max<uint64_t>(st->arena_per_edge, (aw * 8 + m - 1) / m);
  MCE_TRY(st->arena.ensure(aw * 8));
  MCE_TRY(st->gids.ensure(gw * 4));
  MCE_TRY_HIP(dev_zero(st->arena.p, aw * 8, s));
  hipLaunchKernelGGL(k_edge_gids, dim3(blocks_for(m * 64, 256)), dim3(256), 0, s, m, st->eu.as<uint32_t>(),
                     st->ev.as<uint32_t>(), srp, scol, st->goff.as<uint64_t>(), st->gids.as<uint32_t>());
  const uint32_t row_chunks = (uint32_t)std::max<uint64_t>((stats[0] + kEdgeRowsPerWave - 1) / kEdgeRowsPerWave, 1);
  hipLaunchKernelGGL(k_edge_rows, dim3(blocks_for(m * 64, 256), row_chunks), dim3(256), 0, s, m, st->eu.as<uint32_t>(),
                     st->ev.as<uint32_t>(), srp, scol, st->p.as<uint32_t>(), st->off.as<uint64_t>(),
                     st->goff.as<uint64_t>(), st->gids.as<uint32_t>(), dk, di, hof, n, st->arena.as<uint64_t>());
  hipLaunchKernelGGL(k_iota32, dim3(blocks_for(m, 256)), dim3(256), 0, s, m, st->order.as<uint32_t>());
  MCE_TRY_HIP(hipGetLastError());

  if (b.cap_nc == 0) {
    b.cap_nc = 1 << 20;
    b.cap_nv = 1 << 24;
  }
  uint64_t ctl[CTL_WORDS];
  for (int attempt = 0;; ++attempt) {
    MCE_TRY(b.new_off.ensure((b.cap_nc + 1) * 8));
    MCE_TRY(b.new_vert.ensure(b.cap_nv * 4));
    EnumJob job;
    job.sub.off = st->off.as<uint64_t>();
    job.sub.goff = st->goff.as<uint64_t>();
    job.sub.p = st->p.as<uint32_t>();
    job.sub.x = st->x.as<uint32_t>();
    job.sub.r0 = st->eu.as<uint32_t>();
    job.sub.r1 = st->ev.as<uint32_t>();
    job.arena = st->arena.as<uint64_t>();
    job.gids = st->gids.as<uint32_t>();
    job.nq = m;
    job.order = st->order.as<uint32_t>();
    job.max_p = stats[0];
    job.max_frame = stats[1];
    job.excl = true;
    job.nodes_v = job.count_v = job.hash_v = nullptr;
    job.cl_off = b.new_off.as<uint64_t>();
    job.cl_vert = b.new_vert.as<uint32_t>();
    job.cap_cliques = b.cap_nc;
    job.cap_verts = b.cap_nv;
    job.opts = &st->opts;
    job.hand_initial_units = kStateHandUnits;
    MCE_TRY(run_enum(job, st->ew, s, ctl, nullptr));
    b.res.nodes = ctl[CTL_NODES];
    b.res.handed = job.handed;
    b.res.compact_ms = job.hand_ms;
    if (ctl[CTL_FLAGS] & 2ULL) {
      set_error("new cliques exceed 2^32 vertices or a clique exceeds the supported size");
      return MCE_ENOTSUP;
    }
    const uint64_t nc = ctl[CTL_CLQ] >> 32, nv = ctl[CTL_CLQ] & 0xFFFFFFFFULL;
    if (nc <= b.cap_nc && nv <= b.cap_nv) break;
    if (attempt >= 2) {
      set_error("new-clique buffer sizing did not converge");
      return MCE_ENOMEM;
    }
    b.cap_nc = std::max(b.cap_nc, nc);
    b.cap_nv = std::max(b.cap_nv, nv);
  }
  b.n_srch = ctl[CTL_COUNT];
  b.h_srch = ctl[CTL_HASH];
  b.nc_new = ctl[CTL_CLQ] >> 32;
  b.nv_new = ctl[CTL_CLQ] & 0xFFFFFFFFULL;
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, b.new_off.as<uint64_t>() + b.nc_new, b.nv_new);
  MCE_TRY_HIP(hipGetLastError());
  MCE_TRY_HIP(hipEventRecord(evs.e[1], s));
  MCE_TRY_HIP(hipStreamSynchronize(s));
  b.res.new_ms = event_ms(evs.e[0], evs.e[1]);
  b.m = m;
  b.nd = nd;
  b.prev = st->cur;
  b.next = nxt;
  b.nnz_next = nnz2;
  // the graph the next batch applies to
  st->cur = nxt;
  st->nnz = nnz2;
  return MCE_OK;
}

// Phase B of slot `si` on stream `s`: the subsumed pass (Algorithm 7) over the
// search's cliques, tested for maximality in the graph without H, then exact
// de-duplication (always written to the slot's lists).  Sets b.n_sub, b.h_sub,
// b.dnc, b.dnv.  Touches only the phase-B buffers and the slot.
int phase_b(imce_state* st, int si, hipStream_t s) {
  BatchSlot& b = st->slot[si];
  if (b.m == 0) return MCE_OK;
  const uint64_t n = st->n, m = b.m, nc_new = b.nc_new;
  const int mb = b.remove ? b.next : b.prev;  // the graph without H
  const uint64_t* mrp = st->rp[mb].as<uint64_t>();
  const uint32_t* mcol = st->col[mb].as<uint32_t>();
  const uint64_t* hk = b.hk.as<uint64_t>();
  const uint64_t* dk = b.dk.as<uint64_t>();
  const uint64_t* hof = b.hoff.as<uint64_t>();
  Events evs;
  MCE_TRY(evs.init());
  MCE_TRY_HIP(hipEventRecord(evs.e[0], s));
  if (st->cap_cc == 0) {
    st->cap_cc = 1 << 20;
    st->cap_cv = 1 << 24;
  }
  uint64_t sctl[4];
  for (int attempt = 0;; ++attempt) {
    MCE_TRY(st->cand_off.ensure((st->cap_cc + 1) * 8));
    MCE_TRY(st->cand_vert.ensure(st->cap_cv * 4));
    MCE_TRY(st->cand_hash.ensure(st->cap_cc * 8));
    MCE_TRY(st->sctl.ensure(4 * 8));
    MCE_TRY(st->sdefer.ensure(std::max<uint64_t>(nc_new, 1) * 4));
    MCE_TRY(st->sbig.ensure(std::max<uint64_t>(nc_new, 1) * 4));
    MCE_TRY_HIP(dev_zero(st->sctl.p, 32, s));
    if (nc_new) {
      // most new cliques hold one or two batch edges: a small-LDS pass with
      // many waves per CU, then the rest with room for kSubMaxS subsets
      const uint32_t grid = (uint32_t)std::min<uint64_t>(nc_new, 32768);
      uint64_t* sc = st->sctl.as<uint64_t>();
      uint32_t* defer = st->sdefer.as<uint32_t>();
      uint32_t* big = st->sbig.as<uint32_t>();
      hipLaunchKernelGGL((k_subsumed<kSubFastS, kSubFastPairs>), dim3(grid), dim3(64), 0, s, nc_new, nullptr, nullptr,
                         defer, big, b.new_off.as<uint64_t>(), b.new_vert.as<uint32_t>(), n, mrp, mcol, hk, m, dk,
                         hof, sc, st->cand_off.as<uint64_t>(), st->cand_vert.as<uint32_t>(),
                         st->cand_hash.as<uint64_t>(), st->cap_cc, st->cap_cv);
      MCE_TRY_HIP(hipGetLastError());
      hipLaunchKernelGGL((k_subsumed<kSubMaxS, kSubMaxPairs>), dim3(1024), dim3(64), 0, s, nc_new, defer, sc + 2,
                         nullptr, nullptr, b.new_off.as<uint64_t>(), b.new_vert.as<uint32_t>(), n, mrp, mcol, hk, m,
                         dk, hof, sc, st->cand_off.as<uint64_t>(), st->cand_vert.as<uint32_t>(),
                         st->cand_hash.as<uint64_t>(), st->cap_cc, st->cap_cv);
      MCE_TRY_HIP(hipGetLastError());
      // new cliques above kSubMaxK vertices (rare: a batch edge inside a very large clique)
      hipLaunchKernelGGL(k_subsumed_big, dim3(256), dim3(64), 0, s, big, sc + 3, b.new_off.as<uint64_t>(),
                         b.new_vert.as<uint32_t>(), n, mrp, mcol, dk, hof, sc, st->cand_off.as<uint64_t>(),
                         st->cand_vert.as<uint32_t>(), st->cand_hash.as<uint64_t>(), st->cap_cc, st->cap_cv);
      MCE_TRY_HIP(hipGetLastError());
    }
    MCE_TRY_HIP(hipMemcpyAsync(sctl, st->sctl.p, 16, hipMemcpyDeviceToHost, s));
    MCE_TRY_HIP(hipStreamSynchronize(s));
    if (sctl[1] & 3ULL) {
      set_error("a new clique holds more than %u batch edges, more than %u of its vertices are ends of batch "
                "edges (cliques above %u vertices), or it splits into more than %u subsets",
                kSubMaxPairs, kBigInvolved, kSubMaxK, kSubMaxS);
      return MCE_ENOTSUP;
    }
    if (!(sctl[1] & 4ULL)) break;
    if (attempt >= 2) {
      set_error("candidate buffer sizing did not converge");
      return MCE_ENOMEM;
    }
    st->cap_cc = std::max<uint64_t>(st->cap_cc, sctl[0] >> 32);
    st->cap_cv = std::max<uint64_t>(st->cap_cv, sctl[0] & 0xFFFFFFFFULL);
  }
  const uint64_t ncand = sctl[0] >> 32, nvcand = sctl[0] & 0xFFFFFFFFULL;
  uint64_t uctl[3] = {0, 0, 0};
  MCE_TRY(st->uniq.ensure(4 * 8));
  MCE_TRY_HIP(dev_zero(st->uniq.p, 32, s));
  MCE_TRY(b.del_off.ensure((ncand + 1) * 8));
  MCE_TRY(b.del_vert.ensure(std::max<uint64_t>(nvcand, 1) * 4));
  if (ncand) {
    MCE_TRY(st->cand_id.ensure(ncand * 4));
    MCE_TRY(st->chash2.ensure(ncand * 8));
    MCE_TRY(st->cid2.ensure(ncand * 4));
    hipLaunchKernelGGL(k_iota32, dim3(blocks_for(ncand, 256)), dim3(256), 0, s, ncand, st->cand_id.as<uint32_t>());
    // sorting reorders the hash array in place: keep the per-candidate hashes
    MCE_TRY_HIP(hipMemcpyAsync(st->chash2.p, st->cand_hash.p, ncand * 8, hipMemcpyDeviceToDevice, s));
    uint64_t* sh;
    uint32_t* sid;
    MCE_TRY(st->chash3.ensure(ncand * 8));
    MCE_TRY(sort_pairs_u64_u32(st->sort_tmp_b, st->sort_bytes_b, st->chash2.as<uint64_t>(),
                               st->cand_id.as<uint32_t>(), st->chash3.as<uint64_t>(), st->cid2.as<uint32_t>(), ncand,
                               s, &sh, &sid));
    hipLaunchKernelGGL(k_dedup, dim3(blocks_for(ncand, 256)), dim3(256), 0, s, ncand, sh, sid,
                       st->cand_off.as<uint64_t>(), st->cand_vert.as<uint32_t>(), nvcand, st->uniq.as<uint64_t>(),
                       b.del_off.as<uint64_t>(), b.del_vert.as<uint32_t>(), nvcand ? ncand : 0, nvcand);
    MCE_TRY_HIP(hipGetLastError());
    MCE_TRY_HIP(hipMemcpyAsync(uctl, st->uniq.p, 24, hipMemcpyDeviceToHost, s));
  }
  MCE_TRY_HIP(hipEventRecord(evs.e[1], s));
  MCE_TRY_HIP(hipStreamSynchronize(s));
  b.n_sub = uctl[0];
  b.h_sub = uctl[1];
  b.dnc = uctl[2] >> 32;
  b.dnv = uctl[2] & 0xFFFFFFFFULL;
  b.res.sub_ms = event_ms(evs.e[0], evs.e[1]);
  return MCE_OK;
}

// The result fields of a slot after both phases (new / del as the caller
// names them, count and hash after the batch given the count and hash before).
void finish_result(const BatchSlot& b, uint64_t count_before, uint64_t hash_before, imce_result* r) {
  *r = b.res;
  r->n_new = b.remove ? b.n_sub : b.n_srch;
  r->n_del = b.remove ? b.n_srch : b.n_sub;
  r->hash_new = b.remove ? b.h_sub : b.h_srch;
  r->hash_del = b.remove ? b.h_srch : b.h_sub;
  r->count = count_before + r->n_new - r->n_del;
  r->set_hash = hash_before + r->hash_new - r->hash_del;
  r->ms = b.res.new_ms + b.res.sub_ms;
}

// Copies a slot's clique lists to the caller's buffers (sizes always written).
int copy_slot_out(const BatchSlot& b, mce_clique_buf* new_cl, mce_clique_buf* del_cl, hipStream_t s) {
  mce_clique_buf* search_cl = b.remove ? del_cl : new_cl;
  mce_clique_buf* sub_cl = b.remove ? new_cl : del_cl;
  if (new_cl) new_cl->n_cliques = new_cl->n_verts = 0;
  if (del_cl) del_cl->n_cliques = del_cl->n_verts = 0;
  if (b.m == 0) return MCE_OK;
  int rc = MCE_OK;
  if (search_cl) {
    int r = copy_cliques_out(search_cl, b.new_off.as<uint64_t>(), b.new_vert.as<uint32_t>(), b.nc_new, b.nv_new, s);
    if (r == MCE_ENOSPC) rc = MCE_ENOSPC;
    else if (r != MCE_OK) return r;
  }
  if (sub_cl) {
    int r = copy_cliques_out(sub_cl, b.del_off.as<uint64_t>(), b.del_vert.as<uint32_t>(), b.dnc, b.dnv, s);
    if (r == MCE_ENOSPC) rc = MCE_ENOSPC;
    else if (r != MCE_OK) return r;
  }
  MCE_TRY_HIP(hipStreamSynchronize(s));
  return rc;
}

// Waits for the running subsumed pass.  When it failed, the graph returns to
// the one before that batch, and any later batch (already searched) is
// discarded; returns that batch's error (MCE_OK otherwise).
int join_sub(imce_state* st) {
  if (st->sub_slot < 0) return MCE_OK;
  st->sub_thread.join();
  const int si = st->sub_slot;
  st->sub_slot = -1;
  BatchSlot& b = st->slot[si];
  if (b.rc != MCE_OK) {
    st->cur = b.prev;
    st->nnz = b.nnz_prev;
    return b.rc;
  }
  // commit the batch's count and hash (passes run in batch order)
  imce_result r;
  finish_result(b, st->count, st->hash, &r);
  st->count = r.count;
  st->hash = r.set_hash;
  b.res = r;
  return MCE_OK;
}

// One batch start to end (imce_add_edges / imce_remove_edges).
int update_impl(imce_state* st, const uint32_t* src, const uint32_t* dst, uint64_t rho, int on_device,
                imce_result* res, mce_clique_buf* new_cl, mce_clique_buf* del_cl, bool remove) {
  std::memset(res, 0, sizeof(*res));
  res->count = st->count;
  res->set_hash = st->hash;
  if (new_cl) new_cl->n_cliques = new_cl->n_verts = 0;
  if (del_cl) del_cl->n_cliques = del_cl->n_verts = 0;
  if (st->nfifo > 0) {
    set_error("submitted batches are pending: collect them with imce_collect first");
    return MCE_EINVAL;
  }
  hipStream_t s = (hipStream_t)st->opts.hip_stream;
  const int prev = st->cur;
  const uint64_t nnz0 = st->nnz;
  int rc = phase_a(st, src, dst, rho, on_device, remove, 0, -1);
  if (rc == MCE_OK) rc = phase_b(st, 0, s);
  if (rc == MCE_OK) {
    rc = copy_slot_out(st->slot[0], new_cl, del_cl, s);
    if (rc == MCE_ENOSPC) set_error("clique buffer too small (sizes written back); the batch was not applied");
  }
  if (rc != MCE_OK) {
    st->cur = prev;  // all or nothing
    st->nnz = nnz0;
    return rc;
  }
  finish_result(st->slot[0], st->count, st->hash, res);
  st->count = res->count;
  st->hash = res->set_hash;
  return MCE_OK;
}

// imce_submit: phase A now (overlapping the previous batch's subsumed pass),
// then the subsumed pass on the state's second stream and a helper thread.
int submit_impl(imce_state* st, const uint32_t* src, const uint32_t* dst, uint64_t rho, int on_device, bool remove) {
  if (st->nfifo >= 2) {
    set_error("two submitted batches are not collected yet: call imce_collect first");
    return MCE_EINVAL;
  }
  const int si = st->nfifo == 0 ? 0 : (st->fifo[0] ^ 1);
  const int keep = st->sub_slot >= 0 ? st->slot[st->sub_slot].prev : -1;  // read by the running pass
  int rc = phase_a(st, src, dst, rho, on_device, remove, si, keep);
  if (rc != MCE_OK) return rc;  // the state (and the pending batch) as before
  const int rb = join_sub(st);
  if (rb != MCE_OK) {
    // the earlier batch failed: the graph went back to before it, and this
    // batch, searched on top of it, is dropped
    set_error("an earlier submitted batch failed (collect it for its error); this batch was discarded and the "
              "state is as before that batch");
    return MCE_ECANCELED;
  }
  BatchSlot* b = &st->slot[si];
  st->fifo[st->nfifo++] = si;
  st->sub_slot = si;
  st->sub_thread = std::thread([st, b, si]() {
    b->rc = phase_b(st, si, st->sub_stream);
    if (b->rc != MCE_OK) snprintf(b->err, sizeof(b->err), "%s", mce_last_error());
  });
  return MCE_OK;
}

int collect_impl(imce_state* st, imce_result* res, mce_clique_buf* new_cl, mce_clique_buf* del_cl) {
  std::memset(res, 0, sizeof(*res));
  if (st->nfifo == 0) {
    set_error("no submitted batch to collect");
    return MCE_EINVAL;
  }
  const int si = st->fifo[0];
  BatchSlot& b = st->slot[si];
  if (st->sub_slot == si) join_sub(st);
  if (b.rc != MCE_OK) {
    set_error("%s", b.err);
    const int rc = b.rc;
    st->fifo[0] = st->fifo[1];
    --st->nfifo;
    return rc;
  }
  const int rc = copy_slot_out(b, new_cl, del_cl, (hipStream_t)st->opts.hip_stream);
  *res = b.res;
  if (rc == MCE_ENOSPC) {
    set_error("clique buffer too small (sizes written back); the batch stays to be collected");
    return rc;
  }
  if (rc != MCE_OK) return rc;
  st->fifo[0] = st->fifo[1];
  --st->nfifo;
  return MCE_OK;
}

uint64_t state_bytes(const imce_state* st) {
  uint64_t t = st->scan_bytes + st->sort_bytes + st->sort_bytes_b + st->ew.sort_bytes;
  for (const DevBuf* b :
       {&st->rp[0], &st->rp[1], &st->rp[2], &st->col[0], &st->col[1], &st->col[2], &st->bsrc, &st->bdst, &st->keys,
        &st->idx, &st->keys2, &st->idx2, &st->keep, &st->pos, &st->eu, &st->ev, &st->hkeys, &st->hidx, &st->hkeys2,
        &st->hidx2, &st->dkeys, &st->didx, &st->dkeys2, &st->didx2, &st->degw, &st->p, &st->x, &st->words,
        &st->gwords, &st->off, &st->goff, &st->stats, &st->arena, &st->gids, &st->order, &st->bad, &st->cand_off,
        &st->cand_vert, &st->cand_hash, &st->cand_id, &st->chash2, &st->chash3, &st->cid2, &st->uniq, &st->sctl,
        &st->sdefer, &st->sbig})
    t += b->bytes;
  for (const BatchSlot& b : st->slot)
    for (const DevBuf* d : {&b.new_off, &b.new_vert, &b.dk, &b.hk, &b.hoff, &b.del_off, &b.del_vert}) t += d->bytes;
  for (const DevBuf* d : {&st->ew.queue, &st->ew.ctl, &st->ew.pool, &st->ew.pool_next, &st->ew.stacks, &st->ew.hand,
                          &st->ew.hand_idx, &st->ew.hkeys, &st->ew.hkeys2, &st->ew.hvals, &st->ew.hvals2,
                          &st->ew.kbig})
    t += d->bytes;
  return t;
}

// Device memory a batch of rho edges may add to the state, from the sizing
// rules of phase A and B: every buffer a batch grows to its size for rho
// applied edges (minus what it already holds), the search tables on the
// state's first batch, and the edge-subproblem rows at the largest bytes per
// applied edge seen so far (4 KiB before any batch).
uint64_t batch_bytes(const imce_state* st, uint64_t rho) {
  auto grow = [](const DevBuf& b, uint64_t need) -> uint64_t { return need > b.bytes ? need - b.bytes : 0; };
  const uint64_t n = st->n, m = rho, nd = 2 * rho;
  uint64_t t = 0;
  t += grow(st->keys, rho * 8) + grow(st->keys2, rho * 8) + grow(st->idx, rho * 4) + grow(st->idx2, rho * 4) +
       grow(st->keep, rho * 8) + grow(st->pos, rho * 8) + grow(st->bsrc, rho * 4) + grow(st->bdst, rho * 4);
  t += grow(st->eu, m * 4) + grow(st->ev, m * 4) + grow(st->hkeys, m * 8) + grow(st->hidx, m * 4) +
       grow(st->hkeys2, m * 8) + grow(st->hidx2, m * 4) + grow(st->dkeys, nd * 8) + grow(st->didx, nd * 4) +
       grow(st->dkeys2, nd * 8) + grow(st->didx2, nd * 4);
  t += grow(st->p, m * 4) + grow(st->x, m * 4) + grow(st->words, m * 8) + grow(st->gwords, m * 8) +
       grow(st->off, m * 8) + grow(st->goff, m * 8) + grow(st->order, m * 4) + grow(st->degw, n * 8);
  // the graph after the batch: one more CSR buffer of the current size plus the batch
  const uint64_t need_csr = (n + 1) * 8 + (st->nnz + nd) * 4;
  uint64_t spare = 0;
  for (int b = 0; b < 3; ++b)
    if (b != st->cur) spare = std::max<uint64_t>(spare, st->rp[b].bytes + st->col[b].bytes);
  t += need_csr > spare ? need_csr - spare : 0;
  // edge-subproblem rows and vertex ids
  const uint64_t per_edge = st->arena_per_edge ? st->arena_per_edge : 4096;
  t += grow(st->arena, m * per_edge) + grow(st->gids, m * 256);
  // slot buffers of one batch (the first batch sizes them)
  const BatchSlot& b = st->slot[0];
  t += grow(b.dk, nd * 8) + grow(b.hk, m * 8) + grow(b.hoff, (n + 1) * 8);
  if (b.cap_nc == 0) t += (1ULL << 20) * 8 + (1ULL << 24) * 4;  // new-clique lists
  if (st->cap_cc == 0) t += (1ULL << 20) * 16 + (1ULL << 24) * 4 + (1ULL << 20) * 24;  // candidates and dedup
  // the search's tables (queue, donation pool, handoff arena) on the first batch
  if (st->ew.pool.bytes == 0)
    t += (1ULL << 16) * kBlockWords * 8 + (1ULL << 16) * 4 + (m + std::max<uint64_t>(1u << 24, 4 * m)) * 8 +
         kStateHandUnits * 64 + kStateHandUnits * 4;
  return t;
}

void release_state(imce_state* st) {
  if (st->sub_slot >= 0) {
    st->sub_thread.join();
    st->sub_slot = -1;
  }
  DevBuf* bufs[] = {&st->rp[0], &st->rp[1], &st->rp[2], &st->col[0], &st->col[1], &st->col[2], &st->bsrc, &st->bdst,
                    &st->keys, &st->idx, &st->keys2, &st->idx2, &st->keep, &st->pos, &st->eu, &st->ev, &st->hkeys,
                    &st->hidx, &st->hkeys2, &st->hidx2, &st->dkeys, &st->didx, &st->dkeys2, &st->didx2, &st->degw,
                    &st->p, &st->x, &st->words, &st->gwords, &st->off, &st->goff, &st->stats, &st->arena, &st->gids,
                    &st->order, &st->bad, &st->cand_off, &st->cand_vert, &st->cand_hash, &st->cand_id, &st->chash2,
                    &st->chash3, &st->cid2, &st->uniq, &st->sctl, &st->sdefer, &st->sbig};
  for (DevBuf* b : bufs) b->release();
  for (BatchSlot& b : st->slot)
    for (DevBuf* d : {&b.new_off, &b.new_vert, &b.dk, &b.hk, &b.hoff, &b.del_off, &b.del_vert}) d->release();
  st->ew.release();
  for (void** t : {&st->scan_tmp, &st->sort_tmp, &st->sort_tmp_b})
    if (*t) (void)hipFree(*t);
  st->scan_tmp = st->sort_tmp = st->sort_tmp_b = nullptr;
  if (st->sub_stream) (void)hipStreamDestroy(st->sub_stream);
  st->sub_stream = nullptr;
}

}  // namespace

extern "C" {

int imce_create(const mce_csr* g, const mce_opts* opts, imce_state** out, mce_result* initial) {
  if (!g || !out) {
    set_error("NULL graph or output");
    return MCE_EINVAL;
  }
  *out = nullptr;
  if (g->n >= 0xFFFFFFFFULL) {
    set_error("n must be below 2^32 - 1");
    return MCE_ENOTSUP;
  }
  imce_state* st = new imce_state();
  std::memset(&st->opts, 0, sizeof(st->opts));
  if (opts) st->opts = *opts;
  st->opts.sched = MCE_SCHED_DEGREE;
  st->opts.sched_cost = nullptr;
  hipStream_t s = (hipStream_t)st->opts.hip_stream;
  const uint64_t n = g->n;
  st->n = n;
  auto fail = [&](int rc) {
    release_state(st);
    delete st;
    return rc;
  };
  uint64_t nnz = 0;
  if (n > 0 && !g->row_ptr) {
    set_error("row_ptr is NULL");
    return fail(MCE_EINVAL);
  }
  if (n > 0) {
    if (g->on_device) {
      if (hipMemcpyAsync(&nnz, g->row_ptr + n, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        set_error("reading row_ptr[n] failed");
        return fail(MCE_EDEVICE);
      }
    } else {
      nnz = g->row_ptr[n];
    }
  }
  st->nnz = nnz;
  int rc;
  if ((rc = st->rp[0].ensure((n + 1) * 8)) != MCE_OK) return fail(rc);
  if ((rc = st->col[0].ensure(std::max<uint64_t>(nnz, 1) * 4)) != MCE_OK) return fail(rc);
  const hipMemcpyKind kind = g->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (n > 0 && hipMemcpyAsync(st->rp[0].p, g->row_ptr, (n + 1) * 8, kind, s) != hipSuccess) return fail(MCE_EDEVICE);
  if (nnz > 0 && hipMemcpyAsync(st->col[0].p, g->col, nnz * 4, kind, s) != hipSuccess) return fail(MCE_EDEVICE);
  if (n == 0) {
    uint64_t z = 0;
    if (hipMemcpyAsync(st->rp[0].p, &z, 8, hipMemcpyHostToDevice, s) != hipSuccess) return fail(MCE_EDEVICE);
  }
  if (hipStreamSynchronize(s) != hipSuccess) return fail(MCE_EDEVICE);
  // the subsumed pass of a submitted batch runs on a stream of its own
  if (hipStreamCreateWithFlags(&st->sub_stream, hipStreamNonBlocking) != hipSuccess) {
    set_error("hipStreamCreateWithFlags failed");
    return fail(MCE_EDEVICE);
  }
  mce_csr dg{n, st->rp[0].as<uint64_t>(), st->col[0].as<uint32_t>(), 1};
  mce_result r;
  rc = mce_static(&dg, MCE_RANK_DEGREE, &st->opts, &r, nullptr, nullptr);
  if (rc != MCE_OK) return fail(rc);
  st->count = r.count;
  st->hash = r.set_hash;
  if (initial) *initial = r;
  *out = st;
  return MCE_OK;
}

int imce_add_edges(imce_state* st, const uint32_t* src, const uint32_t* dst, uint64_t rho, int on_device,
                   imce_result* out, mce_clique_buf* new_cl, mce_clique_buf* del_cl) {
  if (!st || !out) {
    set_error("NULL state or result");
    return MCE_EINVAL;
  }
  return update_impl(st, src, dst, rho, on_device, out, new_cl, del_cl, false);
}

int imce_remove_edges(imce_state* st, const uint32_t* src, const uint32_t* dst, uint64_t rho, int on_device,
                      imce_result* out, mce_clique_buf* new_cl, mce_clique_buf* del_cl) {
  if (!st || !out) {
    set_error("NULL state or result");
    return MCE_EINVAL;
  }
  return update_impl(st, src, dst, rho, on_device, out, new_cl, del_cl, true);
}

int imce_submit(imce_state* st, const uint32_t* src, const uint32_t* dst, uint64_t rho, int on_device, int remove) {
  if (!st) {
    set_error("NULL state");
    return MCE_EINVAL;
  }
  return submit_impl(st, src, dst, rho, on_device, remove != 0);
}

int imce_collect(imce_state* st, imce_result* out, mce_clique_buf* new_cl, mce_clique_buf* del_cl) {
  if (!st || !out) {
    set_error("NULL state or result");
    return MCE_EINVAL;
  }
  return collect_impl(st, out, new_cl, del_cl);
}

int imce_device_bytes(const imce_state* st, uint64_t* bytes) {
  if (!st || !bytes) {
    set_error("NULL state or output");
    return MCE_EINVAL;
  }
  *bytes = state_bytes(st);
  return MCE_OK;
}

int imce_batch_bytes(const imce_state* st, uint64_t rho, uint64_t* bytes) {
  if (!st || !bytes) {
    set_error("NULL state or output");
    return MCE_EINVAL;
  }
  *bytes = batch_bytes(st, rho);
  return MCE_OK;
}

int imce_info(const imce_state* st, uint64_t* n, uint64_t* nnz, uint64_t* count, uint64_t* set_hash) {
  if (!st) {
    set_error("NULL state");
    return MCE_EINVAL;
  }
  if (n) *n = st->n;
  if (nnz) *nnz = st->nnz;
  if (count) *count = st->count;
  if (set_hash) *set_hash = st->hash;
  return MCE_OK;
}

void imce_destroy(imce_state* st) {
  if (!st) return;
  release_state(st);
  delete st;
}

}  // extern "C"
