// Subproblem construction for the per-vertex decomposition (Algorithm 4):
// for each vertex v, cand(v) = neighbours of higher rank and fini(v) = the
// others.  The GPU form of G_v is a set of bit rows over local indices:
//   - cand(v) gets local indices 0..p-1 in ascending vertex id;
//   - fini vertices with at least one neighbour in cand(v) get local indices
//     p..p+x-1 in ascending vertex id (the others can never be a pivot or
//     stop an emission below the root, because every child intersects fini
//     with the neighbourhood of a cand vertex);
//   - rowP, word-major [wp][p+x]: row u restricted to the cand columns
//     (word j of row u at j*(p+x)+u), wp = ceil(p/64);
//   - rowPX, row-major [p][wx]: cand row a restricted to the fini columns,
//     wx = ceil(x/64).
// Cost: one binary search of every neighbour of every cand vertex in the
// sorted row of v (an L2/HBM gather of sum_{q in cand(v)} d(q) entries).

#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "dev.h"
#include "internal.h"

namespace mce {

namespace {

inline uint32_t blocks_for(uint64_t n, uint32_t bs) { return (uint32_t)((n + bs - 1) / bs); }

__global__ void k_sizes(uint64_t n, const uint64_t* __restrict__ rp, const uint32_t* __restrict__ col,
                        const uint64_t* __restrict__ metric, uint32_t* __restrict__ P, uint64_t* stats,
                        uint64_t* nodes_v, uint64_t* count_v, uint64_t* hash_v) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t c = 0, h = 0, nd = 0, nontriv = 0;
  uint32_t pmax = 0;
  if (v < n) {
    uint64_t b = rp[v], e = rp[v + 1];
    uint32_t p = 0;
    // bit 63 of the metric: v owns no subproblem (MCE_RANK_TTT_ROOT)
    const bool owner = !(metric[v] >> 63);
    if (owner)
      for (uint64_t i = b; i < e; ++i) p += rank_gt(metric, col[i], (uint32_t)v) ? 1u : 0u;
    P[v] = p;
    uint64_t nv = 0, cv = 0, hv = 0;
    if (!owner) {
      // no subproblem, no node
    } else if (p == 0) {
      // cand is empty: a single search node; {v} is maximal iff fini is empty
      nv = 1;
      if (e == b) {
        cv = 1;
        hv = clique_term(mix64(v), 1);
      }
      c = cv; h = hv; nd = nv;
    } else {
      nontriv = 1;
      pmax = p;
    }
    if (nodes_v) nodes_v[v] = nv;
    if (count_v) count_v[v] = cv;
    if (hash_v) hash_v[v] = hv;
  }
  c = wave_sum_u64(c);
  h = wave_sum_u64(h);
  nd = wave_sum_u64(nd);
  nontriv = wave_sum_u64(nontriv);
  uint64_t pm = wave_max_u64(pmax);
  if (lane_id() == 0) {
    if (c) atomicAdd((unsigned long long*)&stats[3], (unsigned long long)c);
    if (h) atomicAdd((unsigned long long*)&stats[4], (unsigned long long)h);
    if (nd) atomicAdd((unsigned long long*)&stats[5], (unsigned long long)nd);
    if (nontriv) atomicAdd((unsigned long long*)&stats[2], (unsigned long long)nontriv);
    if (pm) atomicMax((unsigned long long*)&stats[0], (unsigned long long)pm);
  }
}

// One wave per vertex: mark the fini positions of v's row that have a cand
// neighbour.
// The sorted neighbour list of v, which every membership test below
// searches: staged in LDS when it has at most kNbLds entries (nearly every
// vertex), so the binary searches read LDS rather than L2/HBM.  One wave per
// block, so the barrier is the wave's.
constexpr uint32_t kNbLds = 2048;

__device__ __forceinline__ const uint32_t* stage_row(const uint32_t* __restrict__ col, uint64_t vb, uint64_t d,
                                                     uint32_t* lds) {
  if (d > kNbLds) return col + vb;
  for (uint64_t i = lane_id(); i < d; i += kWave) lds[i] = col[vb + i];
  __syncthreads();
  return lds;
}

// One wave (block) per vertex.
__global__ void __launch_bounds__(64) k_mark(uint64_t n, const uint64_t* __restrict__ rp,
                                             const uint32_t* __restrict__ col, const uint64_t* __restrict__ metric,
                                             const uint32_t* __restrict__ P, uint32_t* xmark) {
  __shared__ uint32_t snb[kNbLds];
  const uint64_t v = blockIdx.x;
  const int lane = lane_id();
  if (v >= n) return;
  const uint32_t p = P[v];
  const uint64_t vb = rp[v], d = rp[v + 1] - vb;
  if (p == 0 || p == d) return;
  const uint32_t* nb = stage_row(col, vb, d, snb);
  for (uint64_t c0 = 0; c0 < d; c0 += kWave) {
    uint64_t i = c0 + lane;
    bool isP = i < d && rank_gt(metric, col[vb + i], (uint32_t)v);
    uint64_t m = ballot(isP);
    while (m) {
      int b = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const uint32_t q = col[vb + c0 + b];
      const uint64_t qb = rp[q], qe = rp[q + 1];
      for (uint64_t j = qb + lane; j < qe; j += kWave) {
        uint32_t y = col[j];
        int64_t pos = bsearch_u32(nb, d, y);
        if (pos >= 0 && !rank_gt(metric, y, (uint32_t)v)) {
          uint64_t bit = vb + (uint64_t)pos;
          atomicOr(&xmark[bit >> 5], 1u << (bit & 31));
        }
      }
    }
  }
}

__device__ __forceinline__ uint32_t count_marked(const uint32_t* xmark, uint64_t b, uint64_t e) {
  uint32_t c = 0;
  for (uint64_t i = b; i < e;) {
    uint64_t w = i >> 5;
    uint32_t lo = (uint32_t)(i & 31);
    uint64_t wend = (w + 1) << 5;
    uint64_t stop = e < wend ? e : wend;
    uint32_t hi = (uint32_t)(stop - (w << 5));  // exclusive, 1..32
    uint32_t mask = (hi == 32 ? 0xFFFFFFFFu : ((1u << hi) - 1)) & ~((1u << lo) - 1);
    c += __popc(xmark[w] & mask);
    i = stop;
  }
  return c;
}

__global__ void k_words(uint64_t n, const uint64_t* __restrict__ rp, const uint32_t* __restrict__ P,
                        const uint32_t* __restrict__ xmark, uint32_t* __restrict__ X, uint64_t* __restrict__ words,
                        uint64_t* __restrict__ gwords, uint64_t* stats) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t fw = 0;
  if (v < n) {
    uint32_t p = P[v];
    uint32_t x = 0;
    uint64_t w = 0, g = 0;
    if (p > 0) {
      x = count_marked(xmark, rp[v], rp[v + 1]);
      uint64_t wp = (p + 63) / 64, wx = (x + 63) / 64, nrow = (uint64_t)p + x;
      w = wp * nrow + (uint64_t)p * wx;
      g = nrow;
      fw = 3 * wp + wx + 1;
    }
    X[v] = x;
    words[v] = w;
    gwords[v] = g;
  }
  fw = wave_max_u64(fw);
  if (lane_id() == 0 && fw) atomicMax((unsigned long long*)&stats[1], (unsigned long long)fw);
}

constexpr uint32_t kLidxP = 0x80000000u;
constexpr uint32_t kLidxNone = 0x7FFFFFFFu;

// One wave (block) per vertex with a non-empty cand: vertex-id table and bit rows.
__global__ void __launch_bounds__(64) k_build(uint64_t n, const uint64_t* __restrict__ rp,
                                              const uint32_t* __restrict__ col, const uint64_t* __restrict__ metric,
                                              const uint32_t* __restrict__ P, const uint32_t* __restrict__ X,
                                              const uint32_t* __restrict__ xmark, uint32_t* __restrict__ lidx,
                                              const uint64_t* __restrict__ off, const uint64_t* __restrict__ goff,
                                              uint64_t* arena, uint32_t* __restrict__ gids) {
  __shared__ uint32_t snb[kNbLds];
  const uint64_t v = blockIdx.x;
  const int lane = lane_id();
  if (v >= n) return;
  const uint32_t p = P[v];
  if (p == 0) return;
  const uint32_t x = X[v];
  const uint64_t vb = rp[v], d = rp[v + 1] - vb;
  const uint32_t* nb = stage_row(col, vb, d, snb);
  const uint64_t wp = (p + 63) / 64, wx = (x + 63) / 64, nrow = (uint64_t)p + x;
  uint64_t* rowP = arena + off[v];
  uint64_t* rowPX = rowP + wp * nrow;
  uint32_t* gid = gids + goff[v];
  // pass 1: local indices, ascending vertex id within cand and within fini'
  uint32_t cp = 0, cx = 0;
  for (uint64_t c0 = 0; c0 < d; c0 += kWave) {
    uint64_t i = c0 + lane;
    bool valid = i < d;
    uint32_t w = valid ? col[vb + i] : 0;
    bool isP = valid && rank_gt(metric, w, (uint32_t)v);
    bool isX = valid && !isP && ((xmark[(vb + i) >> 5] >> ((vb + i) & 31)) & 1u);
    uint64_t mP = ballot(isP), mX = ballot(isX);
    if (isP) {
      uint32_t a = cp + mask_prefix(mP, lane);
      gid[a] = w;
      lidx[vb + i] = a | kLidxP;
    } else if (isX) {
      uint32_t c = cx + mask_prefix(mX, lane);
      gid[p + c] = w;
      lidx[vb + i] = c;
    } else if (valid) {
      lidx[vb + i] = kLidxNone;
    }
    cp += (uint32_t)__popcll(mP);
    cx += (uint32_t)__popcll(mX);
  }
  __threadfence();
  // pass 2: rows of the cand vertices, in local order a = 0..p-1
  uint32_t a = 0;
  for (uint64_t c0 = 0; c0 < d; c0 += kWave) {
    uint64_t i = c0 + lane;
    bool isP = i < d && rank_gt(metric, col[vb + i], (uint32_t)v);
    uint64_t m = ballot(isP);
    while (m) {
      int b = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const uint32_t q = col[vb + c0 + b];
      const uint64_t qb = rp[q], qe = rp[q + 1];
      for (uint64_t j = qb + lane; j < qe; j += kWave) {
        uint32_t y = col[j];
        int64_t pos = bsearch_u32(nb, d, y);
        if (pos < 0) continue;
        uint32_t L = lidx[vb + pos];
        if (L & kLidxP) {
          uint32_t a2 = L & ~kLidxP;
          atomicOr((unsigned long long*)&rowP[(uint64_t)(a2 >> 6) * nrow + a], 1ULL << (a2 & 63));
        } else if (L != kLidxNone) {
          uint32_t c = L;
          atomicOr((unsigned long long*)&rowPX[(uint64_t)a * wx + (c >> 6)], 1ULL << (c & 63));
          atomicOr((unsigned long long*)&rowP[(uint64_t)(a >> 6) * nrow + p + c], 1ULL << (a & 63));
        }
      }
      ++a;
    }
  }
}

// Queue keys: non-trivial subproblems get (1 << 63) | primary, trivial ones 0,
// so a stable descending sort puts the queue first, ties in ascending id.
__global__ void k_queue_keys(uint64_t n, const uint64_t* __restrict__ rp, const uint32_t* __restrict__ P, int sched,
                             const uint64_t* __restrict__ tri, const float* __restrict__ cost, uint64_t* keys,
                             uint32_t* vals) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  uint64_t key = 0;
  if (P[v] > 0) {
    uint64_t prim;
    switch (sched) {
      case MCE_SCHED_TRIANGLE: prim = tri[v]; break;
      case MCE_SCHED_COST: {
        // order-preserving map of the float onto 32 bits; NaN sorts last
        const float c = cost[v];
        const uint32_t u = __float_as_uint(c);
        prim = (c != c) ? 0 : (uint64_t)((u & 0x80000000u) ? ~u : (u | 0x80000000u));
        break;
      }
      case MCE_SCHED_ID: prim = 0xFFFFFFFFull - v; break;
      default: prim = rp[v + 1] - rp[v]; break;
    }
    key = (1ULL << 63) | (prim & ~(1ULL << 63));
  }
  keys[v] = key;
  vals[v] = (uint32_t)v;
}

// Root task of subproblem v: v + 1, with its chunk count in bits 32..47 when
// the root is to be split.
__global__ void k_queue_fill(uint64_t nq, const uint32_t* __restrict__ vals, const uint32_t* __restrict__ split,
                             uint64_t* queue) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const uint32_t v = vals[i];
  const uint64_t k = split ? split[v] : 1u;
  queue[i] = (k > 1 ? (k << 32) : 0) | ((uint64_t)v + 1);
}

// Predicted work of subproblem v: exp(cost[v]), cost = predicted log search
// nodes (clamped to a finite range; NaN counts as no work).
__device__ __forceinline__ double predicted_work(float c) {
  if (!(c == c)) return 0.0;
  return exp((double)fminf(fmaxf(c, -80.0f), 80.0f));
}

__global__ void k_split_total(uint64_t n, const uint32_t* __restrict__ P, const float* __restrict__ cost,
                              double* total) {
  double w = 0.0;
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x)
    if (P[v] > 0) w += predicted_work(cost[v]);
  for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o);
  if (lane_id() == 0 && w != 0.0) atomicAdd(total, w);
}

// chunks = ceil(work / share), share = total / waves, at most split_max.
__global__ void k_split_plan(uint64_t n, const uint32_t* __restrict__ P, const float* __restrict__ cost,
                             const double* __restrict__ total, uint32_t waves, uint32_t split_max, uint32_t* split) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  uint32_t k = 1;
  const double share = *total / (double)waves;
  if (P[v] > 1 && share > 0.0) {
    const double c = ceil(predicted_work(cost[v]) / share);
    k = c >= (double)split_max ? split_max : (c > 1.0 ? (uint32_t)c : 1u);
  }
  split[v] = k;
}

}  // namespace

hipError_t launch_sizes(uint64_t n, const uint64_t* rp, const uint32_t* col, const uint64_t* metric, BuildBufs b,
                        uint64_t* nodes_v, uint64_t* count_v, uint64_t* hash_v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sizes, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, col, metric, b.p, b.stats, nodes_v,
                     count_v, hash_v);
  return hipGetLastError();
}

hipError_t launch_mark(uint64_t n, const uint64_t* rp, const uint32_t* col, const uint64_t* metric, BuildBufs b,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark, dim3((uint32_t)n), dim3(64), 0, s, n, rp, col, metric, b.p, b.xmark);
  return hipGetLastError();
}

hipError_t launch_words(uint64_t n, const uint64_t* rp, BuildBufs b, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_words, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, b.p, b.xmark, b.x, b.words,
                     b.gwords, b.stats);
  return hipGetLastError();
}

hipError_t launch_build(uint64_t n, const uint64_t* rp, const uint32_t* col, const uint64_t* metric, BuildBufs b,
                        const uint64_t* off, const uint64_t* goff, uint64_t* arena, uint32_t* gids, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_build, dim3((uint32_t)n), dim3(64), 0, s, n, rp, col, metric, b.p, b.x,
                     b.xmark, b.lidx, off, goff, arena, gids);
  return hipGetLastError();
}

hipError_t launch_queue_keys(uint64_t n, const uint64_t* rp, const uint32_t* p, mce_sched sched, const uint64_t* tri,
                             const float* cost, uint64_t* keys, uint32_t* vals, uint64_t* /*count*/,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_queue_keys, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, p, (int)sched, tri, cost, keys,
                     vals);
  return hipGetLastError();
}

hipError_t launch_queue_fill(uint64_t nq, const uint32_t* vals, const uint32_t* split, uint64_t* queue,
                             hipStream_t s) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_queue_fill, dim3(blocks_for(nq, 256)), dim3(256), 0, s, nq, vals, split, queue);
  return hipGetLastError();
}

hipError_t launch_split_plan(uint64_t n, const uint32_t* p, const float* cost, uint32_t waves, uint32_t split_max,
                             double* total, uint32_t* split, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipError_t e = dev_zero(total, sizeof(double), s);
  if (e != hipSuccess) return e;
  const uint32_t blocks = std::min<uint32_t>(blocks_for(n, 256), 1024);
  hipLaunchKernelGGL(k_split_total, dim3(blocks), dim3(256), 0, s, n, p, cost, total);
  hipLaunchKernelGGL(k_split_plan, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, p, cost, total, waves,
                     split_max, split);
  return hipGetLastError();
}

int device_exclusive_scan(const uint64_t* in, uint64_t* out, uint64_t n, void*& tmp, size_t& tmp_bytes,
                          hipStream_t s) {
  size_t need = 0;
  MCE_TRY_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, need, in, out, (int)n, s));
  MCE_TRY(ensure_temp(tmp, tmp_bytes, need));
  MCE_TRY_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, need, in, out, (int)n, s));
  return MCE_OK;
}

int device_sort_desc(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, uint64_t n, void*& tmp,
                     size_t& tmp_bytes, hipStream_t s, uint64_t** keys_out, uint32_t** vals_out, int end_bit) {
  hipcub::DoubleBuffer<uint64_t> kb(keys, keys_alt);
  hipcub::DoubleBuffer<uint32_t> vb(vals, vals_alt);
  size_t need = 0;
  MCE_TRY_HIP(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, need, kb, vb, (int)n, 0, end_bit, s));
  MCE_TRY(ensure_temp(tmp, tmp_bytes, need));
  MCE_TRY_HIP(hipcub::DeviceRadixSort::SortPairsDescending(tmp, need, kb, vb, (int)n, 0, end_bit, s));
  *keys_out = kb.Current();
  *vals_out = vb.Current();
  return MCE_OK;
}

}  // namespace mce
