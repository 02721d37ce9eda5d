// Vertex metrics behind the rank functions of Section 4.2 (degree, core
// number, peel round, triangle count), the cost-model features, and CSR
// validation.
// All integer work; bound by HBM/L2 gathers over the adjacency.

#include <math.h>

#include "dev.h"
#include "internal.h"

namespace mce {

namespace {

__global__ void k_validate(uint64_t n, const uint64_t* __restrict__ rp, const uint32_t* __restrict__ col,
                           uint32_t* bad) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  uint64_t b = rp[v], e = rp[v + 1];
  if (e < b) { atomicOr(bad, 1u); return; }
  for (uint64_t i = b; i < e; ++i) {
    uint32_t w = col[i];
    if (w >= n || w == v || (i > b && w <= col[i - 1])) { atomicOr(bad, 2u); return; }
    uint64_t wb = rp[w], we = rp[w + 1];
    if (we < wb || bsearch_u32(col + wb, we - wb, (uint32_t)v) < 0) { atomicOr(bad, 4u); return; }
  }
}

__global__ void k_degree(uint64_t n, const uint64_t* __restrict__ rp, uint64_t* __restrict__ metric) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (v < n) metric[v] = rp[v + 1] - rp[v];
}

// --- peeling: core numbers and peel rounds -----------------------------------
// Level-synchronous peeling.  Level k starts at 0.  A round removes, all at
// once, every remaining vertex whose remaining degree is <= k; a round that
// would remove nobody instead raises k to the smallest remaining degree.  A
// round is two kernels: k_peel_mark decides who leaves from the degrees at the
// start of the round and lists the leavers, then k_peel_drop takes them out of
// their neighbours' degrees, one wave per leaver.  Each vertex gets either the
// level it left at (its core number) or the index of its round (the peel
// order); both depend on the graph only, not on the order in which waves run.
// ctl: [0] level k, [1] leavers in this round (length of the list),
//      [2] smallest remaining degree seen, [3] vertices remaining,
//      [4] round index.
constexpr uint64_t kAlive = ~0ULL;

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    uint32_t o = __shfl_xor(v, m, kWave);
    v = o < v ? o : v;
  }
  return v;
}

__global__ void k_peel_init(uint64_t n, const uint64_t* __restrict__ rp, uint32_t* deg, uint64_t* out,
                            uint64_t* ctl) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (v < n) {
    deg[v] = (uint32_t)(rp[v + 1] - rp[v]);
    out[v] = kAlive;
  }
  if (v == 0) {
    ctl[0] = 0;
    ctl[1] = 0;
    ctl[2] = ~0ULL;
    ctl[3] = n;
    ctl[4] = 0;
  }
}

// out[v] = level (core numbers) or round index (peel order) of each leaver;
// leavers go to list[0 .. ctl[1]).
__global__ void k_peel_mark(uint64_t n, const uint32_t* __restrict__ deg, uint64_t* out, uint32_t* list,
                            uint64_t* ctl, int store_level) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t k = ctl[0];
  bool leave = false;
  uint32_t stay = ~0u;  // degree of a vertex that stays, for the next level
  if (v < n && out[v] == kAlive) {
    uint32_t d = deg[v];
    if (d <= k) leave = true;
    else stay = d;
  }
  // one atomic per wave on the shared control words
  stay = wave_min_u32(stay);
  const uint64_t mask = ballot(leave);
  uint64_t base = 0;
  if (lane_id() == 0) {
    if (mask) base = atomicAdd((unsigned long long*)&ctl[1], (unsigned long long)__popcll(mask));
    if (stay != ~0u) atomicMin((unsigned long long*)&ctl[2], (unsigned long long)stay);
  }
  base = readlane64(base, 0);
  if (leave) {
    out[v] = store_level ? k : ctl[4];
    list[base + mask_prefix(mask, lane_id())] = (uint32_t)v;
  }
}

// One wave per leaver, lanes over its neighbours: a hub's neighbourhood is
// spread over the wave instead of one lane walking it.
__global__ void k_peel_drop(const uint64_t* __restrict__ rp, const uint32_t* __restrict__ col, uint32_t* deg,
                            const uint64_t* __restrict__ out, const uint32_t* __restrict__ list,
                            const uint64_t* __restrict__ ctl) {
  const uint64_t cnt = ctl[1];
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / kWave);
  const int lane = lane_id();
  for (uint64_t i = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / kWave; i < cnt; i += waves) {
    const uint32_t v = list[i];
    const uint64_t e = rp[v + 1];
    for (uint64_t j = rp[v] + lane; j < e; j += kWave) {
      uint32_t w = col[j];
      if (out[w] == kAlive) atomicSub(&deg[w], 1u);
    }
  }
}

// A round that removed nobody raises the level to the smallest remaining
// degree and keeps its index; otherwise the index advances.
__global__ void k_peel_advance(uint64_t* ctl) {
  uint64_t removed = ctl[1];
  ctl[3] -= removed;
  if (removed) ctl[4] += 1;
  else if (ctl[3] > 0) ctl[0] = ctl[2];
  ctl[1] = 0;
  ctl[2] = ~0ULL;
}

// --- triangles -------------------------------------------------------------
// One wave per vertex v.  Each triangle is found once, from its lowest vertex
// in the order (degree, id): v < u < w; all three endpoints are credited.
__device__ __forceinline__ bool deg_less(const uint64_t* rp, uint32_t a, uint32_t b) {
  uint64_t da = rp[a + 1] - rp[a], db = rp[b + 1] - rp[b];
  return da < db || (da == db && a < b);
}

__global__ void __launch_bounds__(256) k_triangles(uint64_t n, const uint64_t* __restrict__ rp,
                                                   const uint32_t* __restrict__ col, uint64_t* tri) {
  const uint64_t v = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = lane_id();
  if (v >= n) return;
  const uint64_t vb = rp[v], ve = rp[v + 1];
  uint64_t tv = 0;
  for (uint64_t i = vb; i < ve; ++i) {
    uint32_t u = col[i];
    if (!deg_less(rp, (uint32_t)v, u)) continue;
    const uint64_t ub = rp[u], ue = rp[u + 1];
    uint64_t tu = 0;
    for (uint64_t j = ub + lane; j < ue; j += kWave) {
      uint32_t w = col[j];
      if (deg_less(rp, u, w) && bsearch_u32(col + vb, ve - vb, w) >= 0) {
        ++tu;
        atomicAdd((unsigned long long*)&tri[w], 1ULL);
      }
    }
    tu = wave_sum_u64(tu);
    if (lane == 0 && tu) atomicAdd((unsigned long long*)&tri[u], (unsigned long long)tu);
    tv += tu;
  }
  if (lane == 0 && tv) atomicAdd((unsigned long long*)&tri[v], (unsigned long long)tv);
}

__global__ void k_features(uint64_t n, const uint64_t* __restrict__ rp, const uint32_t* __restrict__ col,
                           const uint64_t* __restrict__ core, const uint64_t* __restrict__ tri,
                           float* __restrict__ feat) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  uint64_t d = rp[v + 1] - rp[v];
  uint64_t walks = 0;
  for (uint64_t i = rp[v]; i < rp[v + 1]; ++i) {
    uint32_t u = col[i];
    walks += rp[u + 1] - rp[u] - 1;
  }
  feat[4 * v + 0] = log1pf((float)d);
  feat[4 * v + 1] = log1pf((float)core[v]);
  feat[4 * v + 2] = log1pf((float)tri[v]);
  feat[4 * v + 3] = log1pf((float)walks);
}

inline uint32_t blocks_for(uint64_t n, uint32_t bs) { return (uint32_t)((n + bs - 1) / bs); }

}  // namespace

// --- whole-graph TTT root (Algorithm 3 at the top level) -------------------

// The root's pivot u maximises |V n Gamma(u)| = d(u), smallest id on ties:
// the maximum of (d << 32) | (2^32 - 1 - id).
__global__ void k_root_pivot(uint64_t n, const uint64_t* __restrict__ rp, uint64_t* best) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t key = 0;
  if (v < n) key = ((rp[v + 1] - rp[v]) << 32) | (0xFFFFFFFFULL - v);
  key = wave_max_u64(key);
  if (lane_id() == 0 && key) atomicMax((unsigned long long*)best, (unsigned long long)key);
}

// metric = 0 for the root's children (ext = V \ Gamma(u), ranked by id),
// bit 63 for the pivot's neighbours, which own no subproblem and rank above
// every child (they stay in every child's cand).
__global__ void k_root_metric_clear(uint64_t n, uint64_t* metric) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (v < n) metric[v] = 0;
}

__global__ void k_root_metric_mark(const uint64_t* __restrict__ rp, const uint32_t* __restrict__ col,
                                   const uint64_t* __restrict__ best, uint64_t* metric) {
  const uint32_t u = 0xFFFFFFFFu - (uint32_t)(*best & 0xFFFFFFFFULL);
  for (uint64_t j = rp[u] + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < rp[u + 1];
       j += (uint64_t)gridDim.x * blockDim.x)
    metric[col[j]] = 1ULL << 63;
}

hipError_t launch_validate(uint64_t n, const uint64_t* rp, const uint32_t* col, uint32_t* bad, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, col, bad);
  return hipGetLastError();
}

hipError_t launch_degree(uint64_t n, const uint64_t* rp, uint64_t* metric, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_degree, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, metric);
  return hipGetLastError();
}

hipError_t launch_root_metric(uint64_t n, const uint64_t* rp, const uint32_t* col, uint64_t* metric, uint64_t* best,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipError_t e = dev_zero(best, sizeof(uint64_t), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_root_pivot, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, best);
  hipLaunchKernelGGL(k_root_metric_clear, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, metric);
  hipLaunchKernelGGL(k_root_metric_mark, dim3(64), dim3(256), 0, s, rp, col, best, metric);
  return hipGetLastError();
}

namespace {

int run_peel(uint64_t n, const uint64_t* rp, const uint32_t* col, uint64_t* out, uint32_t* deg, uint32_t* list,
             uint64_t* ctl, int store_level, hipStream_t s) {
  if (n == 0) return MCE_OK;
  const uint32_t g = blocks_for(n, 256);
  const uint32_t gd = std::min<uint32_t>(g, 2048);
  hipLaunchKernelGGL(k_peel_init, dim3(g), dim3(256), 0, s, n, rp, deg, out, ctl);
  MCE_TRY_HIP(hipGetLastError());
  // Rounds are enqueued in growing groups; the host reads the remaining count
  // only between groups.  Rounds after the last vertex left change nothing.
  uint32_t group = 16;
  for (;;) {
    for (uint32_t r = 0; r < group; ++r) {
      hipLaunchKernelGGL(k_peel_mark, dim3(g), dim3(256), 0, s, n, deg, out, list, ctl, store_level);
      hipLaunchKernelGGL(k_peel_drop, dim3(gd), dim3(256), 0, s, rp, col, deg, out, list, ctl);
      hipLaunchKernelGGL(k_peel_advance, dim3(1), dim3(1), 0, s, ctl);
    }
    MCE_TRY_HIP(hipGetLastError());
    uint64_t remaining = 0;
    MCE_TRY_HIP(hipMemcpyAsync(&remaining, ctl + 3, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    MCE_TRY_HIP(hipStreamSynchronize(s));
    if (remaining == 0) break;
    if (group < 256) group *= 2;
  }
  return MCE_OK;
}

}  // namespace

int run_core_numbers(uint64_t n, const uint64_t* rp, const uint32_t* col, uint64_t* core, uint32_t* deg,
                     uint32_t* list, uint64_t* ctl, hipStream_t s) {
  return run_peel(n, rp, col, core, deg, list, ctl, 1, s);
}

int run_peel_rounds(uint64_t n, const uint64_t* rp, const uint32_t* col, uint64_t* round, uint32_t* deg,
                    uint32_t* list, uint64_t* ctl, hipStream_t s) {
  return run_peel(n, rp, col, round, deg, list, ctl, 0, s);
}

hipError_t launch_triangles(uint64_t n, const uint64_t* rp, const uint32_t* col, uint64_t* tri, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipError_t e = dev_zero(tri, n * sizeof(uint64_t), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_triangles, dim3(blocks_for(n * 64, 256)), dim3(256), 0, s, n, rp, col, tri);
  return hipGetLastError();
}

hipError_t launch_features(uint64_t n, const uint64_t* rp, const uint32_t* col, const uint64_t* core,
                           const uint64_t* tri, float* feat, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, col, core, tri, feat);
  return hipGetLastError();
}

}  // namespace mce
