// Device-side helpers for the gfx950 kernels: hashing, 64-lane wave
// primitives and agent-scope atomics.  Everything here is integer work.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mce {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ULL;
constexpr int kWave = 64;

// splitmix64 output function: the per-vertex term and the per-clique mix of
// the clique-set hash.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x += kGolden;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

__device__ __forceinline__ uint64_t clique_term(uint64_t zsum, uint64_t k) { return mix64(zsum + k * kGolden); }

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p); }

// Broadcast lane `l`'s 64-bit value (l wave-uniform).
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
  uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t readlane32(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    uint64_t o = __shfl_xor(v, m, kWave);
    v = o > v ? o : v;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

// Inclusive prefix sum across the wave.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

// Number of set bits of `mask` below lane l (exclusive prefix of a ballot).
__device__ __forceinline__ uint32_t mask_prefix(uint64_t mask, int l) {
  return (uint32_t)__popcll(mask & ((l == 0) ? 0ULL : (~0ULL >> (64 - l))));
}

// Word k of the bitset {0..nbits-1}.
__device__ __forceinline__ uint64_t full_word(uint32_t nbits, uint32_t k) {
  uint32_t lo = k * 64;
  if (lo >= nbits) return 0;
  uint32_t r = nbits - lo;
  return r >= 64 ? ~0ULL : ((1ULL << r) - 1);
}

template <class T>
__device__ __forceinline__ T ld_acquire(T* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T ld_relaxed(T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_release(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t fetch_add(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// rank(w) > rank(v) for rank = (metric, id), lexicographic.
__device__ __forceinline__ bool rank_gt(const uint64_t* metric, uint32_t w, uint32_t v) {
  uint64_t mw = metric[w], mv = metric[v];
  return mw > mv || (mw == mv && w > v);
}

// Position of x in the sorted array a[0..n), or -1.
__device__ __forceinline__ int64_t bsearch_u32(const uint32_t* a, uint64_t n, uint32_t x) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    uint64_t mid = (lo + hi) >> 1;
    uint32_t y = a[mid];
    if (y < x) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n && a[lo] == x) ? (int64_t)lo : -1;
}

}  // namespace mce
