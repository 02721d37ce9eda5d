// Persistent enumeration kernel: pivoted backtracking (Algorithm 1, TTT) over
// bitset subproblems, one wavefront per task, tasks pulled from a global
// atomic queue.
//
// A task is the root of a subproblem (Algorithm 4: K = {v}, cand = the p
// higher-rank neighbours, fini = the rest; or an edge subproblem of
// Algorithm 5) or a donated continuation: a search node whose pivot and ext
// are known, with the not yet visited part of ext.  Donation is the unrolled
// child formula of Algorithm 3: child i of a node only needs
// cand \ ext[1..i-1] and fini u ext[1..i-1], which is the node's (cand, fini)
// after its first i-1 children, so a suffix of ext can be handed to another
// wave without changing the recursion tree (node counts match a sequential
// run).
//
// Two representations of a search node:
//  * wide: bitsets over the subproblem's local indices (cand 0..p-1, then the
//    relevant fini vertices), rows in the global arena, lane k holding word k
//    of P (cand), Xp (fini from cand) and ext, and word 64 + k too when cand
//    has more than 4096 vertices; Xx (fini from the root fini) lives in the
//    frame.  Frames sit in LDS when the deepest possible stack fits, else in
//    a per-wave global region.
//  * compact: once a node has |cand| <= 64 and at most 64 fini vertices with a
//    neighbour in cand, its subtree is re-based onto a 64 + 64 vertex
//    universe.  Fini vertices with no neighbour in cand never enter a child's
//    fini and can only tie as pivot when every t_u is 0, where ext = cand for
//    any pivot, so dropping them changes neither cliques nor the recursion
//    tree.  Lane l holds the compact rows of cand vertex l and fini vertex l
//    (64-bit words) in VGPRs; P, PX = P u Xp, Xx and ext are wave-uniform
//    64-bit words.
//
// Pivot (Algorithm 2): t_u = popcount(P & row_u) for every u in P u X in
// parallel, then a wave max over (t_u, smallest id) picks the pivot.

#include "dev.h"
#include "internal.h"

#include <type_traits>

namespace mce {

namespace {

constexpr uint32_t kLdsWords = 1024;  // per-wave LDS stack of the wide path: 8 KiB
constexpr uint32_t kCF = 8;           // words per compact frame
constexpr uint32_t kCFrames = 66;     // compact depth <= 64 below the re-based node

// pool record layout (64-bit words)
enum { R_S = 0, R_TYPE = 1, R_DEPTH = 2, R_KLEN = 3, R_HDR = 4 };
// compact record: a frame (kCF words) at R_HDR, then rows and tables
constexpr uint32_t kCR_PP = 12, kCR_XP = 76, kCR_PX = 140, kCR_EX = 204, kCR_KEY = 268, kCR_GP = 332, kCR_K = 364;

// Per-wave diagnostic counters (see mce_result.diag).
struct Diag {
  uint64_t rebases, cnodes, t_rebase, t_compact, t_idle, t_donate, attempts, tasks;
};

// Per-wave totals and diagnostics.  They change only at task boundaries and
// on donation attempts, so they live in the wave's LDS (lane 0 updates them)
// instead of holding 28 scalar registers for the whole kernel, registers the
// search loop needs.  Intervals are tallied as -start ... +end.
// Per-task tallies.  The algorithmic op count of a node is
// 3*s*w + 2*|ext|*w + 2*s with w fixed per subproblem, so the task keeps the
// sums of s and |ext| and multiplies once at the end (ops()).
struct Acc {
  uint64_t tn, tc, th, ssum, esum;
  uint64_t cssum, cesum;  // the part of ssum, esum from compact (re-based) nodes
  __device__ uint64_t ops(uint32_t wv) const { return (3 * ssum + 2 * esum) * wv + 2 * ssum; }
  // the same operations at the width the kernels execute: a wide node's rows
  // span the subproblem's wp 64-bit cand words, a compact node's one
  __device__ uint64_t exec_ops(uint32_t wp) const {
    const uint64_t ws = ssum - cssum, we = esum - cesum;
    return (3 * ws + 2 * we) * (2ULL * wp) + 2 * ws + (3 * cssum + 2 * cesum) * 2 + 2 * cssum;
  }
  // algorithmic LDS bytes of the formula 4 * w * (s + |ext|)
  __device__ uint64_t lds_bytes(uint32_t wv) const { return 4ULL * wv * (ssum + esum); }
  __device__ void add(const Acc& o) {
    tn += o.tn;
    tc += o.tc;
    th += o.th;
    ssum += o.ssum;
    esum += o.esum;
    cssum += o.cssum;
    cesum += o.cesum;
  }
};

struct WaveStat {
  uint64_t c, h, n, ops, xops, lds;
  Diag dg;
  Acc cacc;  // the compact search's tallies of the current task
};

__device__ __forceinline__ void stat_add(uint64_t& f, uint64_t v) {
  if (lane_id() == 0) f += v;
}

struct Lds {
  uint64_t sP[kMaxCand / 64];
  uint64_t cstk[kCFrames * kCF];
  uint32_t kG[kKLds];  // ids of K, roots first
  uint32_t xl[64];     // wide rows of the fini vertices kept by a re-base
  uint64_t hist[kHistLds];  // clique sizes tallied by this wave (when requested)
  WaveStat st;
};

// LDS of the compact kernel: frames and a K list long enough for a handed-off
// node (kHandK) plus its compact depth.
struct LdsC {
  uint64_t cstk[kCFrames * kCF];
  uint32_t kG[kHandK + kCFrames + 2];
  uint64_t hist[kHistLds];
  WaveStat st;
};

static_assert(kHistLds == kWave, "one LDS histogram bin per lane");

// One clique of k vertices into the size histogram (lane 0 of the wave).
__device__ __forceinline__ void hist_add(const EnumArgs& a, uint64_t* lhist, uint32_t k) {
  if (lane_id() == 0) {
    if (k < kHistLds)
      lhist[k] += 1;
    else
      atomicAdd((unsigned long long*)&a.hist[k < a.hist_len - 1 ? k : a.hist_len - 1], 1ULL);
  }
}

__device__ __forceinline__ void hist_clear(const EnumArgs& a, uint64_t* lhist) {
  if (a.hist) lhist[lane_id()] = 0;
}

__device__ __forceinline__ void hist_flush(const EnumArgs& a, const uint64_t* lhist) {
  if (!a.hist) return;
  __syncthreads();
  const uint32_t k = (uint32_t)lane_id();
  const uint64_t c = lhist[k];
  if (c) atomicAdd((unsigned long long*)&a.hist[k < a.hist_len - 1 ? k : a.hist_len - 1], (unsigned long long)c);
}


__device__ __forceinline__ uint64_t now() { return __builtin_readcyclecounter(); }

struct Compact {
  uint64_t rowPP, rowXP, rowPX, rowEx, zP;
  uint32_t keyP, keyX, gP;
  uint32_t np, nx;
};

// Claims the next queue slot and waits until it is filled or all work is
// done.  The wait polls with relaxed (coherent) loads: an acquire at agent
// scope invalidates the whole L2 of the XCD, which idle waves must not do
// while others compute.  One acquire fence follows a successful claim, so the
// task record written before the slot was published is visible.
__device__ __forceinline__ uint64_t claim_task(const EnumArgs& a) {
  uint64_t idx = fetch_add(&a.ctl[CTL_HEAD], 1);
  if (idx >= a.qcap) return 0;
  // back off while waiting: idle waves must not crowd the memory channel of
  // the control words that busy waves update
  uint32_t naps = 1;
  for (;;) {
    uint64_t v = ld_relaxed(&a.queue[idx]);
    if (v) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      return v;
    }
    if (ld_relaxed(&a.ctl[CTL_PENDING]) == 0) return 0;
    for (uint32_t z = 0; z < naps; ++z) __builtin_amdgcn_s_sleep(8);
    if (naps < 16) naps <<= 1;
  }
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_max(uint32_t v) {
  uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, false);
  return v > o ? v : o;
}

// Max over the 64 lanes: prefix max within rows of 16 (row_shr 1, 2, 4, 8),
// then across rows (row_bcast 15, row_bcast 31); lane 63 holds the result.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = dpp_max<0x111, 0xF>(v);
  v = dpp_max<0x112, 0xF>(v);
  v = dpp_max<0x114, 0xF>(v);
  v = dpp_max<0x118, 0xF>(v);
  v = dpp_max<0x142, 0xA>(v);
  v = dpp_max<0x143, 0xC>(v);
  return readlane32(v, 63);
}

// Waves waiting for work (claims beyond the filled queue), at most 4.
__device__ uint32_t idle_waves(const EnumArgs& a) {
  uint64_t h = 0, tl = 0;
  if (lane_id() == 0) {
    h = ld_relaxed(&a.ctl[CTL_HEAD]);
    tl = ld_relaxed(&a.ctl[CTL_TAIL]);
  }
  h = readlane64(h, 0);
  tl = readlane64(tl, 0);
  return h > tl ? (uint32_t)(h - tl < 4 ? h - tl : 4) : 0u;
}

__device__ bool starving(const EnumArgs& a) {
  uint64_t h = 0, tl = 0;
  if (lane_id() == 0) {
    h = ld_relaxed(&a.ctl[CTL_HEAD]);
    tl = ld_relaxed(&a.ctl[CTL_TAIL]);
  }
  return readlane64(h, 0) > readlane64(tl, 0);
}

constexpr uint32_t kNil = 0xFFFFFFFFu;

// Donated-task records live in fixed blocks of a pool with a lock-free free
// list (head = (tag << 32) | block, the tag defeats ABA).  A receiver copies
// its record out and returns the block at once, so the pool recycles.
//
// Ordering: a push writes the block's next link and then swings the head with
// a release CAS, so the link (and the pusher's last reads of the block) are
// complete before the block can be popped; a pop reads the head with acquire
// before it follows the link.  Without these a pop can read a stale link,
// hand one block to two donors (one record lost, another run twice) or cut
// the list short.
__device__ uint32_t pool_pop(const EnumArgs& a) {
  for (int tries = 0; tries < 64; ++tries) {
    uint64_t old = __hip_atomic_load(&a.ctl[CTL_FREE], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t idx = (uint32_t)old;
    if (idx == kNil) return kNil;
    const uint32_t nxt = __hip_atomic_load(&a.pool_next[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t nw = (((old >> 32) + 1) << 32) | nxt;
    if (__hip_atomic_compare_exchange_strong(&a.ctl[CTL_FREE], &old, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return idx;
  }
  return kNil;
}

// Returns a block whose contents the caller has finished reading.
__device__ __forceinline__ void pool_push(const EnumArgs& a, uint32_t idx) {
  for (;;) {
    uint64_t old = ld_relaxed(&a.ctl[CTL_FREE]);
    __hip_atomic_store(&a.pool_next[idx], (uint32_t)old, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t nw = (((old >> 32) + 1) << 32) | idx;
    if (__hip_atomic_compare_exchange_strong(&a.ctl[CTL_FREE], &old, nw, __ATOMIC_RELEASE, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return;
  }
}

// A queue ticket and a pool block for one donation (kNil: not now).
__device__ uint32_t reserve_record(const EnumArgs& a, bool& can_donate) {
  uint32_t blk = kNil;
  uint32_t out_of_tickets = 0;
  if (lane_id() == 0) {
    blk = pool_pop(a);
    if (blk != kNil) {
      uint64_t tk = fetch_add(&a.ctl[CTL_TICKETS], 1);
      if (tk >= a.max_tickets) {
        pool_push(a, blk);
        blk = kNil;
        out_of_tickets = 1;
      }
    }
  }
  if (readlane32(out_of_tickets, 0)) can_donate = false;
  return readlane32(blk, 0);
}

// Makes the record (plain stores of all lanes) visible at agent scope with
// one release fence, then fills a queue slot.  `pending` is raised before the
// slot is filled, and a task's own decrement comes after its donations in the
// same counter's modification order, so pending reaches zero only when no
// task is queued or running.
__device__ void publish_record(const EnumArgs& a, uint32_t blk) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (lane_id() == 0) {
    fetch_add(&a.ctl[CTL_PENDING], 1);
    uint64_t slot = fetch_add(&a.ctl[CTL_TAIL], 1);
    __hip_atomic_store(&a.queue[slot], (uint64_t)((1ULL << 63) | blk), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    fetch_add(&a.ctl[CTL_DONATED], 1);
  }
}

// The wide frames [base, top) of the current task, whose unvisited children
// can be donated while the wave works deeper (also from the compact path).
struct WideCtx {
  uint64_t* stk;
  const uint32_t* kG;  // the task's K list (LDS or the wave's global region)
  uint32_t F, wp, base, top, s, kroot;
};

// A wide node's per-lane masks (cand, fini from cand, unvisited ext, excluded
// branches) hold NW 64-bit words to a lane: word j lives in lane j % 64 of
// register j / 64, so a subproblem may have 64 * NW words of candidates.
// Word j (wave-uniform) of such a mask:
template <int NW>
__device__ __forceinline__ uint64_t word_of(const uint64_t (&v)[NW], uint32_t j) {
  if constexpr (NW == 1) {
    return readlane64(v[0], (int)j);
  } else {
    const uint64_t lo = readlane64(v[0], (int)(j & 63));
    const uint64_t hi = readlane64(v[1], (int)(j & 63));
    return (j >> 6) ? hi : lo;
  }
}

// Some word of the mask is non-zero.
template <int NW>
__device__ __forceinline__ bool any_word(const uint64_t (&v)[NW]) {
  uint64_t o = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) o |= v[i];
  return ballot(o != 0) != 0;
}

// Rank of each lane's first set bit among all set bits of a mask, in word
// order: cc[i] = this lane's bits in register i, before[i] = set bits in the
// words below word lane + 64 i; returns the total.
template <int NW>
__device__ __forceinline__ uint32_t word_ranks(const uint64_t (&v)[NW], uint32_t wp, uint32_t (&cc)[NW],
                                               uint32_t (&before)[NW]) {
  const int lane = lane_id();
  uint32_t total = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    cc[i] = (uint32_t)lane + 64u * i < wp ? (uint32_t)__popcll(v[i]) : 0u;
    const uint32_t incl = wave_incl_scan_u32(cc[i]);
    before[i] = total + incl - cc[i];
    total += readlane32(incl, 63);
  }
  return total;
}

// The lowest r bits of x.
__device__ __forceinline__ uint64_t low_bits(uint64_t x, uint32_t r) {
  uint64_t lo = 0;
  for (uint32_t z = 0; z < r; ++z) {
    lo |= x & (~x + 1);
    x &= x - 1;
  }
  return lo;
}

// Hands the second half of the shallowest wide frame's unvisited children to
// an idle wave.  Returns true if a record was queued.
template <int NW>
__device__ bool donate_wide_n(const EnumArgs& a, const WideCtx& w, bool& can_donate) {
  const int lane = lane_id();
  const uint32_t O_XP = w.wp, O_EXT = 2 * w.wp;
  uint32_t i = w.base;
  uint64_t e[NW];
  for (; i < w.top; ++i) {
#pragma unroll
    for (int r = 0; r < NW; ++r) {
      const uint32_t j = (uint32_t)lane + 64u * r;
      e[r] = j < w.wp ? w.stk[(uint64_t)i * w.F + O_EXT + j] : 0;
    }
    if (any_word(e)) break;
  }
  if (i >= w.top) return false;
  const uint32_t klen = w.kroot + i;
  const uint64_t size = R_HDR + w.F + (klen + 1) / 2;
  if (size > kBlockWords) return false;
  uint32_t cc[NW], before[NW];
  const uint32_t keep = word_ranks(e, w.wp, cc, before) / 2;
  uint64_t km[NW];  // kept: the lowest `keep` children
#pragma unroll
  for (int r = 0; r < NW; ++r) {
    const uint32_t n = keep > before[r] ? (keep - before[r] < cc[r] ? keep - before[r] : cc[r]) : 0u;
    km[r] = low_bits(e[r], n);
  }
  const uint32_t blk = reserve_record(a, can_donate);
  if (blk == kNil) return false;
  uint64_t* rec = a.pool + (uint64_t)blk * kBlockWords;
  const uint64_t* fi = w.stk + (uint64_t)i * w.F;
  __syncthreads();  // K entries written by single lanes, possibly in global memory
  if (lane == 0) {
    rec[R_S] = w.s;
    rec[R_TYPE] = 0;
    rec[R_DEPTH] = i;
    rec[R_KLEN] = klen;
  }
  // word j of P, Xp and ext: P minus the kept children, Xp plus them, ext =
  // the donated children
#pragma unroll
  for (int r = 0; r < NW; ++r) {
    const uint32_t j = (uint32_t)lane + 64u * r;
    if (j < w.wp) {
      rec[R_HDR + j] = fi[j] & ~km[r];
      rec[R_HDR + O_XP + j] = fi[O_XP + j] | km[r];
      rec[R_HDR + O_EXT + j] = e[r] & ~km[r];
    }
  }
  for (uint32_t k = 3 * w.wp + lane; k < w.F; k += kWave) rec[R_HDR + k] = fi[k];
  for (uint32_t j = lane; j < klen; j += kWave) ((uint32_t*)(rec + R_HDR + w.F))[j] = w.kG[j];
#pragma unroll
  for (int r = 0; r < NW; ++r) {
    const uint32_t j = (uint32_t)lane + 64u * r;
    if (j < w.wp) w.stk[(uint64_t)i * w.F + O_EXT + j] = km[r];
  }
  publish_record(a, blk);
  __threadfence_block();
  return true;
}

__device__ bool donate_wide(const EnumArgs& a, Lds& L, const WideCtx& w, bool& can_donate) {
  (void)L;
  return w.wp > 64 ? donate_wide_n<2>(a, w, can_donate) : donate_wide_n<1>(a, w, can_donate);
}

// Deals a root's children out at launch (mce_opts.split): `k` chunks of
// consecutive children in ascending order.  The highest chunk is queued first
// and this wave keeps the lowest ones, so a failed reservation simply leaves
// the rest here.  Each chunk is a continuation of the root whose cand lacks
// the earlier children and whose fini holds them (Algorithm 3's child
// formula), so the recursion tree is unchanged.  `fr` is the root frame with
// its fini words already in place; rExt is left holding the kept children.
template <bool EXCL, int NW>
__device__ void split_root(const EnumArgs& a, const uint32_t* kG, uint64_t* fr, uint32_t F, uint32_t wp, uint32_t s,
                           uint32_t kroot, const uint64_t (&rP)[NW], const uint64_t (&rXp)[NW], uint64_t (&rExt)[NW],
                           const uint64_t (&rF)[NW], uint64_t zsum, uint32_t k, bool& can_donate) {
  const int lane = lane_id();
  const uint32_t O_XP = wp, O_EXT = 2 * wp, O_FB = 3 * wp;
  uint32_t cc[NW], before[NW];
  const uint32_t total = word_ranks(rExt, wp, cc, before);
  const uint32_t chunks = k < total ? k : total;
  if (chunks < 2 || R_HDR + F + (kroot + 1) / 2 > kBlockWords) return;
  const uint32_t size = (total + chunks - 1) / chunks;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const uint32_t j = (uint32_t)lane + 64u * i;
    if (EXCL && j < wp) fr[O_FB + j] = rF[i];
  }
  if (lane == 0) fr[F - 1] = zsum;
  __threadfence_block();
  uint64_t keep[NW];
#pragma unroll
  for (int i = 0; i < NW; ++i) keep[i] = rExt[i];
  for (uint32_t c = chunks - 1; c >= 1 && can_donate; --c) {
    const uint32_t lo = c * size;  // rank of the chunk's first child
    if (lo >= total) continue;
    // this lane's children of rank < lo
    uint64_t below[NW], chunk[NW];
    uint64_t any = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const uint32_t r = lo > before[i] ? (lo - before[i] < cc[i] ? lo - before[i] : cc[i]) : 0u;
      below[i] = low_bits(rExt[i], r);
      chunk[i] = keep[i] & ~below[i];
      any |= chunk[i];
    }
    if (ballot(any != 0) == 0) continue;
    const uint32_t blk = reserve_record(a, can_donate);
    if (blk == kNil) break;
    uint64_t* rec = a.pool + (uint64_t)blk * kBlockWords;
    if (lane == 0) {
      rec[R_S] = s;
      rec[R_TYPE] = 0;
      rec[R_DEPTH] = 0;
      rec[R_KLEN] = kroot;
    }
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const uint32_t j = (uint32_t)lane + 64u * i;
      if (j < wp) {
        rec[R_HDR + j] = rP[i] & ~below[i];
        rec[R_HDR + O_XP + j] = rXp[i] | below[i];
        rec[R_HDR + O_EXT + j] = chunk[i];
      }
    }
    for (uint32_t q = 3 * wp + lane; q < F; q += kWave) rec[R_HDR + q] = fr[q];
    for (uint32_t q = lane; q < kroot; q += kWave) ((uint32_t*)(rec + R_HDR + F))[q] = kG[q];
    publish_record(a, blk);
#pragma unroll
    for (int i = 0; i < NW; ++i) keep[i] &= below[i];
  }
#pragma unroll
  for (int i = 0; i < NW; ++i) rExt[i] = keep[i];
}

// K is maximal: count it, hash it, and optionally write it out.
__device__ void store_clique(const EnumArgs& a, uint32_t k, const uint32_t* kG);

__device__ void emit(const EnumArgs& a, Acc& acc, uint64_t* lhist, uint64_t zsum, uint32_t k, const uint32_t* kG) {
  ++acc.tc;
  acc.th += clique_term(zsum, k);
  if (a.emit_extra) {
    if (a.cl_vert) store_clique(a, k, kG);
    if (a.hist) hist_add(a, lhist, k);
  }
}

__device__ void store_clique(const EnumArgs& a, uint32_t k, const uint32_t* kG) {
  const int lane = lane_id();
  __syncthreads();  // K entries written by single lanes, possibly in global memory
  uint64_t old = 0;
  if (lane == 0) old = fetch_add(&a.ctl[CTL_CLQ], (1ULL << 32) | k);
  old = readlane64(old, 0);
  const uint64_t id = old >> 32, pos = old & 0xFFFFFFFFULL;
  if (pos + k > 0xFFFFFFFFULL || k > kKBig) {
    if (lane == 0) atomicOr((unsigned long long*)&a.ctl[CTL_FLAGS], 2ULL);
    return;
  }
  if (id >= a.cap_cliques || pos + k > a.cap_verts) return;
  for (uint32_t j = lane; j < k; j += kWave) {
    uint32_t g = kG[j], r = 0;
    for (uint32_t i = 0; i < k; ++i) r += kG[i] < g ? 1u : 0u;
    a.cl_vert[pos + r] = g;
  }
  if (lane == 0) a.cl_off[id] = pos;
}

// --- compact path ------------------------------------------------------------

// The compact search is bound by scalar issue (one scalar instruction per CU
// per cycle) while the vector unit has room, so its tallies live in vector
// registers: every lane holds the same value.  A zero the compiler cannot see
// through moves the arithmetic that depends on it to the vector unit.
__device__ __forceinline__ uint64_t opaque_vzero64() {
  uint32_t z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return ((uint64_t)z << 32) | z;
}

// acc + popcount(x) on the vector unit, for a wave-uniform x.
__device__ __forceinline__ uint32_t vbcnt_add(uint64_t x, uint32_t acc) {
  uint32_t r, t;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(t) : "s"((uint32_t)x), "v"(acc));
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "s"((uint32_t)(x >> 32)), "v"(t));
  return r;
}

// Tallies of the compact search.  Counts decided for the whole wave (nodes,
// cliques, op terms of a node or of a set of children given as a lane mask)
// are scalar; the clique-hash terms and the op terms of single-candidate
// children are summed per lane (each lane adds the children it decides) and
// reduced over the wave once per task.
// The scalar counts are 32-bit (one instruction per add instead of two):
// one expansion adds at most 129 to any of them, and they are flushed into the
// wave's 64-bit task tallies (in LDS) at least every 2^16 + 1 expansions.
struct VTally {
  uint32_t tn, tc, ss, es;  // scalar
  uint64_t vh, vss;         // per lane
  __device__ void init() {
    tn = tc = ss = es = 0;
    vh = vss = 0;
  }
  // the scalar counts only (in the search loop)
  __device__ void flush_counts(Acc& la, Diag& dg) {
    if (lane_id() == 0) {
      la.tn += tn;
      la.tc += tc;
      la.ssum += ss;
      la.esum += es;
      la.cssum += ss;
      la.cesum += es;
      dg.cnodes += tn;
    }
    tn = tc = ss = es = 0;
  }
  // everything, the per-lane sums reduced over the wave (at the end)
  __device__ void flush(Acc& la, Diag& dg) {
    flush_counts(la, dg);
    const uint64_t h = wave_sum_u64(vh);
    const uint64_t v = wave_sum_u64(vss);
    if (lane_id() == 0) {
      la.th += h;
      la.ssum += v;
      la.cssum += v;
    }
    vh = vss = 0;
  }
};

// 64-bit value of lane `src` (per lane) through the LDS crossbar; every lane
// must be active.
__device__ __forceinline__ uint64_t bpermute64(uint64_t v, uint32_t src) {
  const int addr = (int)(src << 2);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// v in the lanes whose bit is set in the lane mask `lanes` (a wave-uniform
// 64-bit value), 0 in the others: one select with the mask as its condition.
__device__ __forceinline__ uint32_t lanes_select(uint64_t lanes, uint32_t v) {
  // the mask is wave-uniform; readfirstlane states that to the compiler so it
  // sits in a scalar register pair (free when it already does)
  const uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(lanes >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)lanes);
  uint32_t r;
  asm("v_cndmask_b32_e64 %0, 0, %1, %2" : "=v"(r) : "v"(v), "s"(m));
  return r;
}

// Frame of a compact node with deep children still to visit (kCF words):
//   0 cand P   1 PX = P u Xp         2 fini from the root fini Xx   3 ext
//   4 zsum     5 excluded-edge mask F  6 |K|                       7 D
// where D = the deep children (two or more candidates) not yet visited.  A
// child q's (cand, fini) follow from the node's by Algorithm 3's formula:
// cand = (P \ ext_{<q}) n Gamma(q), fini = (Xp u ext_{<q}) n Gamma(q) plus
// Xx n Gamma(q), with ext_{<q} the children before q (ascending).
//
// Expanding a node (Algorithm 1): the pivot by a wave max over (t_u, id),
// ext = P \ Gamma(pivot), then ONE vector pass over the children: lane q
// (q in ext) forms its child's cand and fini and decides it at once when the
// child's cand is empty (a leaf: one node, a clique iff its fini is empty) or
// holds one vertex w (one node; the grandchild K+q+w is a second node and a
// clique unless a fini vertex is adjacent to w, which then is the pivot with
// ext empty, or the branch on w is excluded).  The remaining "deep" children
// are visited in ascending order by descending into them.  The recursion
// tree, and with it every count, is the sequential one.
//
// The search keeps PX = P u Xp (Xp: the fini vertices from the cand universe)
// rather than Xp: a child's PX is PX n Gamma(q), and Xp = PX \ P.
//
// Entry: expand = true starts at the node (P, Xp, Xx) itself; expand = false
// resumes a node whose deep children D are left (a donated record).
template <bool EXCL, bool BIGK, class LT, bool EXTRA = true>
__device__ __forceinline__ void compact_dfs(const EnumArgs& a, LT& L, uint32_t* gK, const Compact& c, uint32_t s, uint64_t P,
                            uint64_t Xp, uint64_t Xx, uint64_t ext, uint64_t D, uint64_t F, uint64_t zsum,
                            bool expand, uint32_t kbase, uint32_t wv, bool& can_donate, uint32_t& since,
                            const WideCtx* wide, Diag& dg) {
  const int lane = lane_id();
  uint32_t* const kG = BIGK ? gK : L.kG;
  uint32_t d = 0;       // frames on the stack (each with deep children left)
  uint32_t kl = kbase;  // |K| of the current node
  bool framed = false;  // the current node's frame is the top of the stack
  stat_add(dg.t_compact, 0 - now());
  // search nodes between donation checks (also the tallies' flush interval)
  const uint32_t dlim = a.donate_interval < (1u << 14) ? 4 * a.donate_interval : (1u << 16);
  const uint64_t lower = (1ULL << lane) - 1;  // the children before this lane's
  uint64_t PX = P | Xp;
  VTally T;
  T.init();
  for (;;) {
    if (expand) {
      expand = false;
      framed = false;
      T.tn += 1;
      D = 0;
      if (P == 0) {
        // only a task's first node can arrive here with an empty cand
        if ((PX | Xx) == 0) {
          T.tc += 1;
          if (lane == 0) T.vh += clique_term(zsum, kl);
          if (EXTRA && a.emit_extra) {
            if (a.cl_vert) store_clique(a, kl, kG);
            if (a.hist) hist_add(a, L.hist, kl);
          }
        }
      } else {
        // pivot: largest |P n Gamma(u)| over u in P u X, smallest id on ties
        const uint32_t k1 = lanes_select(PX, ((uint32_t)__popcll(P & c.rowPP) << 16) | c.keyP);
        const uint32_t k2 = lanes_select(Xx, ((uint32_t)__popcll(P & c.rowXP) << 16) | c.keyX);
        const uint32_t mx = wave_max_u32(k1 > k2 ? k1 : k2);
        const uint32_t row = mx & 0xFFu;
        const uint64_t prow = row < 64 ? readlane64(c.rowPP, row) : readlane64(c.rowXP, row & 63);
        ext = P & ~prow;
        T.ss += (uint32_t)(__popcll(PX) + __popcll(Xx));
        T.es += (uint32_t)__popcll(ext);
        // the child pass: lane q forms child q's cand and fini; the lane masks
        // of the children that are leaves or have one candidate decide them
        const uint64_t chm = EXCL ? (ext & ~F) : ext;  // excluded q join fini unvisited
        const uint64_t below = ext & lower;
        const uint64_t cP = (P & ~below) & c.rowPP;
        // the child's PX (its Xp plus cP): for a leaf it is the child's Xp, and
        // for a one-candidate child it differs from Xp only in w, which is
        // never adjacent to itself
        const uint64_t cPX = PX & c.rowPP;
        const uint64_t cXx = Xx & c.rowPX;
        const uint32_t pc = (uint32_t)__popcll(cP);
        const uint64_t zm = ballot(pc == 0);
        const uint64_t om = ballot(pc == 1);
        const uint64_t fm = ballot((cPX | cXx) == 0);
        const uint64_t leafm = chm & zm;
        const uint64_t onem = chm & om;
        D = chm & ~(zm | om);
        uint64_t cliqm = leafm & fm;
        uint64_t grandm = 0;
        uint32_t w = 0;
        T.tn += (uint32_t)(__popcll(leafm) + __popcll(onem));
        if (onem) {
          // one candidate w: the child is one node; if no fini vertex is
          // adjacent to w (then the pivot, with ext empty) and the branch on w
          // is not excluded, the grandchild K+q+w is a second node and a clique
          w = pc ? (uint32_t)__builtin_ctzll(cP) : 0u;
          const uint64_t rw = bpermute64(c.rowPP, w);
          const uint64_t rwx = bpermute64(c.rowPX, w);
          const uint64_t blk = ballot(((cPX & rw) | (cXx & rwx)) != 0);
          uint64_t ok = onem & ~blk;
          if (EXCL) ok &= ~ballot((((F | c.rowEx) >> w) & 1ULL) != 0);
          grandm = ok;
          cliqm |= grandm;
          T.tn += (uint32_t)__popcll(grandm);
          T.es += (uint32_t)__popcll(onem & ~blk);
          // the child's pivot step, counted like an expanded node's
          if ((onem >> lane) & 1ULL) T.vss += (uint32_t)__popcll(cPX) + (uint32_t)__popcll(cXx);
        }
        if (cliqm) {
          T.tc += (uint32_t)__popcll(cliqm);
          const uint64_t zw = grandm ? bpermute64(c.zP, w) : 0ULL;
          // clique_term(zsum + z(q) [+ z(w)], |K| + 1 [+ 1]) with the sums over K
          // and the size term formed once, in scalar registers
          const uint64_t b1 = zsum + (uint64_t)(kl + 1) * kGolden;
          const uint64_t b2 = b1 + kGolden;
          if ((cliqm >> lane) & 1ULL) {
            const bool two = (grandm >> lane) & 1ULL;
            T.vh += mix64((two ? b2 + zw : b1) + c.zP);
          }
          if (EXTRA && a.emit_extra) {
            uint64_t cm = cliqm;
            while (cm) {
              const uint32_t q = (uint32_t)__builtin_ctzll(cm);
              cm &= cm - 1;
              const bool two = (grandm >> q) & 1ULL;
              if (a.cl_vert) {
                if (lane == 0) {
                  kG[kl] = readlane32(c.gP, q);
                  if (two) kG[kl + 1] = readlane32(c.gP, readlane32(w, q));
                }
                __syncthreads();  // the K list is read by every lane
                store_clique(a, kl + (two ? 2u : 1u), kG);
              }
              if (a.hist) hist_add(a, L.hist, kl + (two ? 2u : 1u));
            }
          }
        }
      }
    }
    if (D == 0) {
      // resume the nearest ancestor with deep children left
      if (d == 0) break;
      const uint64_t v = lane < (int)kCF ? L.cstk[(d - 1) * kCF + lane] : 0;
      P = readlane64(v, 0);
      PX = readlane64(v, 1);
      Xx = readlane64(v, 2);
      ext = readlane64(v, 3);
      zsum = readlane64(v, 4);
      if (EXCL) F = readlane64(v, 5);
      kl = readlane32((uint32_t)v, 6);
      D = readlane64(v, 7);
      framed = true;
    }
    // descend into the lowest deep child q
    const uint32_t q = (uint32_t)__builtin_ctzll(D);
    D &= D - 1;
    if (D) {
      if (framed) {
        if (lane == 0) L.cstk[(d - 1) * kCF + 7] = D;
      } else {
        if (lane == 0) {
          uint64_t* f = &L.cstk[d * kCF];
          f[0] = P;
          f[1] = PX;
          f[2] = Xx;
          f[3] = ext;
          f[4] = zsum;
          f[5] = EXCL ? F : 0;
          f[6] = kl;
          f[7] = D;
        }
        ++d;
      }
    } else if (framed) {
      --d;  // its last deep child: the frame's slot is free
    }
    const uint64_t below = ext & ((1ULL << q) - 1);
    const uint64_t rq = readlane64(c.rowPP, q);
    const uint64_t rqx = readlane64(c.rowPX, q);
    if (EXTRA && lane == 0) kG[kl] = readlane32(c.gP, q);  // K's ids serve only the clique output
    ++kl;
    PX &= rq;
    P = (P & ~below) & rq;
    Xx &= rqx;
    if (EXCL) F |= readlane64(c.rowEx, q);
    zsum += readlane64(c.zP, q);
    expand = true;

    if (++since >= dlim) {
      since = 0;
      T.flush_counts(L.st.cacc, dg);
    }
    if (can_donate && since == 0) {
      stat_add(dg.t_donate, 0 - now());
      for (uint32_t piece = 0, want = starving(a) ? 1u : 0u; piece < want && can_donate; ++piece) {
        stat_add(dg.attempts, 1);
        if constexpr (std::is_same<LT, Lds>::value) {
          if (wide && donate_wide(a, L, *wide, can_donate)) continue;
        }
        // the shallowest frame with two or more deep children left gives away
        // the upper half of them (it keeps at least one, so it stays a frame)
        uint32_t i = 0;
        uint64_t e = 0;
        for (; i < d; ++i) {
          e = L.cstk[i * kCF + 7];
          if (__popcll(e) >= 2) break;
        }
        if (i >= d) break;
        const uint32_t klen = (uint32_t)L.cstk[i * kCF + 6];
        if (kCR_K + (klen + 1) / 2 > kBlockWords) break;
        const uint32_t keep = (uint32_t)__popcll(e) / 2;
        uint64_t don = e;
        for (uint32_t z = 0; z < keep; ++z) don &= don - 1;
        const uint64_t km = e & ~don;  // the lowest `keep` deep children stay here
        const uint32_t blk = reserve_record(a, can_donate);
        if (blk == kNil) break;
        uint64_t* rec = a.pool + (uint64_t)blk * kBlockWords;
        if (lane == 0) {
          rec[R_S] = s;
          rec[R_TYPE] = 1;
          rec[R_DEPTH] = c.np | (c.nx << 8);
          rec[R_KLEN] = klen;
        }
        if (lane < (int)kCF) rec[R_HDR + lane] = lane == 7 ? don : L.cstk[i * kCF + lane];
        rec[kCR_PP + lane] = c.rowPP;
        rec[kCR_XP + lane] = c.rowXP;
        rec[kCR_PX + lane] = c.rowPX;
        if (EXCL) rec[kCR_EX + lane] = c.rowEx;
        rec[kCR_KEY + lane] = (uint64_t)c.keyP | ((uint64_t)c.keyX << 32);
        ((uint32_t*)(rec + kCR_GP))[lane] = c.gP;
        if (BIGK) __syncthreads();  // K entries written by single lanes in global memory
        if (EXTRA)
          for (uint32_t j = lane; j < klen; j += kWave) ((uint32_t*)(rec + kCR_K))[j] = kG[j];
        if (lane == 0) L.cstk[i * kCF + 7] = km;
        publish_record(a, blk);
      }
      stat_add(dg.t_donate, now());
    }
  }
  T.flush(L.st.cacc, dg);
  stat_add(dg.t_compact, now());
}

// Tie-break keys: rank of each compact row's vertex id among all compact rows
// (smaller id -> larger key), row index in the low byte.
__device__ void compact_keys(Compact& c) {
  const int lane = lane_id();
  uint32_t rp = 0, rx = 0;
  for (uint32_t j = 0; j < c.np; ++j) {
    const uint32_t g = readlane32(c.gP, j);
    rp += g < c.gP ? 1u : 0u;
  }
  uint32_t gX = c.keyX;  // caller stashes the fini ids here before ranking
  for (uint32_t j = 0; j < c.np; ++j) {
    const uint32_t g = readlane32(c.gP, j);
    rx += g < gX ? 1u : 0u;
  }
  for (uint32_t j = 0; j < c.nx; ++j) {
    const uint32_t g = readlane32(gX, j);
    rp += g < c.gP ? 1u : 0u;
    rx += g < gX ? 1u : 0u;
  }
  c.keyP = lane < (int)c.np ? (((255u - rp) << 8) | (uint32_t)lane) : 0u;
  c.keyX = lane < (int)c.nx ? (((255u - rx) << 8) | (64u + (uint32_t)lane)) : 0u;
  c.zP = lane < (int)c.np ? mix64(c.gP) : 0;
}

template <bool EXCL, bool EXTRA = true>
__device__ __forceinline__ void compact_from_record(const uint64_t* rec, Compact& c, uint32_t* kG, uint64_t& P, uint64_t& Xp,
                                    uint64_t& Xx, uint64_t& ext, uint64_t& D, uint64_t& zsum, uint64_t& F,
                                    uint32_t& klen) {
  const int lane = lane_id();
  const uint64_t hdr = readlane64(rec[R_DEPTH], 0);
  c.np = (uint32_t)(hdr & 0xFF);
  c.nx = (uint32_t)((hdr >> 8) & 0xFF);
  klen = (uint32_t)readlane64(rec[R_KLEN], 0);
  c.rowPP = rec[kCR_PP + lane];
  c.rowXP = rec[kCR_XP + lane];
  c.rowPX = rec[kCR_PX + lane];
  c.rowEx = EXCL ? rec[kCR_EX + lane] : 0;
  const uint64_t key = rec[kCR_KEY + lane];
  c.keyP = (uint32_t)key;
  c.keyX = (uint32_t)(key >> 32);
  c.gP = ((const uint32_t*)(rec + kCR_GP))[lane];
  c.zP = lane < (int)c.np ? mix64(c.gP) : 0;
  if (EXTRA)
    for (uint32_t j = lane; j < klen; j += kWave) kG[j] = ((const uint32_t*)(rec + kCR_K))[j];
  const uint64_t v = lane < (int)kCF ? rec[R_HDR + lane] : 0;
  P = readlane64(v, 0);
  Xp = readlane64(v, 1);
  Xx = readlane64(v, 2);
  ext = readlane64(v, 3);
  zsum = readlane64(v, 4);
  F = readlane64(v, 5);
  D = readlane64(v, 7);
}

// Handoff records (one per re-based node, for the compact kernel, which
// expands and counts it), in 64-byte units of the handoff arena:
//   word 0  s | np << 32 | nx << 40      word 1  |K|
//   word 2  zsum                         word 3  0
//   then the node's wide cand mask (wp words) and, with exclusion, its wide
//   excluded-branch mask (wp words); then as u32 the local rows of its kept
//   fini vertices (nx) and K's ids (|K| of them, only when the launch writes
//   cliques out or tallies their sizes: the search needs |K| and zsum only).
// The compact kernel gathers the compact rows and recomputes the keys.
__device__ __forceinline__ uint32_t hand_words(uint32_t wp, uint32_t nx, uint32_t klen, bool excl) {
  return 4 + (excl ? 2 : 1) * wp + (nx + klen + 1) / 2;
}

// Re-bases a wide node onto the compact 64 + 64 universe: gathers the rows of
// its candidates (the set bits of the wide mask whose word k is wordP(k), in
// ascending order) and of its kept fini vertices (local row ux, lane < nx)
// from the subproblem's bit rows.  Sets c (rows, ids, np, nx), the fini ids
// gX (lane < nx) and, with exclusion, the compact mask of candidates whose
// branch is excluded (from the wide mask whose word k is wordF(k)).
template <bool EXCL, class WordP, class WordF>
__device__ void compact_gather(const uint64_t* rowP, const uint64_t* excl, const uint32_t* gid, uint64_t nrow,
                               uint32_t wp, const WordP& wordP, const WordF& wordF, uint32_t ux,
                               uint32_t np, uint32_t nx, Compact& c, uint32_t& gX, uint64_t& Fc) {
  const int lane = lane_id();
  c.np = np;
  c.nx = nx;
  uint32_t pm = 0;  // lane j: local row of the j-th candidate
  {
    uint32_t j = 0;
    for (uint32_t k = 0; k < wp; ++k) {
      uint64_t m = wordP(k);
      while (m) {
        const uint32_t b = (uint32_t)__builtin_ctzll(m);
        if (lane == (int)j) pm = k * 64 + b;
        ++j;
        m &= m - 1;
      }
    }
  }
  uint64_t cPP = 0, cXP = 0, cEx = 0, cF = 0;
  uint32_t cnt = 0;
  for (uint32_t k = 0; k < wp; ++k) {
    uint64_t m = wordP(k);
    if (m == 0) continue;
    const uint64_t wP = lane < (int)np ? rowP[(uint64_t)k * nrow + pm] : 0;
    const uint64_t wX = lane < (int)nx ? rowP[(uint64_t)k * nrow + ux] : 0;
    const uint64_t wE = (EXCL && lane < (int)np) ? excl[(uint64_t)pm * wp + k] : 0;
    const uint64_t fk = EXCL ? wordF(k) : 0;
    while (m) {
      const uint32_t b = (uint32_t)__builtin_ctzll(m);
      cPP |= ((wP >> b) & 1ULL) << cnt;
      cXP |= ((wX >> b) & 1ULL) << cnt;
      if (EXCL) {
        cEx |= ((wE >> b) & 1ULL) << cnt;
        cF |= ((fk >> b) & 1ULL) << cnt;
      }
      ++cnt;
      m &= m - 1;
    }
  }
  c.rowPP = cPP;
  c.rowXP = cXP;
  c.rowEx = cEx;
  // cand rows over the compact fini columns = transpose of cXP
  uint64_t cPX = 0;
  for (uint32_t j = 0; j < np; ++j) {
    const uint64_t col = ballot(lane < (int)nx && ((cXP >> j) & 1ULL));
    if (lane == (int)j) cPX = col;
  }
  c.rowPX = cPX;
  c.gP = lane < (int)np ? gid[pm] : 0xFFFFFFFFu;
  gX = lane < (int)nx ? gid[ux] : 0xFFFFFFFFu;
  Fc = EXCL ? readlane64(cF, 0) : 0;
}

// Hands a re-based node to the compact kernel: one record of its subproblem,
// K, zsum, the wide masks of its candidates (and excluded branches) and the
// local rows of its kept fini vertices; the compact kernel gathers the rows
// itself (compact_gather), so a record holds no row data.  False when the
// arena or the index is full (the request still counts, so the host learns
// the size it needs).
template <bool EXCL, int NW>
__device__ bool hand_off(const EnumArgs& a, const uint32_t* kG, uint32_t s, uint32_t wp, const uint64_t (&rP)[NW],
                         const uint64_t (&rF)[NW], uint32_t ux, uint32_t np, uint32_t nx, uint64_t zsum,
                         uint32_t klen) {
  const int lane = lane_id();
  const uint32_t kst = a.emit_extra ? klen : 0u;  // K's ids serve only the clique output
  const uint32_t units = (hand_words(wp, nx, kst, EXCL) + 7) / 8;
  uint64_t old = 0;
  if (lane == 0) old = fetch_add(&a.ctl[CTL_HAND], (1ULL << 32) | units);
  old = readlane64(old, 0);
  const uint64_t idx = old >> 32, at = old & 0xFFFFFFFFULL;
  if (idx >= a.hand_cap || at + units > a.hand_units) return false;
  uint64_t* rec = a.hand + at * 8;
  __syncthreads();  // K entries written by single lanes, possibly in global memory
  if (lane == 0) {
    rec[0] = (uint64_t)s | ((uint64_t)np << 32) | ((uint64_t)nx << 40);
    rec[1] = klen;
    rec[2] = zsum;
    rec[3] = 0;
    a.hand_idx[idx] = (uint32_t)at;
    fetch_add(&a.ctl[CTL_HANDOK], 1);
  }
  uint64_t* w = rec + 4;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const uint32_t j = (uint32_t)lane + 64u * i;
    if (j < wp) w[j] = rP[i];
  }
  w += wp;
  if (EXCL) {
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const uint32_t j = (uint32_t)lane + 64u * i;
      if (j < wp) w[j] = rF[i];
    }
    w += wp;
  }
  uint32_t* u = (uint32_t*)w;
  if (lane < (int)nx) u[lane] = ux;
  for (uint32_t j = lane; j < kst; j += kWave) u[nx + j] = kG[j];
  return true;
}

// Reads a handoff record into compact form (the node still to be expanded).
template <bool EXCL, bool EXTRA, class LT>
__device__ void compact_from_hand(const EnumArgs& a, const uint64_t* rec, Compact& c, LT& L, uint64_t& P,
                                  uint64_t& Xx, uint64_t& zsum, uint64_t& F, uint32_t& klen, uint32_t& s) {
  const int lane = lane_id();
  const uint64_t h = readlane64(rec[0], 0);
  s = (uint32_t)h;
  const uint32_t np = (uint32_t)(h >> 32) & 0xFF, nx = (uint32_t)(h >> 40) & 0xFF;
  klen = (uint32_t)readlane64(rec[1], 0);
  zsum = readlane64(rec[2], 0);
  const uint32_t p = readlane32(a.sub.p[s], 0);
  const uint32_t x = readlane32(a.sub.x[s], 0);
  const uint32_t wp = (p + 63) >> 6, wx = (x + 63) >> 6;
  const uint64_t nrow = (uint64_t)p + x;
  const uint64_t* rowG = a.arena + readlane64(a.sub.off[s], 0);
  const uint64_t* excl = rowG + (uint64_t)wp * nrow + (uint64_t)p * wx;
  const uint32_t* gid = a.gids + readlane64(a.sub.goff[s], 0);
  // the record's wide masks, word k read where the gather needs it
  const uint64_t* wP = rec + 4;
  const uint64_t* wF = wP + wp;
  const uint32_t* u = (const uint32_t*)(wP + (EXCL ? 2 : 1) * wp);
  const uint32_t ux = lane < (int)nx ? u[lane] : 0;
  if (EXTRA)
    for (uint32_t j = lane; j < klen; j += kWave) L.kG[j] = u[nx + j];
  uint32_t gX;
  compact_gather<EXCL>(rowG, excl, gid, nrow, wp, [&](uint32_t k) { return wP[k]; },
                       [&](uint32_t k) { return EXCL ? wF[k] : 0ULL; }, ux, np, nx, c, gX, F);
  c.keyX = gX;
  compact_keys(c);
  P = np == 64 ? ~0ULL : ((1ULL << np) - 1);
  Xx = nx == 64 ? ~0ULL : ((1ULL << nx) - 1);
}

// One wide task: a subproblem's root or a donated wide continuation, searched
// with its node masks NW words to a lane (word j in lane j % 64 of register
// j / 64).  Descends until a node's cand fits the compact universe, then
// re-bases it (searched here, or handed to the compact kernel).
template <bool EXCL, int NW>
__device__ __forceinline__ void wide_task(const EnumArgs& a, Lds& L, uint64_t* lds_stack, uint64_t* gstk,
                                          uint32_t* gK, bool cont, uint32_t blk, const uint64_t* rec, uint32_t s,
                                          uint32_t ksplit, uint32_t p, uint32_t x, uint32_t wv, bool bigk,
                                          uint32_t* kG, uint32_t kcap, Acc& acc, bool& overflow, bool& can_donate,
                                          uint32_t& since, Diag& dg) {
  const int lane = lane_id();
  const uint32_t wp = (p + 63) >> 6, wx = (x + 63) >> 6, wf = EXCL ? wp : 0;
  const uint32_t F = 3 * wp + wf + wx + 1;
  const uint32_t O_XP = wp, O_EXT = 2 * wp, O_FB = 3 * wp, O_XX = 3 * wp + wf, O_Z = O_XX + wx;
  const uint64_t nrow = (uint64_t)p + x;
  const uint64_t* rowG = a.arena + readlane64(a.sub.off[s], 0);
  const uint64_t* rowPX = rowG + (uint64_t)wp * nrow;
  const uint64_t* excl = rowPX + (uint64_t)p * wx;
  const uint64_t* F0 = excl + (uint64_t)p * wp;
  const uint32_t* gid = a.gids + readlane64(a.sub.goff[s], 0);
  const uint32_t kroot = EXCL ? 2 : 1;
  // width class: rows over the cand columns that fit the wave's LDS row
  // cache are read from LDS for the whole task, wider ones from the arena
  const uint64_t rwords = (uint64_t)wp * nrow;
  const uint64_t* rowP = rowG;
  if (rwords <= a.lds_rows && (p > 64 || x > 64)) {
    uint64_t* cache = lds_stack + kLdsWords;
    for (uint64_t k = lane; k < rwords; k += kWave) cache[k] = rowG[k];
    __syncthreads();
    rowP = cache;
  }

  uint64_t* stk;
  uint32_t cap;
  if ((uint64_t)(p + 2) * F <= kLdsWords) {
    stk = lds_stack;
    cap = kLdsWords / F;
  } else {
    stk = gstk;
    cap = (uint32_t)(a.stack_words / F);
  }
  const uint32_t base = cont ? (uint32_t)readlane64(rec[R_DEPTH], 0) : 0u;
  overflow = base + 2 > cap || base + kroot >= kcap;

  uint64_t rP[NW], rXp[NW], rExt[NW], rF[NW];
#pragma unroll
  for (int i = 0; i < NW; ++i) rP[i] = rXp[i] = rExt[i] = rF[i] = 0;
  uint64_t zsum = 0;
  uint32_t d = base;
  uint64_t* fr = stk + (uint64_t)d * F;
  bool expand = false;
  if (!overflow) {
    if (!cont) {
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const uint32_t j = (uint32_t)lane + 64u * i;
        if (j < wp) {
          rP[i] = full_word(p, j);
          if (EXCL) rF[i] = F0[j];
        }
      }
      for (uint32_t k = lane; k < wx; k += kWave) fr[O_XX + k] = full_word(x, k);
      const uint32_t r0 = readlane32(a.sub.r0[s], 0);
      zsum = mix64(r0);
      if (lane == 0) kG[0] = r0;
      if (EXCL) {
        const uint32_t r1 = readlane32(a.sub.r1[s], 0);
        zsum += mix64(r1);
        if (lane == 0) kG[1] = r1;
      }
      expand = true;
    } else {
      const uint32_t klen = (uint32_t)readlane64(rec[R_KLEN], 0);
      for (uint32_t k = lane; k < F; k += kWave) fr[k] = rec[R_HDR + k];
      for (uint32_t j = lane; j < klen; j += kWave) kG[j] = ((const uint32_t*)(rec + R_HDR + F))[j];
      __threadfence_block();
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const uint32_t j = (uint32_t)lane + 64u * i;
        if (j < wp) {
          rP[i] = fr[j];
          rXp[i] = fr[O_XP + j];
          rExt[i] = fr[O_EXT + j];
          if (EXCL) rF[i] = fr[O_FB + j];
        }
      }
      zsum = readlane64(fr[O_Z], 0);
    }
  }
  if (cont) {
    __threadfence_block();
    if (lane == 0) pool_push(a, blk);
  }
  WideCtx wctx;
  wctx.stk = stk;
  wctx.kG = kG;
  wctx.F = F;
  wctx.wp = wp;
  wctx.base = base;
  wctx.top = base;
  wctx.s = s;
  wctx.kroot = kroot;

  while (!overflow) {
    bool do_pop = false;
    if (expand) {
      expand = false;
      if (!any_word(rP)) {
        ++acc.tn;
        // cand empty: K is maximal iff fini is empty too
        bool xe = !any_word(rXp);
        if (xe) {
          bool nz = false;
          for (uint32_t k = lane; k < wx; k += kWave) nz |= fr[O_XX + k] != 0;
          xe = ballot(nz) == 0;
        }
        if (xe) emit(a, acc, L.hist, zsum, kroot + d, kG);
        do_pop = true;
      } else {
#pragma unroll
        for (int i = 0; i < NW; ++i) {
          const uint32_t j = (uint32_t)lane + 64u * i;
          if (j < wp) L.sP[j] = rP[i];
        }
        __syncthreads();
        uint32_t p_cnt = 0;
        for (uint32_t j = 0; j < wp; ++j) p_cnt += (uint32_t)__popcll(L.sP[j]);
        // One pass over the rows of P u X: t_u for the pivot and, when
        // |cand| <= 64, the fini vertices with a neighbour in cand (the
        // vertices a re-based node keeps; give up beyond 64).
        bool ok = p_cnt <= 64 && kroot + d + kCFrames <= kcap;
        uint32_t nx = 0;
        uint64_t best = 0;
        uint32_t bu = 0;
        uint32_t s_mem = 0;
        // one 64-row chunk: member mask M, fini members MX, first row u0
        auto chunk = [&](uint64_t M, uint64_t MX, uint32_t u0) {
          s_mem += (uint32_t)__popcll(M);
          const uint32_t u = u0 + lane;
          uint32_t tu = 0;
          if ((M >> lane) & 1ULL) {
            for (uint32_t j = 0; j < wp; ++j) tu += (uint32_t)__popcll(L.sP[j] & rowP[(uint64_t)j * nrow + u]);
            const uint64_t key = ((uint64_t)tu << 32) | (0xFFFFFFFFu - gid[u]);
            if (key > best) {
              best = key;
              bu = u;
            }
          }
          if (ok) {
            const bool keepx = ((MX >> lane) & 1ULL) && tu > 0;
            const uint64_t b = ballot(keepx);
            const uint32_t cnt = (uint32_t)__popcll(b);
            if (nx + cnt > 64) {
              ok = false;
            } else {
              if (keepx) L.xl[nx + mask_prefix(b, lane)] = u;
              nx += cnt;
            }
          }
        };
        uint64_t mem[NW];
#pragma unroll
        for (int i = 0; i < NW; ++i) mem[i] = rP[i] | rXp[i];
        for (uint32_t k = 0; k < wp; ++k) {
          const uint64_t M = word_of(mem, k);
          if (M) chunk(M, word_of(rXp, k), k * 64);
        }
        // fini words of the root fini: loaded lane-parallel, only non-zero words visited
        for (uint32_t kb = 0; kb < wx; kb += kWave) {
          const uint64_t xw = kb + lane < wx ? fr[O_XX + kb + lane] : 0;
          uint64_t nzm = ballot(xw != 0);
          while (nzm) {
            const uint32_t jj = (uint32_t)__builtin_ctzll(nzm);
            nzm &= nzm - 1;
            const uint64_t M = readlane64(xw, jj);
            chunk(M, M, p + (kb + jj) * 64);
          }
        }
        bool rebased = false;
        if (ok) {
          // re-base this node and search its subtree in compact form,
          // here or (handed off) in the compact kernel
          const uint64_t tr = now();
          stat_add(dg.rebases, 1);
          __syncthreads();
          const uint32_t ux = lane < (int)nx ? L.xl[lane] : 0;
          wctx.top = d;
          const bool handed = a.hand && kroot + d <= kHandK &&
                              hand_off<EXCL, NW>(a, kG, s, wp, rP, rF, ux, p_cnt, nx, zsum, kroot + d);
          if (handed) {
            // a handed-off subtree is work done here as far as donation
            // pacing goes, else the wide frames would rarely be offered
            since += a.donate_interval / 16 + 1;
            stat_add(dg.t_rebase, now() - tr);
          } else {
            Compact c;
            uint32_t gX;
            uint64_t Fc;
            compact_gather<EXCL>(rowP, excl, gid, nrow, wp, [&](uint32_t k) { return word_of(rP, k); },
                                 [&](uint32_t k) { return word_of(rF, k); }, ux, p_cnt, nx, c, gX, Fc);
            c.keyX = gX;
            compact_keys(c);
            const uint64_t P0 = c.np == 64 ? ~0ULL : ((1ULL << c.np) - 1);
            const uint64_t X0 = nx == 64 ? ~0ULL : ((1ULL << nx) - 1);
            stat_add(dg.t_rebase, now() - tr);
            if (bigk)
              compact_dfs<EXCL, true>(a, L, gK, c, s, P0, 0, X0, 0, 0, Fc, zsum, true, kroot + d, wv, can_donate,
                                      since, &wctx, dg);
            else
              compact_dfs<EXCL, false>(a, L, gK, c, s, P0, 0, X0, 0, 0, Fc, zsum, true, kroot + d, wv, can_donate,
                                       since, &wctx, dg);
          }
          rebased = true;
          do_pop = true;
        }
        if (!rebased) {
          ++acc.tn;
          // pivot: largest |P n Gamma(u)| over u in P u X, smallest id on ties
          const uint64_t mx = wave_max_u64(best);
          const int wl = __ffsll((unsigned long long)ballot(best == mx)) - 1;
          const uint32_t piv = readlane32(bu, wl);
          uint32_t ce = 0;
#pragma unroll
          for (int i = 0; i < NW; ++i) {
            const uint32_t j = (uint32_t)lane + 64u * i;
            rExt[i] = j < wp ? (rP[i] & ~rowP[(uint64_t)j * nrow + piv]) : 0;
            ce += (uint32_t)__popcll(rExt[i]);
          }
          const uint64_t n_ext = wave_sum_u64((uint64_t)ce);
          acc.ssum += s_mem;
          acc.esum += n_ext;
          if (ksplit > 1 && !cont && d == 0)
            split_root<EXCL, NW>(a, kG, fr, F, wp, s, kroot, rP, rXp, rExt, rF, zsum, ksplit, can_donate);
        }
        __syncthreads();
      }
    }
    if (!do_pop) {
      // the lowest unvisited child q: the first word with a set bit
      uint32_t wq = kNone;
      uint64_t w = 0;
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        if (wq == kNone) {
          const uint64_t m = ballot(rExt[i] != 0);
          if (m) {
            const int kq = __ffsll((unsigned long long)m) - 1;
            w = readlane64(rExt[i], kq);
            wq = 64u * i + (uint32_t)kq;
          }
        }
      }
      if (wq == kNone) {
        do_pop = true;
      } else {
        const int b = __ffsll((unsigned long long)w) - 1;
        const uint32_t q = wq * 64 + b;
        uint64_t qb[NW];
#pragma unroll
        for (int i = 0; i < NW; ++i) {
          qb[i] = (uint32_t)lane + 64u * i == wq ? (1ULL << b) : 0;
          rExt[i] &= ~qb[i];
        }
        if (EXCL && ((word_of(rF, wq) >> b) & 1ULL)) {
          // K u {q} would contain an excluded edge: q moves to fini unvisited
#pragma unroll
          for (int i = 0; i < NW; ++i) {
            rP[i] &= ~qb[i];
            rXp[i] |= qb[i];
          }
          continue;
        }
        if (d + 2 > cap || kroot + d + 1 >= kcap) {
          overflow = true;
          break;
        }
        uint64_t cP[NW], cXp[NW], cF[NW];
#pragma unroll
        for (int i = 0; i < NW; ++i) {
          const uint32_t j = (uint32_t)lane + 64u * i;
          const uint64_t rq = j < wp ? rowP[(uint64_t)j * nrow + q] : 0;
          cP[i] = rP[i] & rq;
          cXp[i] = rXp[i] & rq;
          rP[i] &= ~qb[i];
          rXp[i] |= qb[i];
        }
        uint64_t* ch = fr + F;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
          const uint32_t j = (uint32_t)lane + 64u * i;
          if (j < wp) {
            fr[j] = rP[i];
            fr[O_XP + j] = rXp[i];
            fr[O_EXT + j] = rExt[i];
            if (EXCL) fr[O_FB + j] = rF[i];
          }
        }
        for (uint32_t k = lane; k < wx; k += kWave) ch[O_XX + k] = fr[O_XX + k] & rowPX[(uint64_t)q * wx + k];
#pragma unroll
        for (int i = 0; i < NW; ++i) {
          const uint32_t j = (uint32_t)lane + 64u * i;
          cF[i] = (EXCL && j < wp) ? (rF[i] | excl[(uint64_t)q * wp + j]) : 0;
        }
        const uint32_t gq = gid[q];
        if (lane == 0) {
          fr[O_Z] = zsum;
          kG[kroot + d] = gq;
        }
        zsum += mix64(gq);
        if (lane == 0) ch[O_Z] = zsum;
        __threadfence_block();
        fr = ch;
        ++d;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
          rP[i] = cP[i];
          rXp[i] = cXp[i];
          rF[i] = cF[i];
          rExt[i] = 0;
        }
        expand = true;

        // hand the second half of the shallowest unvisited siblings to idle waves
        if (can_donate && ++since >= a.donate_interval) {
          since = 0;
          stat_add(dg.t_donate, 0 - now());
          wctx.top = d;
          if (starving(a)) {
            stat_add(dg.attempts, 1);
            donate_wide(a, L, wctx, can_donate);
          }
          stat_add(dg.t_donate, now());
        }
        continue;
      }
    }
    // pop
    if (d == base) break;
    fr -= F;
    --d;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const uint32_t j = (uint32_t)lane + 64u * i;
      if (j < wp) {
        rP[i] = fr[j];
        rXp[i] = fr[O_XP + j];
        rExt[i] = fr[O_EXT + j];
        if (EXCL) rF[i] = fr[O_FB + j];
      }
    }
    zsum = readlane64(fr[O_Z], 0);
  }
}

// --- the kernel ---------------------------------------------------------------

template <bool EXCL>
__global__ void __launch_bounds__(64) k_enum(EnumArgs a) {
  extern __shared__ uint64_t lds_stack[];
  __shared__ Lds L;
  const int lane = threadIdx.x;
  uint64_t* const gstk = a.stacks + (uint64_t)blockIdx.x * a.stack_words;
  uint32_t* const gK = a.kbig ? a.kbig + (uint64_t)blockIdx.x * kKBig : nullptr;
  bool can_donate = a.max_tickets > 0;
  uint32_t since = 0;
  if (lane == 0) L.st = WaveStat{};
  Diag& dg = L.st.dg;
  const uint64_t t_start = now();
  hist_clear(a, L.hist);

  for (;;) {
    uint64_t ref = 0;
    const uint64_t tw = now();
    if (lane == 0) ref = claim_task(a);
    ref = readlane64(ref, 0);
    stat_add(dg.t_idle, now() - tw);
    if (ref == 0) break;
    stat_add(dg.tasks, 1);

    const bool cont = (ref >> 63) != 0;
    const uint32_t blk = cont ? (uint32_t)(ref & 0xFFFFFFFFULL) : kNil;
    const uint64_t* rec = cont ? a.pool + (uint64_t)blk * kBlockWords : nullptr;
    const uint32_t s = cont ? (uint32_t)readlane64(rec[R_S], 0) : (uint32_t)ref - 1u;
    const uint32_t ksplit = cont ? 1u : (uint32_t)(ref >> 32) & 0xFFFFu;
    const uint32_t rtype = cont ? (uint32_t)readlane64(rec[R_TYPE], 0) : 0u;
    const uint32_t p = readlane32(a.sub.p[s], 0);
    const uint32_t x = readlane32(a.sub.x[s], 0);
    const uint32_t wv = (p + x + 31) / 32;  // subproblem universe in 32-bit words
    Acc acc = {0, 0, 0, 0, 0, 0, 0};
    bool overflow = false;
    // K list: LDS unless this subproblem's cliques (at most |K at the root| +
    // p vertices) could outgrow it; then the wave's global region
    const bool bigk = gK != nullptr && (EXCL ? 2u : 1u) + p + 2 > kKLds;
    uint32_t* const kG = bigk ? gK : L.kG;
    const uint32_t kcap = bigk ? kKBig : kKLds;

    if (rtype == 1) {
      // donated compact subtree
      Compact c;
      uint64_t P, Xp, Xx, ext, D, zsum, F;
      uint32_t klen;
      compact_from_record<EXCL>(rec, c, kG, P, Xp, Xx, ext, D, zsum, F, klen);
      __syncthreads();
      if (lane == 0) pool_push(a, blk);
      if (bigk)
        compact_dfs<EXCL, true>(a, L, gK, c, s, P, Xp, Xx, ext, D, F, zsum, false, klen, wv, can_donate,
                                since, nullptr, dg);
      else
        compact_dfs<EXCL, false>(a, L, gK, c, s, P, Xp, Xx, ext, D, F, zsum, false, klen, wv, can_donate,
                                 since, nullptr, dg);
    } else {
      // masks of subproblems with more than 64 cand words take two words a lane
      if (p > 64 * 64)
        wide_task<EXCL, 2>(a, L, lds_stack, gstk, gK, cont, blk, rec, s, ksplit, p, x, wv, bigk, kG, kcap, acc,
                           overflow, can_donate, since, dg);
      else
        wide_task<EXCL, 1>(a, L, lds_stack, gstk, gK, cont, blk, rec, s, ksplit, p, x, wv, bigk, kG, kcap, acc,
                           overflow, can_donate, since, dg);
    }

    if (overflow) {
      if (lane == 0) atomicOr((unsigned long long*)&a.ctl[CTL_FLAGS], 1ULL);
    }
    if (lane == 0) {
      // the wide nodes' tallies (registers) plus the compact search's (LDS)
      Acc t = acc;
      t.add(L.st.cacc);
      L.st.cacc = Acc{};
      if (a.nodes_v) atomicAdd((unsigned long long*)&a.nodes_v[s], (unsigned long long)t.tn);
      if (a.count_v && t.tc) atomicAdd((unsigned long long*)&a.count_v[s], (unsigned long long)t.tc);
      if (a.hash_v && t.th) atomicAdd((unsigned long long*)&a.hash_v[s], (unsigned long long)t.th);
      fetch_add(&a.ctl[CTL_PENDING], ~0ULL);  // this task is done
      L.st.n += t.tn;
      L.st.c += t.tc;
      L.st.h += t.th;
      L.st.ops += t.ops(wv);
      L.st.xops += t.exec_ops((p + 63) >> 6);
      L.st.lds += t.lds_bytes(wv);
    }
  }
  hist_flush(a, L.hist);
  if (lane == 0) {
    const WaveStat& t = L.st;
    if (t.c) atomicAdd((unsigned long long*)&a.ctl[CTL_COUNT], (unsigned long long)t.c);
    if (t.h) atomicAdd((unsigned long long*)&a.ctl[CTL_HASH], (unsigned long long)t.h);
    if (t.n) atomicAdd((unsigned long long*)&a.ctl[CTL_NODES], (unsigned long long)t.n);
    if (t.ops) atomicAdd((unsigned long long*)&a.ctl[CTL_OPS], (unsigned long long)t.ops);
    if (t.xops) atomicAdd((unsigned long long*)&a.ctl[CTL_OPS_EXEC], (unsigned long long)t.xops);
    if (t.lds) atomicAdd((unsigned long long*)&a.ctl[CTL_LDS_BYTES], (unsigned long long)t.lds);
    const uint64_t t_all = now() - t_start;
    // donation inside the compact path is also inside t_compact
    const uint64_t t_wide = t_all - dg.t_idle - dg.t_rebase - dg.t_compact;
    atomicAdd((unsigned long long*)&a.ctl[CTL_DIAG + 0], (unsigned long long)dg.rebases);
    atomicAdd((unsigned long long*)&a.ctl[CTL_DIAG + 1], (unsigned long long)dg.cnodes);
    atomicAdd((unsigned long long*)&a.ctl[CTL_DIAG + 2], (unsigned long long)t_wide);
    atomicAdd((unsigned long long*)&a.ctl[CTL_DIAG + 3], (unsigned long long)dg.t_rebase);
    atomicAdd((unsigned long long*)&a.ctl[CTL_DIAG + 4], (unsigned long long)dg.t_compact);
    atomicAdd((unsigned long long*)&a.ctl[CTL_DIAG + 5], (unsigned long long)dg.t_idle);
    atomicAdd((unsigned long long*)&a.ctl[CTL_DIAG + 6], (unsigned long long)dg.t_donate);
    atomicAdd((unsigned long long*)&a.ctl[CTL_DIAG + 7], (unsigned long long)((dg.tasks << 32) | (dg.attempts & 0xFFFFFFFFULL)));
  }
}

// The compact kernel: searches handed-off re-based nodes (queue value
// bit 62 | record) and the compact donations among its own waves (bit 63 |
// pool block).  Its register footprint is a fraction of k_enum's, so many
// more waves fit per SIMD to hide the latency of the search's serial chain.
// EXTRA: the launch writes cliques out or tallies their sizes (else the
// search loop carries no test for it).
template <bool EXCL, bool EXTRA>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(7))) k_compact(EnumArgs a) {
  __shared__ LdsC L;
  const int lane = threadIdx.x;
  bool can_donate = a.max_tickets > 0;
  uint32_t since = 0;
  if (lane == 0) L.st = WaveStat{};
  Diag& dg = L.st.dg;
  hist_clear(a, L.hist);
  for (;;) {
    uint64_t ref = 0;
    const uint64_t tw = now();
    if (lane == 0) ref = claim_task(a);
    ref = readlane64(ref, 0);
    stat_add(dg.t_idle, now() - tw);
    if (ref == 0) break;
    stat_add(dg.tasks, 1);
    const bool pooled = (ref >> 63) != 0;
    const uint64_t idx = ref & 0xFFFFFFFFULL;
    Compact c;
    uint64_t P, Xp = 0, Xx, ext = 0, D = 0, zsum, F;
    uint32_t klen, s;
    if (pooled) {
      // a donation among the compact kernel's own waves
      const uint64_t* rec = a.pool + idx * kBlockWords;
      s = (uint32_t)readlane64(rec[R_S], 0);
      compact_from_record<EXCL, EXTRA>(rec, c, L.kG, P, Xp, Xx, ext, D, zsum, F, klen);
      __threadfence_block();
      if (lane == 0) pool_push(a, (uint32_t)idx);
    } else {
      const uint64_t* rec = a.hand + (uint64_t)a.hand_idx[idx] * 8;
      compact_from_hand<EXCL, EXTRA>(a, rec, c, L, P, Xx, zsum, F, klen, s);
    }
    const uint32_t p = readlane32(a.sub.p[s], 0);
    const uint32_t x = readlane32(a.sub.x[s], 0);
    const uint32_t wv = (p + x + 31) / 32;
    compact_dfs<EXCL, false, LdsC, EXTRA>(a, L, nullptr, c, s, P, Xp, Xx, ext, D, F, zsum, !pooled, klen, wv,
                                          can_donate, since, (const WideCtx*)nullptr, dg);
    if (lane == 0) {
      const Acc t = L.st.cacc;
      L.st.cacc = Acc{};
      if (a.nodes_v) atomicAdd((unsigned long long*)&a.nodes_v[s], (unsigned long long)t.tn);
      if (a.count_v && t.tc) atomicAdd((unsigned long long*)&a.count_v[s], (unsigned long long)t.tc);
      if (a.hash_v && t.th) atomicAdd((unsigned long long*)&a.hash_v[s], (unsigned long long)t.th);
      fetch_add(&a.ctl[CTL_PENDING], ~0ULL);  // this task is done
      L.st.n += t.tn;
      L.st.c += t.tc;
      L.st.h += t.th;
      L.st.ops += t.ops(wv);
      L.st.xops += t.exec_ops((p + 63) >> 6);
      L.st.lds += t.lds_bytes(wv);
    }
  }
  hist_flush(a, L.hist);
  if (lane == 0) {
    const WaveStat& t = L.st;
    if (t.c) atomicAdd((unsigned long long*)&a.ctl[CTL_COUNT], (unsigned long long)t.c);
    if (t.h) atomicAdd((unsigned long long*)&a.ctl[CTL_HASH], (unsigned long long)t.h);
    if (t.n) atomicAdd((unsigned long long*)&a.ctl[CTL_NODES], (unsigned long long)t.n);
    if (t.ops) atomicAdd((unsigned long long*)&a.ctl[CTL_OPS], (unsigned long long)t.ops);
    if (t.xops) atomicAdd((unsigned long long*)&a.ctl[CTL_OPS_EXEC], (unsigned long long)t.xops);
    if (t.lds) atomicAdd((unsigned long long*)&a.ctl[CTL_LDS_BYTES], (unsigned long long)t.lds);
    atomicAdd((unsigned long long*)&a.ctl[CTL_DIAG + 1], (unsigned long long)dg.cnodes);
    atomicAdd((unsigned long long*)&a.ctl[CTL_DIAG + 4], (unsigned long long)dg.t_compact);
    atomicAdd((unsigned long long*)&a.ctl[CTL_DIAG + 5], (unsigned long long)dg.t_idle);
    atomicAdd((unsigned long long*)&a.ctl[CTL_DIAG + 6], (unsigned long long)dg.t_donate);
    atomicAdd((unsigned long long*)&a.ctl[CTL_DIAG + 7], (unsigned long long)((dg.tasks << 32) | (dg.attempts & 0xFFFFFFFFULL)));
  }
}

__global__ void k_queue_fill_hand(uint64_t nh, const uint32_t* __restrict__ order, uint64_t* queue) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < nh) queue[i] = (1ULL << 62) | (order ? order[i] : i);
}

__global__ void k_hand_keys(uint64_t nh, const uint64_t* __restrict__ hand, const uint32_t* __restrict__ hand_idx,
                            uint32_t by_sub, uint64_t* keys, uint32_t* vals) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i >= nh) return;
  const uint64_t h = hand[(uint64_t)hand_idx[i] * 8];
  const uint64_t size = (((h >> 32) & 0xFF) << 8) | ((h >> 40) & 0xFF);
  // by subproblem: the records that gather the same rows are claimed together
  keys[i] = by_sub ? (((h & 0xFFFFFFFFULL) << 16) | size) : size;
  vals[i] = (uint32_t)i;
}

__global__ void k_finish_offsets(uint64_t* off, uint64_t nc, uint64_t nv) { off[nc] = nv; }

}  // namespace

hipError_t launch_compact(const EnumArgs& a, uint32_t grid, bool exclusion, hipStream_t s) {
  if (exclusion) {
    if (a.emit_extra)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_compact<true, true>), dim3(grid), dim3(64), 0, s, a);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_compact<true, false>), dim3(grid), dim3(64), 0, s, a);
  } else {
    if (a.emit_extra)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_compact<false, true>), dim3(grid), dim3(64), 0, s, a);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_compact<false, false>), dim3(grid), dim3(64), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_queue_fill_hand(uint64_t nh, const uint32_t* order, uint64_t* queue, hipStream_t s) {
  if (nh == 0) return hipSuccess;
  hipLaunchKernelGGL(k_queue_fill_hand, dim3((uint32_t)((nh + 255) / 256)), dim3(256), 0, s, nh, order, queue);
  return hipGetLastError();
}

hipError_t launch_hand_keys(uint64_t nh, const uint64_t* hand, const uint32_t* hand_idx, uint32_t by_sub, uint64_t* keys,
                            uint32_t* vals, hipStream_t s) {
  if (nh == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hand_keys, dim3((uint32_t)((nh + 255) / 256)), dim3(256), 0, s, nh, hand, hand_idx, by_sub, keys,
                     vals);
  return hipGetLastError();
}

hipError_t launch_enum(const EnumArgs& a, uint32_t grid, bool exclusion, hipStream_t s) {
  const size_t lds = ((size_t)kLdsWords + a.lds_rows) * sizeof(uint64_t);
  if (exclusion)
    hipLaunchKernelGGL(k_enum<true>, dim3(grid), dim3(64), lds, s, a);
  else
    hipLaunchKernelGGL(k_enum<false>, dim3(grid), dim3(64), lds, s, a);
  return hipGetLastError();
}

__global__ void k_pool_init(uint32_t* next, uint64_t blocks) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < blocks) next[i] = i + 1 < blocks ? (uint32_t)(i + 1) : 0xFFFFFFFFu;
}

hipError_t launch_pool_init(uint32_t* next, uint64_t blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_init, dim3((uint32_t)((blocks + 255) / 256)), dim3(256), 0, s, next, blocks);
  return hipGetLastError();
}

hipError_t launch_finish_offsets(uint64_t* off, uint64_t n_cliques, uint64_t n_verts, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_offsets, dim3(1), dim3(1), 0, s, off, n_cliques, n_verts);
  return hipGetLastError();
}

}  // namespace mce
