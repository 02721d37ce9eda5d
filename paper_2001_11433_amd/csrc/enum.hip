// Persistent enumeration kernel: pivoted backtracking (Algorithm 1, TTT) over
// bitset subproblems, one wavefront per task, tasks pulled from a global
// atomic queue.
//
// A task is either the root of a subproblem (Algorithm 4: K = {v},
// cand = the p higher-rank neighbours, fini = the rest) or a donated
// continuation: a search node whose pivot and ext were already computed,
// together with the not yet visited part of ext.  Donation is the unrolled
// child formula of Algorithm 3: child i of a node only needs
// cand \ ext[1..i-1] and fini u ext[1..i-1], which is exactly the node's
// (cand, fini) after its first i-1 children, so a suffix of ext can be handed
// to another wave without changing the recursion tree (node counts match a
// sequential run).
//
// Search state of a node (one "frame"), in 64-bit words:
//   P    [wp]  cand, over the local cand indices 0..p-1
//   Xp   [wp]  the part of fini that came from cand (earlier siblings)
//   ext  [wp]  children not yet visited
//   Fb   [wf]  edge subproblems only: vertices whose addition would complete an
//              excluded edge (Algorithms 6 and 8)
//   Xx   [wx]  the part of fini from the subproblem's root fini
//   z    [1]   sum of mix(id) over K (for the clique hash)
//   q    [1]   the local vertex added to reach this node
// Lane k of the wave holds word k of P, Xp, ext and Fb in registers (p <=
// 4096, so wp <= 64).  Frames live in LDS when the subproblem's deepest
// possible stack fits, else in a per-wave global region.
//
// Pivot (Algorithm 2): lanes take the candidate rows u in P u X, 64 at a
// time, and compute t_u = sum_j popcount(P[j] & row_u[j]); a wave max over
// (t_u, ~id(u)) picks the largest t_u, smallest id on ties.

#include "dev.h"
#include "internal.h"

namespace mce {

namespace {

constexpr uint32_t kKMax = 1024;     // largest materialised clique
constexpr uint32_t kLdsWords = 1536; // per-wave LDS stack: 12 KiB

struct Task {
  uint32_t s;     // subproblem
  uint32_t base;  // depth of the task's first frame
  bool cont;
  const uint64_t* rec;
};

__device__ uint64_t claim_task(const EnumArgs& a) {
  uint64_t idx = fetch_add(&a.ctl[CTL_HEAD], 1);
  if (idx >= a.qcap) return 0;
  for (;;) {
    uint64_t v = ld_acquire(&a.queue[idx]);
    if (v) return v;
    if (ld_acquire(&a.ctl[CTL_PENDING]) == 0) return 0;
    __builtin_amdgcn_s_sleep(8);
  }
}

template <bool EXCL>
__global__ void __launch_bounds__(64) k_enum(EnumArgs a) {
  extern __shared__ uint64_t lds_stack[];
  __shared__ uint64_t sP[64];
  __shared__ uint32_t sK[kKMax];
  const int lane = threadIdx.x;
  uint64_t* const gstk = a.stacks + (uint64_t)blockIdx.x * a.stack_words;
  uint64_t tot_c = 0, tot_h = 0, tot_n = 0;
  bool can_donate = a.max_tickets > 0;

  for (;;) {
    uint64_t ref = 0;
    if (lane == 0) ref = claim_task(a);
    ref = readlane64(ref, 0);
    if (ref == 0) break;

    Task t;
    t.cont = (ref >> 63) != 0;
    if (!t.cont) {
      t.s = (uint32_t)(ref - 1);
      t.base = 0;
      t.rec = nullptr;
    } else {
      t.rec = a.pool + (ref & ~(1ULL << 63));
      t.s = (uint32_t)readlane64(t.rec[0], 0);
      t.base = (uint32_t)readlane64(t.rec[1], 0);
    }
    const uint32_t s = t.s;
    const uint32_t p = readlane32(a.sub.p[s], 0);
    const uint32_t x = readlane32(a.sub.x[s], 0);
    const uint32_t wp = (p + 63) >> 6, wx = (x + 63) >> 6, wf = EXCL ? wp : 0;
    const uint32_t F = 3 * wp + wf + wx + 2;
    const uint32_t O_XP = wp, O_EXT = 2 * wp, O_FB = 3 * wp, O_XX = 3 * wp + wf, O_Z = O_XX + wx, O_Q = O_Z + 1;
    const uint64_t nrow = (uint64_t)p + x;
    const uint64_t* rowP = a.arena + readlane64(a.sub.off[s], 0);
    const uint64_t* rowPX = rowP + (uint64_t)wp * nrow;
    const uint64_t* excl = rowPX + (uint64_t)p * wx;
    const uint64_t* F0 = excl + (uint64_t)p * wp;
    const uint32_t* gid = a.gids + readlane64(a.sub.goff[s], 0);
    const uint32_t r0 = readlane32(a.sub.r0[s], 0);
    const uint32_t r1 = EXCL ? readlane32(a.sub.r1[s], 0) : 0;
    const uint32_t kroot = EXCL ? 2 : 1;

    // deepest absolute frame index is p (one cand vertex per level)
    uint64_t* stk;
    uint32_t cap;
    if ((uint64_t)(p + 2) * F <= kLdsWords) {
      stk = lds_stack;
      cap = kLdsWords / F;
    } else {
      stk = gstk;
      cap = (uint32_t)(a.stack_words / F);
    }
    uint64_t tn = 0, tc = 0, th = 0;
    bool overflow = t.base + 2 > cap;

    uint64_t rP = 0, rXp = 0, rExt = 0, rF = 0, zsum = 0;
    uint32_t d = t.base;
    uint64_t* fr = stk + (uint64_t)d * F;
    bool expand = false;
    if (!overflow) {
      if (!t.cont) {
        rP = lane < (int)wp ? full_word(p, lane) : 0;
        if (EXCL && lane < (int)wp) rF = F0[lane];
        for (uint32_t k = lane; k < wx; k += kWave) fr[O_XX + k] = full_word(x, k);
        zsum = mix64(r0) + (EXCL ? mix64(r1) : 0);
        expand = true;
      } else {
        const uint64_t* rf = t.rec + 2;
        for (uint32_t k = lane; k < F; k += kWave) fr[k] = rf[k];
        const uint32_t* rq = (const uint32_t*)(t.rec + 2 + F);
        for (uint32_t i = lane; i + 1 < t.base; i += kWave) stk[(uint64_t)(i + 1) * F + O_Q] = rq[i];
        __threadfence_block();
        if (lane < (int)wp) {
          rP = fr[lane];
          rXp = fr[O_XP + lane];
          rExt = fr[O_EXT + lane];
          if (EXCL) rF = fr[O_FB + lane];
        }
        zsum = readlane64(fr[O_Z], 0);
      }
    }
    uint32_t since = 0;

    while (!overflow) {
      bool do_pop = false;
      if (expand) {
        expand = false;
        ++tn;
        if (ballot(rP != 0) == 0) {
          // cand empty: K is maximal iff fini is empty too
          bool xe = ballot(rXp != 0) == 0;
          if (xe) {
            bool nz = false;
            for (uint32_t k = lane; k < wx; k += kWave) nz |= fr[O_XX + k] != 0;
            xe = ballot(nz) == 0;
          }
          if (xe) {
            const uint32_t k = kroot + (d);
            ++tc;
            th += clique_term(zsum, k);
            if (a.cl_vert) {
              uint64_t old = 0;
              if (lane == 0) old = fetch_add(&a.ctl[CTL_CLQ], (1ULL << 32) | k);
              old = readlane64(old, 0);
              const uint64_t id = old >> 32, pos = old & 0xFFFFFFFFULL;
              if (pos + k > 0xFFFFFFFFULL || k > kKMax) {
                if (lane == 0) atomicOr((unsigned long long*)&a.ctl[CTL_FLAGS], 2ULL);
              } else if (id < a.cap_cliques && pos + k <= a.cap_verts) {
                if (lane == 0) {
                  sK[0] = r0;
                  if (EXCL) sK[1] = r1;
                }
                for (uint32_t i = lane + 1; i <= d; i += kWave)
                  sK[kroot + i - 1] = gid[(uint32_t)stk[(uint64_t)i * F + O_Q]];
                __syncthreads();
                for (uint32_t j = lane; j < k; j += kWave) {
                  uint32_t g = sK[j], r = 0;
                  for (uint32_t i = 0; i < k; ++i) r += sK[i] < g ? 1u : 0u;
                  a.cl_vert[pos + r] = g;
                }
                if (lane == 0) a.cl_off[id] = pos;
                __syncthreads();
              }
            }
          }
          do_pop = true;
        } else {
          // pivot: argmax over u in P u X of |P n Gamma(u)|, smallest id on ties
          if (lane < (int)wp) sP[lane] = rP;
          __syncthreads();
          uint64_t best = 0;
          uint32_t bu = 0;
          const uint64_t mem = rP | rXp;
          for (uint32_t k = 0; k < wp; ++k) {
            const uint64_t M = readlane64(mem, k);
            if (M == 0) continue;
            if ((M >> lane) & 1ULL) {
              const uint32_t u = k * 64 + lane;
              uint32_t tu = 0;
              for (uint32_t j = 0; j < wp; ++j) tu += (uint32_t)__popcll(sP[j] & rowP[(uint64_t)j * nrow + u]);
              const uint64_t key = ((uint64_t)tu << 32) | (0xFFFFFFFFu - gid[u]);
              if (key > best) { best = key; bu = u; }
            }
          }
          for (uint32_t k = 0; k < wx; ++k) {
            const uint64_t M = fr[O_XX + k];
            if (M == 0) continue;
            if ((M >> lane) & 1ULL) {
              const uint32_t u = p + k * 64 + lane;
              uint32_t tu = 0;
              for (uint32_t j = 0; j < wp; ++j) tu += (uint32_t)__popcll(sP[j] & rowP[(uint64_t)j * nrow + u]);
              const uint64_t key = ((uint64_t)tu << 32) | (0xFFFFFFFFu - gid[u]);
              if (key > best) { best = key; bu = u; }
            }
          }
          const uint64_t mx = wave_max_u64(best);
          const int wl = __ffsll((unsigned long long)ballot(best == mx)) - 1;
          const uint32_t piv = readlane32(bu, wl);
          rExt = lane < (int)wp ? (rP & ~rowP[(uint64_t)lane * nrow + piv]) : 0;
          __syncthreads();
        }
      }
      if (!do_pop) {
        const uint64_t m = ballot(rExt != 0);
        if (m == 0) {
          do_pop = true;
        } else {
          const int kq = __ffsll((unsigned long long)m) - 1;
          const uint64_t w = readlane64(rExt, kq);
          const int b = __ffsll((unsigned long long)w) - 1;
          const uint32_t q = (uint32_t)kq * 64 + b;
          const uint64_t qb = lane == kq ? (1ULL << b) : 0;
          rExt &= ~qb;
          if (EXCL && ((readlane64(rF, kq) >> b) & 1ULL)) {
            // K u {q} would contain an excluded edge: q moves to fini unvisited
            rP &= ~qb;
            rXp |= qb;
            continue;
          }
          if (d + 2 > cap) {
            overflow = true;
            break;
          }
          const uint64_t rq = lane < (int)wp ? rowP[(uint64_t)lane * nrow + q] : 0;
          const uint64_t cP = rP & rq, cXp = rXp & rq;
          rP &= ~qb;
          rXp |= qb;
          uint64_t* ch = fr + F;
          if (lane < (int)wp) {
            fr[lane] = rP;
            fr[O_XP + lane] = rXp;
            fr[O_EXT + lane] = rExt;
            if (EXCL) fr[O_FB + lane] = rF;
          }
          for (uint32_t k = lane; k < wx; k += kWave) ch[O_XX + k] = fr[O_XX + k] & rowPX[(uint64_t)q * wx + k];
          uint64_t cF = 0;
          if (EXCL && lane < (int)wp) cF = rF | excl[(uint64_t)q * wp + lane];
          fr[O_Z] = zsum;  // (same value from every lane)
          zsum += mix64(gid[q]);
          if (lane == 0) {
            ch[O_Z] = zsum;
            ch[O_Q] = q;
          }
          __threadfence_block();
          fr = ch;
          ++d;
          rP = cP;
          rXp = cXp;
          rF = cF;
          rExt = 0;
          expand = true;

          // hand the second half of the shallowest unvisited siblings to idle waves
          if (can_donate && ++since >= a.donate_interval) {
            since = 0;
            uint64_t h = 0, tl = 0;
            if (lane == 0) {
              h = ld_relaxed(&a.ctl[CTL_HEAD]);
              tl = ld_relaxed(&a.ctl[CTL_TAIL]);
            }
            h = readlane64(h, 0);
            tl = readlane64(tl, 0);
            if (h > tl) {
              uint32_t i = t.base;
              uint64_t e = 0;
              for (; i < d; ++i) {
                e = lane < (int)wp ? stk[(uint64_t)i * F + O_EXT + lane] : 0;
                if (ballot(e != 0)) break;
              }
              if (i < d) {
                const uint32_t c = (uint32_t)__popcll(e);
                const uint32_t incl = wave_incl_scan_u32(c);
                const uint32_t total = readlane32(incl, 63);
                const uint32_t keep = total / 2;
                const uint32_t before = incl - c;
                uint32_t r = keep > before ? (keep - before < c ? keep - before : c) : 0;
                uint64_t rest = e;
                for (uint32_t z = 0; z < r; ++z) rest &= rest - 1;
                const uint64_t km = e & ~rest;  // kept: the lowest `keep` children
                const uint64_t don = rest;
                const uint64_t size = 2 + F + (i + 1) / 2;
                uint64_t off = 0;
                uint32_t ok = 0;
                if (lane == 0) {
                  uint64_t tk = fetch_add(&a.ctl[CTL_TICKETS], 1);
                  if (tk < a.max_tickets) {
                    off = fetch_add(&a.ctl[CTL_POOL], size);
                    ok = off + size <= a.pool_cap;
                  }
                }
                ok = readlane32(ok, 0);
                off = readlane64(off, 0);
                if (!ok) {
                  can_donate = false;
                } else {
                  uint64_t* rec = a.pool + off;
                  const uint64_t* fi = stk + (uint64_t)i * F;
                  if (lane == 0) {
                    rec[0] = s;
                    rec[1] = i;
                  }
                  // lane j owns word j of P, Xp and ext: P minus the kept
                  // children, Xp plus them, ext = the donated children
                  if (lane < (int)wp) {
                    rec[2 + lane] = fi[lane] & ~km;
                    rec[2 + O_XP + lane] = fi[O_XP + lane] | km;
                    rec[2 + O_EXT + lane] = don;
                  }
                  for (uint32_t k = 3 * wp + lane; k < F; k += kWave) rec[2 + k] = fi[k];
                  uint32_t* rq = (uint32_t*)(rec + 2 + F);
                  for (uint32_t j = lane; j + 1 < i; j += kWave) rq[j] = (uint32_t)stk[(uint64_t)(j + 1) * F + O_Q];
                  if (lane < (int)wp) stk[(uint64_t)i * F + O_EXT + lane] = km;
                  __threadfence();
                  if (lane == 0) {
                    fetch_add(&a.ctl[CTL_PENDING], 1);
                    uint64_t slot = fetch_add(&a.ctl[CTL_TAIL], 1);
                    st_release(&a.queue[slot], (uint64_t)((1ULL << 63) | off));
                    fetch_add(&a.ctl[CTL_DONATED], 1);
                  }
                  __threadfence_block();
                }
              }
            }
          }
          continue;
        }
      }
      // pop
      if (d == t.base) break;
      fr -= F;
      --d;
      if (lane < (int)wp) {
        rP = fr[lane];
        rXp = fr[O_XP + lane];
        rExt = fr[O_EXT + lane];
        if (EXCL) rF = fr[O_FB + lane];
      }
      zsum = readlane64(fr[O_Z], 0);
    }

    if (overflow) {
      if (lane == 0) atomicOr((unsigned long long*)&a.ctl[CTL_FLAGS], 1ULL);
    }
    if (lane == 0) {
      if (a.nodes_v) atomicAdd((unsigned long long*)&a.nodes_v[s], (unsigned long long)tn);
      if (a.count_v && tc) atomicAdd((unsigned long long*)&a.count_v[s], (unsigned long long)tc);
      if (a.hash_v && th) atomicAdd((unsigned long long*)&a.hash_v[s], (unsigned long long)th);
      __threadfence();
      fetch_add(&a.ctl[CTL_PENDING], ~0ULL);  // this task is done
    }
    tot_n += tn;
    tot_c += tc;
    tot_h += th;
  }
  if (lane == 0) {
    if (tot_c) atomicAdd((unsigned long long*)&a.ctl[CTL_COUNT], (unsigned long long)tot_c);
    if (tot_h) atomicAdd((unsigned long long*)&a.ctl[CTL_HASH], (unsigned long long)tot_h);
    if (tot_n) atomicAdd((unsigned long long*)&a.ctl[CTL_NODES], (unsigned long long)tot_n);
  }
}

__global__ void k_finish_offsets(uint64_t* off, uint64_t nc, uint64_t nv) { off[nc] = nv; }

}  // namespace

hipError_t launch_enum(const EnumArgs& a, uint32_t grid, bool exclusion, hipStream_t s) {
  const size_t lds = (size_t)kLdsWords * sizeof(uint64_t);
  if (exclusion)
    hipLaunchKernelGGL(k_enum<true>, dim3(grid), dim3(64), lds, s, a);
  else
    hipLaunchKernelGGL(k_enum<false>, dim3(grid), dim3(64), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_finish_offsets(uint64_t* off, uint64_t n_cliques, uint64_t n_verts, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_offsets, dim3(1), dim3(1), 0, s, off, n_cliques, n_verts);
  return hipGetLastError();
}

}  // namespace mce
