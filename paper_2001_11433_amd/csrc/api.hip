// Host side of the C ABI: argument checks, device workspace, the static MCE
// pipeline (rank -> subproblem build -> queue -> persistent enumeration) and
// error reporting.  No computation of the method happens on the host; it
// only sizes buffers and launches kernels.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace mce {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

Carver*& active_carver() {
  static thread_local Carver* c = nullptr;
  return c;
}

int carve(void** p, uint64_t b) {
  Carver* c = active_carver();
  *p = c ? c->take(b) : nullptr;
  if (!*p) {
    set_error("the call needs more than the %llu bytes of scratch of the allocation-free entry point "
              "(%llu in use, %llu more asked)", (unsigned long long)(c ? c->cap : 0),
              (unsigned long long)(c ? c->used : 0), (unsigned long long)b);
    return MCE_ENOTSUP;
  }
  return MCE_OK;
}

int ensure_temp(void*& tmp, size_t& tmp_bytes, size_t need) {
  if (need <= tmp_bytes && tmp) return MCE_OK;
  if (active_carver()) {
    MCE_TRY(carve(&tmp, std::max<size_t>(need, 256)));
    tmp_bytes = std::max<size_t>(need, 256);
    return MCE_OK;
  }
  if (tmp) MCE_TRY_HIP(hipFree(tmp));
  tmp = nullptr;
  tmp_bytes = 0;
  MCE_TRY_HIP(hipMalloc(&tmp, need));
  tmp_bytes = need;
  return MCE_OK;
}

namespace {
__global__ void k_zero32(uint32_t* p, uint64_t words) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}
}  // namespace

hipError_t dev_zero(void* p, uint64_t bytes, hipStream_t s) {
  const uint64_t words = bytes / 4;
  if (words == 0) return hipSuccess;
  const uint32_t blocks = (uint32_t)std::min<uint64_t>((words + 255) / 256, 8192);
  hipLaunchKernelGGL(k_zero32, dim3(blocks), dim3(256), 0, s, (uint32_t*)p, words);
  return hipGetLastError();
}

namespace {

// Device workspace of the static pipeline; grown on demand, reused across
// calls on the same device, guarded by one mutex per device.
struct Workspace {
  DevBuf rp, col, metric, tri, core, coredeg, corelist, corectl, P, X, xmark, lidx, words, gwords, off, goff, stats, arena,
      gids, keys, vals, keys2, vals2, iota, clq_off, clq_vert, bad, split, split_total, feat, cost;
  EnumWork ew;
  // second stream of the learned schedule (features and inference while the
  // subproblems are built), created on first use; default priority
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int side_init() {
    if (!side) MCE_TRY_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
    if (!ev_fork) MCE_TRY_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
    if (!ev_join) MCE_TRY_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
    return MCE_OK;
  }
  void* scan_tmp = nullptr;
  size_t scan_bytes = 0;
  void* sort_tmp = nullptr;
  size_t sort_bytes = 0;
};

std::mutex g_mu[64];
Workspace g_ws[64];

int current_device(int* dev) {
  MCE_TRY_HIP(hipGetDevice(dev));
  if (*dev < 0 || *dev >= 64) {
    set_error("device index %d out of range", *dev);
    return MCE_ENOTSUP;
  }
  return MCE_OK;
}

int cu_count() {
  int dev = 0, cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) return 256;
  return cu;
}

__global__ void k_iota(uint64_t n, uint32_t* a) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = (uint32_t)i;
}

// Isolated vertices are the cliques of size 1, found by the subproblem sizing
// (stats[3]); the search tallies every other size.
__global__ void k_hist_singletons(uint64_t* hist, uint64_t len, const uint64_t* stats) {
  hist[len > 1 ? 1 : 0] += stats[3];
}

// Singletons {v} of isolated vertices, for materialised output.
__global__ void k_emit_isolated(uint64_t n, const uint64_t* __restrict__ rp, uint64_t* ctl, uint64_t* off,
                                uint32_t* vert, uint64_t cap_c, uint64_t cap_v) {
  uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (v >= n || rp[v + 1] != rp[v]) return;
  uint64_t old = atomicAdd((unsigned long long*)&ctl[CTL_CLQ], (unsigned long long)((1ULL << 32) | 1ULL));
  uint64_t id = old >> 32, pos = old & 0xFFFFFFFFULL;
  if (id < cap_c && pos + 1 <= cap_v) {
    off[id] = pos;
    vert[pos] = (uint32_t)v;
  }
}

inline uint32_t blocks_for(uint64_t n, uint32_t bs) { return (uint32_t)((n + bs - 1) / bs); }

// Device-time events; `on` = false (the allocation-free entry point) creates
// none and reports 0 ms.
struct Timer {
  hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
  bool on = false;
  ~Timer() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
  int init(bool enable = true) {
    on = enable;
    if (on)
      for (auto& x : e) MCE_TRY_HIP(hipEventCreate(&x));
    return MCE_OK;
  }
  hipError_t record(int i, hipStream_t s) { return on ? hipEventRecord(e[i], s) : hipSuccess; }
  double ms(int a, int b) {
    float t = 0;
    if (!on || hipEventElapsedTime(&t, e[a], e[b]) != hipSuccess) return 0;
    return t;
  }
};

mce_opts default_opts() {
  mce_opts o;
  std::memset(&o, 0, sizeof(o));
  o.sched = MCE_SCHED_DEGREE;
  return o;
}

// Host view of the input: either borrowed device pointers or an upload.
int stage_csr(const mce_csr* g, Workspace& ws, hipStream_t s, const uint64_t** rp, const uint32_t** col,
              uint64_t* nnz) {
  const uint64_t n = g->n;
  if (n > 0 && !g->row_ptr) {
    set_error("row_ptr is NULL");
    return MCE_EINVAL;
  }
  if (g->on_device) {
    uint64_t last = 0;
    if (n > 0) {
      MCE_TRY_HIP(hipMemcpyAsync(&last, g->row_ptr + n, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
      MCE_TRY_HIP(hipStreamSynchronize(s));
    }
    *nnz = last;
    *rp = g->row_ptr;
    *col = g->col;
  } else {
    *nnz = n ? g->row_ptr[n] : 0;
    MCE_TRY(ws.rp.ensure((n + 1) * sizeof(uint64_t)));
    MCE_TRY(ws.col.ensure(std::max<uint64_t>(*nnz, 1) * sizeof(uint32_t)));
    if (n > 0) MCE_TRY_HIP(hipMemcpyAsync(ws.rp.p, g->row_ptr, (n + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    if (*nnz) MCE_TRY_HIP(hipMemcpyAsync(ws.col.p, g->col, *nnz * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    *rp = ws.rp.as<uint64_t>();
    *col = ws.col.as<uint32_t>();
  }
  if (*nnz > 0 && !g->col) {
    set_error("col is NULL");
    return MCE_EINVAL;
  }
  if (*nnz >= (1ULL << 40)) {
    set_error("graph too large");
    return MCE_ENOTSUP;
  }
  return MCE_OK;
}

int validate_csr(uint64_t n, const uint64_t* rp, const uint32_t* col, Workspace& ws, hipStream_t s) {
  MCE_TRY(ws.bad.ensure(sizeof(uint32_t)));
  MCE_TRY_HIP(dev_zero(ws.bad.p, sizeof(uint32_t), s));
  uint64_t first = 1;
  if (n) {
    MCE_TRY_HIP(hipMemcpyAsync(&first, rp, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  }
  MCE_TRY_HIP(launch_validate(n, rp, col, ws.bad.as<uint32_t>(), s));
  uint32_t bad = 0;
  MCE_TRY_HIP(hipMemcpyAsync(&bad, ws.bad.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipStreamSynchronize(s));
  if (n && first != 0) {
    set_error("row_ptr[0] != 0");
    return MCE_EINVAL;
  }
  if (bad) {
    set_error("malformed CSR (code %u: 1 row_ptr decreasing, 2 bad/unsorted/self-loop column, 4 asymmetric)", bad);
    return MCE_EINVAL;
  }
  return MCE_OK;
}

int compute_metric(mce_rank rank, uint64_t n, const uint64_t* rp, const uint32_t* col, uint64_t* metric,
                   Workspace& ws, hipStream_t s) {
  switch (rank) {
    case MCE_RANK_DEGREE:
      MCE_TRY_HIP(launch_degree(n, rp, metric, s));
      return MCE_OK;
    case MCE_RANK_DEGENERACY:
      MCE_TRY(ws.coredeg.ensure(std::max<uint64_t>(n, 1) * sizeof(uint32_t)));
      MCE_TRY(ws.corelist.ensure(std::max<uint64_t>(n, 1) * sizeof(uint32_t)));
      MCE_TRY(ws.corectl.ensure(8 * sizeof(uint64_t)));
      return run_core_numbers(n, rp, col, metric, ws.coredeg.as<uint32_t>(), ws.corelist.as<uint32_t>(),
                              ws.corectl.as<uint64_t>(), s);
    case MCE_RANK_TRIANGLE:
      MCE_TRY_HIP(launch_triangles(n, rp, col, metric, s));
      return MCE_OK;
    case MCE_RANK_PEEL:
      MCE_TRY(ws.coredeg.ensure(std::max<uint64_t>(n, 1) * sizeof(uint32_t)));
      MCE_TRY(ws.corelist.ensure(std::max<uint64_t>(n, 1) * sizeof(uint32_t)));
      MCE_TRY(ws.corectl.ensure(8 * sizeof(uint64_t)));
      return run_peel_rounds(n, rp, col, metric, ws.coredeg.as<uint32_t>(), ws.corelist.as<uint32_t>(),
                             ws.corectl.as<uint64_t>(), s);
    case MCE_RANK_TTT_ROOT:
      MCE_TRY(ws.corectl.ensure(8 * sizeof(uint64_t)));
      MCE_TRY_HIP(launch_root_metric(n, rp, col, metric, ws.corectl.as<uint64_t>(), s));
      return MCE_OK;
  }
  set_error("unknown rank %d", (int)rank);
  return MCE_EINVAL;
}

}  // namespace

// Handoff arena for the compact kernel: grown to the demand of the previous
// run, at most kHandRecsMax records in kHandUnitsMax 64-byte units (64 GiB).
constexpr uint64_t kHandRecsMax = 1ULL << 26;
constexpr uint64_t kHandUnitsMax = 1ULL << 30;
constexpr uint64_t kHandDefaultMb = 16384;

// The arena's budget in 64-byte units (mce_opts.hand_mb).
uint64_t hand_budget_units(const mce_opts& o) {
  const uint64_t mb = o.hand_mb ? o.hand_mb : kHandDefaultMb;
  return std::min<uint64_t>(mb << 14, kHandUnitsMax);
}
constexpr uint32_t kCompactWavesPerCu = 20;

uint32_t enum_grid(const mce_opts& opts) {
  const uint32_t wpc = opts.waves_per_cu ? opts.waves_per_cu : 8;
  return (uint32_t)cu_count() * wpc;
}

int run_enum(EnumJob& j, EnumWork& w, hipStream_t s, uint64_t* ctl, uint32_t* retries) {
  const mce_opts& opts = *j.opts;
  const uint32_t grid = enum_grid(opts);
  uint32_t frame_cap = opts.frame_cap ? opts.frame_cap : 128;
  frame_cap = std::min<uint32_t>(frame_cap, (uint32_t)j.max_p + 2);
  frame_cap = std::max<uint32_t>(frame_cap, 2);
  const uint64_t max_tickets = j.max_tickets ? j.max_tickets : std::max<uint64_t>(1u << 24, 4 * j.nq);
  const uint64_t qcap = j.nq + max_tickets;
  const uint64_t pool_blocks = j.pool_blocks ? j.pool_blocks : 1ULL << 16;  // records of 8 KiB, recycled
  MCE_TRY(w.queue.ensure(qcap * sizeof(uint64_t)));
  MCE_TRY(w.pool.ensure(pool_blocks * kBlockWords * sizeof(uint64_t)));
  MCE_TRY(w.pool_next.ensure(pool_blocks * sizeof(uint32_t)));
  MCE_TRY(w.ctl.ensure(CTL_WORDS * sizeof(uint64_t)));
  if (retries) *retries = 0;
  for (uint32_t attempt = 0;; ++attempt) {
    const uint64_t stack_words = (uint64_t)frame_cap * std::max<uint64_t>(j.max_frame + 1, 8);
    MCE_TRY(w.stacks.ensure((uint64_t)grid * stack_words * sizeof(uint64_t)));
    MCE_TRY_HIP(dev_zero(w.queue.p, qcap * sizeof(uint64_t), s));
    MCE_TRY_HIP(launch_queue_fill(j.nq, j.order, j.split, w.queue.as<uint64_t>(), s));
    std::memset(ctl, 0, CTL_WORDS * sizeof(uint64_t));
    ctl[CTL_TAIL] = j.nq;
    ctl[CTL_PENDING] = j.nq;
    ctl[CTL_FREE] = 0;  // tag 0, first block 0
    MCE_TRY_HIP(launch_pool_init(w.pool_next.as<uint32_t>(), pool_blocks, s));
    MCE_TRY_HIP(hipMemcpyAsync(w.ctl.p, ctl, CTL_WORDS * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    if (j.before_launch) MCE_TRY(j.before_launch(attempt, w.ctl.as<uint64_t>()));
    EnumArgs a;
    std::memset(&a, 0, sizeof(a));
    a.sub = j.sub;
    a.arena = j.arena;
    a.gids = j.gids;
    a.queue = w.queue.as<uint64_t>();
    a.qcap = qcap;
    a.ctl = w.ctl.as<uint64_t>();
    a.pool = w.pool.as<uint64_t>();
    a.pool_next = w.pool_next.as<uint32_t>();
    a.pool_blocks = pool_blocks;
    a.max_tickets = max_tickets;
    a.stacks = w.stacks.as<uint64_t>();
    a.stack_words = stack_words;
    a.frame_cap = frame_cap;
    a.frame_words = (uint32_t)j.max_frame + 1;
    a.donate_interval = opts.donate_interval ? opts.donate_interval : 256;
    a.nodes_v = j.nodes_v;
    a.count_v = j.count_v;
    a.hash_v = j.hash_v;
    a.cl_off = j.cl_off;
    a.cl_vert = j.cl_vert;
    a.hist = j.hist;
    a.hist_len = j.hist_len;
    a.lds_rows = std::min<uint32_t>(opts.lds_row_words, kLdsRowsMax);
    a.emit_extra = (j.cl_vert || j.hist) ? 1u : 0u;
    a.cap_cliques = j.cap_cliques;
    a.cap_verts = j.cap_verts;
    if (j.max_p + (j.excl ? 2u : 1u) + 2 > kKLds) {
      // some clique may outgrow the LDS K list: one global list per wave
      MCE_TRY(w.kbig.ensure((uint64_t)grid * kKBig * sizeof(uint32_t)));
      a.kbig = w.kbig.as<uint32_t>();
    }
    const bool handoff = !opts.inline_compact;
    uint64_t hand_cap = 0;
    if (handoff) {
      // sized to what the previous run asked for; requests beyond the
      // capacity are searched in place
      const uint64_t first = std::max<uint64_t>(j.hand_initial_units, 1u << 20);
      const uint64_t units = std::min<uint64_t>(std::max<uint64_t>(w.hand_want_units, first), hand_budget_units(opts));
      // a record takes at least one unit
      hand_cap = std::min<uint64_t>(std::max<uint64_t>(w.hand_want_recs, units), kHandRecsMax);
      MCE_TRY(w.hand.ensure(units * 64));
      MCE_TRY(w.hand_idx.ensure(hand_cap * sizeof(uint32_t)));
      a.hand = w.hand.as<uint64_t>();
      a.hand_units = units;
      a.hand_idx = w.hand_idx.as<uint32_t>();
      a.hand_cap = hand_cap;
    }
    if (j.nq > 0) MCE_TRY_HIP(launch_enum(a, grid, j.excl, s));
    MCE_TRY_HIP(hipMemcpyAsync(ctl, w.ctl.p, CTL_WORDS * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    MCE_TRY_HIP(hipStreamSynchronize(s));
    if (!(ctl[CTL_FLAGS] & 1ULL)) {
      if (!handoff) return MCE_OK;
      // second launch: the compact kernel over the handed-off nodes (the
      // records written form a prefix of the request order)
      const uint64_t req_recs = ctl[CTL_HAND] >> 32, req_units = ctl[CTL_HAND] & 0xFFFFFFFFULL;
      w.hand_want_recs = std::max(w.hand_want_recs, req_recs);
      w.hand_want_units = std::max(w.hand_want_units, req_recs <= kHandRecsMax ? req_units : kHandUnitsMax);
      const uint64_t nh = ctl[CTL_HANDOK];
      if (nh == 0) return MCE_OK;
      const uint64_t qcap2 = nh + max_tickets;
      if (qcap2 > qcap) MCE_TRY(w.queue.ensure(qcap2 * sizeof(uint64_t)));
      a.queue = w.queue.as<uint64_t>();
      a.qcap = qcap2;
      MCE_TRY_HIP(dev_zero(w.queue.p, qcap2 * sizeof(uint64_t), s));
      const uint32_t* order = nullptr;
      if (opts.compact_order == 1 || opts.compact_order == 2) {
        // 1: largest candidate set first (then largest fini); 2: grouped by
        // subproblem (its records gather the same rows), larger first within
        const uint32_t by_sub = opts.compact_order == 2 ? 1u : 0u;
        MCE_TRY(w.hkeys.ensure(nh * 8));
        MCE_TRY(w.hkeys2.ensure(nh * 8));
        MCE_TRY(w.hvals.ensure(nh * 4));
        MCE_TRY(w.hvals2.ensure(nh * 4));
        MCE_TRY_HIP(launch_hand_keys(nh, a.hand, a.hand_idx, by_sub, w.hkeys.as<uint64_t>(), w.hvals.as<uint32_t>(),
                                     s));
        uint64_t* sk;
        uint32_t* sv;
        MCE_TRY(device_sort_desc(w.hkeys.as<uint64_t>(), w.hvals.as<uint32_t>(), w.hkeys2.as<uint64_t>(),
                                 w.hvals2.as<uint32_t>(), nh, w.sort_tmp, w.sort_bytes, s, &sk, &sv, by_sub ? 48 : 16));
        order = sv;
      }
      MCE_TRY_HIP(launch_queue_fill_hand(nh, order, a.queue, s));
      MCE_TRY_HIP(launch_pool_init(w.pool_next.as<uint32_t>(), pool_blocks, s));
      ctl[CTL_HEAD] = 0;
      ctl[CTL_TAIL] = nh;
      ctl[CTL_PENDING] = nh;
      ctl[CTL_FREE] = 0;
      ctl[CTL_TICKETS] = 0;
      MCE_TRY_HIP(hipMemcpyAsync(w.ctl.p, ctl, CTL_WORDS * sizeof(uint64_t), hipMemcpyHostToDevice, s));
      const uint32_t cwpc = opts.compact_waves_per_cu ? opts.compact_waves_per_cu : kCompactWavesPerCu;
      Timer tm;
      MCE_TRY(tm.init(j.timing));
      MCE_TRY_HIP(tm.record(0, s));
      MCE_TRY_HIP(launch_compact(a, (uint32_t)cu_count() * cwpc, j.excl, s));
      MCE_TRY_HIP(tm.record(1, s));
      MCE_TRY_HIP(hipMemcpyAsync(ctl, w.ctl.p, CTL_WORDS * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
      MCE_TRY_HIP(hipStreamSynchronize(s));
      j.hand_ms = tm.ms(0, 1);
      j.handed = nh;
      return MCE_OK;
    }
    if (frame_cap >= j.max_p + 2 || attempt >= 12) {
      set_error("DFS stack overflow at %u frames", frame_cap);
      return MCE_ENOMEM;
    }
    frame_cap = std::min<uint32_t>(frame_cap * 2, (uint32_t)j.max_p + 2);
    if (retries) *retries = attempt + 1;
  }
}

namespace {

// `noalloc`: every buffer comes from the active Carver (the caller installed
// one), no events are created, and the launch uses smaller donation tables.
int static_impl(const mce_csr* g, mce_rank rank, const mce_opts& opts, mce_result* out, mce_clique_buf* cl,
                const mce_per_vertex* pv, Workspace& ws, bool noalloc = false) {
  hipStream_t s = (hipStream_t)opts.hip_stream;
  const uint64_t n = g->n;
  if (n >= 0xFFFFFFFFULL) {
    set_error("n must be below 2^32 - 1");
    return MCE_ENOTSUP;
  }
  if (rank != MCE_RANK_DEGREE && rank != MCE_RANK_DEGENERACY && rank != MCE_RANK_TRIANGLE &&
      rank != MCE_RANK_TTT_ROOT && rank != MCE_RANK_PEEL) {
    set_error("unknown rank %d", (int)rank);
    return MCE_EINVAL;
  }
  if (opts.sched == MCE_SCHED_COST && !opts.sched_cost) {
    set_error("MCE_SCHED_COST needs sched_cost");
    return MCE_EINVAL;
  }
  if ((unsigned)opts.sched > MCE_SCHED_MLP) {
    set_error("unknown schedule %d", (int)opts.sched);
    return MCE_EINVAL;
  }
  if (opts.sched == MCE_SCHED_MLP && (!opts.sched_model || !opts.sched_model_bf16)) {
    set_error("MCE_SCHED_MLP needs sched_model and sched_model_bf16");
    return MCE_EINVAL;
  }
  if (cl && ((cl->cap_cliques && !cl->off) || (cl->cap_verts && !cl->vert))) {
    set_error("clique buffer has capacity but no array");
    return MCE_EINVAL;
  }
  std::memset(out, 0, sizeof(*out));
  const uint64_t* rp;
  const uint32_t* col;
  uint64_t nnz;
  MCE_TRY(stage_csr(g, ws, s, &rp, &col, &nnz));
  if (n == 0) {
    if (pv && pv->size_hist && pv->hist_len)
      MCE_TRY_HIP(dev_zero(pv->size_hist, pv->hist_len * sizeof(uint64_t), s));
    if (cl) {
      cl->n_cliques = 0;
      cl->n_verts = 0;
      if (cl->cap_cliques >= 0 && cl->off) {
        uint64_t z = 0;
        if (cl->on_device) MCE_TRY_HIP(hipMemcpyAsync(cl->off, &z, sizeof(z), hipMemcpyHostToDevice, s));
        else cl->off[0] = 0;
      }
    }
    MCE_TRY_HIP(hipStreamSynchronize(s));
    return MCE_OK;
  }
  if (opts.validate) MCE_TRY(validate_csr(n, rp, col, ws, s));

  Timer tm;
  MCE_TRY(tm.init(!noalloc));
  MCE_TRY_HIP(tm.record(0, s));

  // --- rank (Section 4.2)
  MCE_TRY(ws.metric.ensure(n * sizeof(uint64_t)));
  uint64_t* metric = ws.metric.as<uint64_t>();
  MCE_TRY(compute_metric(rank, n, rp, col, metric, ws, s));
  const uint64_t* tri = nullptr;
  if (opts.sched == MCE_SCHED_TRIANGLE) {
    if (rank == MCE_RANK_TRIANGLE) {
      tri = metric;
    } else {
      MCE_TRY(ws.tri.ensure(n * sizeof(uint64_t)));
      MCE_TRY_HIP(launch_triangles(n, rp, col, ws.tri.as<uint64_t>(), s));
      tri = ws.tri.as<uint64_t>();
    }
  }
  MCE_TRY_HIP(tm.record(1, s));

  // --- learned schedule: the cost model's inputs and prediction on a second
  // stream, forked here and joined before the queue is ordered, so they
  // overlap the subproblem build (the allocation-free call creates no streams
  // or events and runs them in order on s)
  const bool mlp = opts.sched == MCE_SCHED_MLP;
  float* mlp_cost = nullptr;
  hipStream_t side = s;
  const uint64_t* mlp_tri = nullptr;
  if (mlp) {
    MCE_TRY(ws.feat.ensure(n * 4 * sizeof(float)));
    if (pv && pv->sched_cost) {
      mlp_cost = pv->sched_cost;
    } else {
      MCE_TRY(ws.cost.ensure(n * sizeof(float)));
      mlp_cost = ws.cost.as<float>();
    }
    if (rank != MCE_RANK_TRIANGLE && !tri) {
      MCE_TRY(ws.tri.ensure(n * sizeof(uint64_t)));
    }
    if (rank != MCE_RANK_DEGENERACY) {
      // every buffer of the side work is sized before the fork
      MCE_TRY(ws.core.ensure(n * sizeof(uint64_t)));
      MCE_TRY(ws.coredeg.ensure(n * sizeof(uint32_t)));
      MCE_TRY(ws.corelist.ensure(n * sizeof(uint32_t)));
      MCE_TRY(ws.corectl.ensure(8 * sizeof(uint64_t)));
    }
    if (!noalloc) {
      MCE_TRY(ws.side_init());
      side = ws.side;
      MCE_TRY_HIP(hipEventRecord(ws.ev_fork, s));
      MCE_TRY_HIP(hipStreamWaitEvent(side, ws.ev_fork, 0));
    }
    if (rank == MCE_RANK_TRIANGLE) {
      mlp_tri = metric;
    } else if (tri) {
      mlp_tri = tri;
    } else {
      MCE_TRY_HIP(launch_triangles(n, rp, col, ws.tri.as<uint64_t>(), side));
      mlp_tri = ws.tri.as<uint64_t>();
    }
  }

  // --- subproblem sizes and build (Algorithm 4, body)
  MCE_TRY(ws.P.ensure(n * sizeof(uint32_t)));
  MCE_TRY(ws.X.ensure(n * sizeof(uint32_t)));
  MCE_TRY(ws.words.ensure(n * sizeof(uint64_t)));
  MCE_TRY(ws.gwords.ensure(n * sizeof(uint64_t)));
  MCE_TRY(ws.off.ensure(n * sizeof(uint64_t)));
  MCE_TRY(ws.goff.ensure(n * sizeof(uint64_t)));
  MCE_TRY(ws.stats.ensure(8 * sizeof(uint64_t)));
  const uint64_t xwords = std::max<uint64_t>((nnz + 31) / 32, 1);
  MCE_TRY(ws.xmark.ensure(xwords * sizeof(uint32_t)));
  MCE_TRY(ws.lidx.ensure(std::max<uint64_t>(nnz, 1) * sizeof(uint32_t)));
  BuildBufs b;
  b.p = ws.P.as<uint32_t>();
  b.x = ws.X.as<uint32_t>();
  b.xmark = ws.xmark.as<uint32_t>();
  b.lidx = ws.lidx.as<uint32_t>();
  b.words = ws.words.as<uint64_t>();
  b.gwords = ws.gwords.as<uint64_t>();
  b.stats = ws.stats.as<uint64_t>();
  uint64_t* nodes_v = pv ? pv->nodes : nullptr;
  uint64_t* count_v = pv ? pv->count : nullptr;
  uint64_t* hash_v = pv ? pv->hash : nullptr;
  uint64_t* hist = pv ? pv->size_hist : nullptr;
  const uint64_t hist_len = pv ? pv->hist_len : 0;
  if (hist && hist_len < 2) {
    set_error("size_hist needs hist_len >= 2");
    return MCE_EINVAL;
  }

  MCE_TRY_HIP(dev_zero(b.stats, 8 * sizeof(uint64_t), s));
  MCE_TRY_HIP(launch_sizes(n, rp, col, metric, b, nodes_v, count_v, hash_v, s));
  MCE_TRY_HIP(dev_zero(b.xmark, xwords * sizeof(uint32_t), s));
  MCE_TRY_HIP(launch_mark(n, rp, col, metric, b, s));
  MCE_TRY_HIP(launch_words(n, rp, b, s));
  MCE_TRY(device_exclusive_scan(b.words, ws.off.as<uint64_t>(), n, ws.scan_tmp, ws.scan_bytes, s));
  MCE_TRY(device_exclusive_scan(b.gwords, ws.goff.as<uint64_t>(), n, ws.scan_tmp, ws.scan_bytes, s));
  uint64_t stats[8], tail[4];
  MCE_TRY_HIP(hipMemcpyAsync(stats, b.stats, sizeof(stats), hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipMemcpyAsync(&tail[0], ws.off.as<uint64_t>() + n - 1, 8, hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipMemcpyAsync(&tail[1], b.words + n - 1, 8, hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipMemcpyAsync(&tail[2], ws.goff.as<uint64_t>() + n - 1, 8, hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipMemcpyAsync(&tail[3], b.gwords + n - 1, 8, hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipStreamSynchronize(s));
  const uint64_t max_p = stats[0], max_frame = stats[1], nq = stats[2];
  out->subproblems = nq;
  out->max_cand = max_p;
  if (max_p > kMaxCand) {
    set_error("a subproblem has %llu candidates; at most %u are supported", (unsigned long long)max_p, kMaxCand);
    return MCE_ENOTSUP;
  }
  const uint64_t arena_words = tail[0] + tail[1], gid_words = tail[2] + tail[3];
  MCE_TRY(ws.arena.ensure(std::max<uint64_t>(arena_words, 1) * sizeof(uint64_t)));
  MCE_TRY(ws.gids.ensure(std::max<uint64_t>(gid_words, 1) * sizeof(uint32_t)));
  MCE_TRY_HIP(dev_zero(ws.arena.p, std::max<uint64_t>(arena_words, 1) * sizeof(uint64_t), s));
  MCE_TRY_HIP(launch_build(n, rp, col, metric, b, ws.off.as<uint64_t>(), ws.goff.as<uint64_t>(),
                           ws.arena.as<uint64_t>(), ws.gids.as<uint32_t>(), s));

  if (mlp) {
    // core numbers (the rank's own metric under degeneracy ownership; the
    // peeling waits on the host between rounds, which is why it is enqueued
    // after the build), features, then the BF16 forward
    const uint64_t* core = metric;
    if (rank != MCE_RANK_DEGENERACY) {
      MCE_TRY(run_core_numbers(n, rp, col, ws.core.as<uint64_t>(), ws.coredeg.as<uint32_t>(),
                               ws.corelist.as<uint32_t>(), ws.corectl.as<uint64_t>(), side));
      core = ws.core.as<uint64_t>();
    }
    MCE_TRY_HIP(launch_features(n, rp, col, core, mlp_tri, ws.feat.as<float>(), side));
    MCE_TRY_HIP(launch_mlp_forward_bf16(opts.sched_model, opts.sched_model_bf16, ws.feat.as<float>(), n, mlp_cost,
                                        side));
    if (side != s) {
      MCE_TRY_HIP(hipEventRecord(ws.ev_join, side));
      MCE_TRY_HIP(hipStreamWaitEvent(s, ws.ev_join, 0));
    }
  }
  const mce_sched qsched = mlp ? MCE_SCHED_COST : opts.sched;
  const float* qcost = mlp ? mlp_cost : opts.sched_cost;

  // --- queue order (never changes results)
  MCE_TRY(ws.keys.ensure(n * sizeof(uint64_t)));
  MCE_TRY(ws.keys2.ensure(n * sizeof(uint64_t)));
  MCE_TRY(ws.vals.ensure(n * sizeof(uint32_t)));
  MCE_TRY(ws.vals2.ensure(n * sizeof(uint32_t)));
  MCE_TRY_HIP(launch_queue_keys(n, rp, b.p, qsched, tri, qcost, ws.keys.as<uint64_t>(),
                                ws.vals.as<uint32_t>(), nullptr, s));
  uint64_t* skeys;
  uint32_t* svals;
  MCE_TRY(device_sort_desc(ws.keys.as<uint64_t>(), ws.vals.as<uint32_t>(), ws.keys2.as<uint64_t>(),
                           ws.vals2.as<uint32_t>(), n, ws.sort_tmp, ws.sort_bytes, s, &skeys, &svals));
  MCE_TRY(ws.iota.ensure(n * sizeof(uint32_t)));
  hipLaunchKernelGGL(k_iota, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, ws.iota.as<uint32_t>());
  MCE_TRY_HIP(hipGetLastError());
  const uint32_t* split = nullptr;
  if (qsched == MCE_SCHED_COST && opts.split > 1) {
    MCE_TRY(ws.split.ensure(n * sizeof(uint32_t)));
    MCE_TRY(ws.split_total.ensure(sizeof(double)));
    MCE_TRY_HIP(launch_split_plan(n, b.p, qcost, enum_grid(opts), std::min<uint32_t>(opts.split, 0xFFFFu),
                                  ws.split_total.as<double>(), ws.split.as<uint32_t>(), s));
    split = ws.split.as<uint32_t>();
  }
  MCE_TRY_HIP(tm.record(2, s));

  // --- clique output buffers
  uint64_t* cl_off = nullptr;
  uint32_t* cl_vert = nullptr;
  if (cl) {
    if (cl->on_device) {
      cl_off = cl->off;
      cl_vert = cl->vert;
    } else {
      MCE_TRY(ws.clq_off.ensure((cl->cap_cliques + 1) * sizeof(uint64_t)));
      MCE_TRY(ws.clq_vert.ensure(std::max<uint64_t>(cl->cap_verts, 1) * sizeof(uint32_t)));
      cl_off = ws.clq_off.as<uint64_t>();
      cl_vert = ws.clq_vert.as<uint32_t>();
    }
  }

  // --- persistent enumeration, restarted with deeper stacks on overflow
  EnumJob job;
  job.sub.off = ws.off.as<uint64_t>();
  job.sub.goff = ws.goff.as<uint64_t>();
  job.sub.p = b.p;
  job.sub.x = b.x;
  job.sub.r0 = ws.iota.as<uint32_t>();
  job.sub.r1 = ws.iota.as<uint32_t>();
  job.arena = ws.arena.as<uint64_t>();
  job.gids = ws.gids.as<uint32_t>();
  job.nq = nq;
  job.order = svals;
  job.split = split;
  job.max_p = max_p;
  job.max_frame = max_frame;
  job.excl = false;
  job.nodes_v = nodes_v;
  job.count_v = count_v;
  job.hash_v = hash_v;
  job.hist = hist;
  job.hist_len = hist_len;
  job.cl_off = cl_off;
  job.cl_vert = cl_vert;
  job.cap_cliques = cl ? cl->cap_cliques : 0;
  job.cap_verts = cl ? cl->cap_verts : 0;
  job.opts = &opts;
  if (noalloc) {
    // modest tables that fit the scratch: 16 MiB of handoff records, 256
    // donation blocks (2 MiB), 2^18 queue tickets (2 MiB)
    job.hand_initial_units = (16ULL << 20) / 64;
    job.pool_blocks = 256;
    job.max_tickets = 1ULL << 18;
    job.timing = false;
  } else if (!opts.inline_compact && nq >= (1u << 17)) {
    // a large call cannot rely on the demand of earlier (maybe smaller) runs
    // to size the handoff arena: offer a quarter of the free device memory
    // (bounded by the arena's maximum; the buffer only grows)
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) job.hand_initial_units = free_b / 4 / 64;
  }
  job.before_launch = [&](uint32_t attempt, uint64_t* ctl_dev) -> int {
    if (hist) MCE_TRY_HIP(dev_zero(hist, hist_len * sizeof(uint64_t), s));
    if (attempt > 0) {
      // results of the aborted run are discarded: reset per-vertex outputs
      MCE_TRY_HIP(dev_zero(b.stats, 8 * sizeof(uint64_t), s));
      MCE_TRY_HIP(launch_sizes(n, rp, col, metric, b, nodes_v, count_v, hash_v, s));
    }
    if (cl) {
      hipLaunchKernelGGL(k_emit_isolated, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, ctl_dev, cl_off,
                         cl_vert, cl->cap_cliques, cl->cap_verts);
      MCE_TRY_HIP(hipGetLastError());
    }
    return MCE_OK;
  };
  uint64_t ctl[CTL_WORDS];
  MCE_TRY(run_enum(job, ws.ew, s, ctl, &out->retries));
  MCE_TRY_HIP(tm.record(3, s));
  if (hist) {
    hipLaunchKernelGGL(k_hist_singletons, dim3(1), dim3(1), 0, s, hist, hist_len, b.stats);
    MCE_TRY_HIP(hipGetLastError());
  }
  MCE_TRY_HIP(hipMemcpyAsync(stats, b.stats, sizeof(stats), hipMemcpyDeviceToHost, s));
  MCE_TRY_HIP(hipStreamSynchronize(s));
  out->count = stats[3] + ctl[CTL_COUNT];
  out->set_hash = stats[4] + ctl[CTL_HASH];
  // the whole-graph root itself is one more search node
  out->nodes_total = stats[5] + ctl[CTL_NODES] + (rank == MCE_RANK_TTT_ROOT ? 1 : 0);
  out->donated = ctl[CTL_DONATED];
  out->alg_ops = ctl[CTL_OPS];
  out->exec_ops = ctl[CTL_OPS_EXEC];
  out->lds_bytes = ctl[CTL_LDS_BYTES];
  out->arena_bytes = arena_words * sizeof(uint64_t) + gid_words * sizeof(uint32_t);
  for (int k = 0; k < 8; ++k) out->diag[k] = ctl[CTL_DIAG + k];
  out->compact_ms = job.hand_ms;
  out->handed = job.handed;
  out->rank_ms = tm.ms(0, 1);
  out->build_ms = tm.ms(1, 2);
  out->enum_ms = tm.ms(2, 3);
  int rc = MCE_OK;
  if (cl) {
    const uint64_t nc = ctl[CTL_CLQ] >> 32, nv = ctl[CTL_CLQ] & 0xFFFFFFFFULL;
    cl->n_cliques = nc;
    cl->n_verts = nv;
    if (ctl[CTL_FLAGS] & 2ULL) {
      set_error("materialised output exceeds 2^32 vertices");
      return MCE_ENOTSUP;
    }
    if (nc > cl->cap_cliques || nv > cl->cap_verts || !cl_off) {
      set_error("clique buffer too small: need %llu cliques, %llu vertices", (unsigned long long)nc,
                (unsigned long long)nv);
      rc = MCE_ENOSPC;
    } else {
      MCE_TRY_HIP(launch_finish_offsets(cl_off, nc, nv, s));
      if (!cl->on_device) {
        MCE_TRY_HIP(hipMemcpyAsync(cl->off, cl_off, (nc + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        if (nv) MCE_TRY_HIP(hipMemcpyAsync(cl->vert, cl_vert, nv * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      }
      MCE_TRY_HIP(hipStreamSynchronize(s));
    }
  }
  return rc;
}

// Scratch of the allocation-free entry point: one copy per GPU, held until the
// process ends.  Host code reaches it only through the per-device address
// from hipGetSymbolAddress (g_scratch), never through the array's name.
static __device__ __align__(256) uint8_t scratch[MCE_NOALLOC_SCRATCH_BYTES];
void* g_scratch[64];  // device address of `scratch` per device, set on first use (under g_mu)

int scratch_of(int dev, void** out) {
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
      return MCE_EDEVICE;
    }
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return MCE_OK;
}

}  // namespace
}  // namespace mce

using namespace mce;

extern "C" {

const char* mce_strerror(int code) {
  switch (code) {
    case MCE_OK: return "ok";
    case MCE_EINVAL: return "invalid argument";
    case MCE_ENOMEM: return "out of device memory";
    case MCE_ENOSPC: return "output buffer too small";
    case MCE_EDEVICE: return "HIP runtime error";
    case MCE_ENOTSUP: return "input outside the supported envelope";
    case MCE_ECANCELED: return "batch dropped after an earlier batch failed";
  }
  return "unknown error";
}

const char* mce_last_error(void) { return g_err; }

int mce_static(const mce_csr* g, mce_rank rank, const mce_opts* opts, mce_result* out, mce_clique_buf* cliques,
               const mce_per_vertex* per_vertex) {
  if (!g || !out) {
    set_error("NULL graph or result");
    return MCE_EINVAL;
  }
  mce_opts o = opts ? *opts : default_opts();
  int dev;
  MCE_TRY(current_device(&dev));
  std::lock_guard<std::mutex> lk(g_mu[dev]);
  return static_impl(g, rank, o, out, cliques, per_vertex, g_ws[dev]);
}

int mce_static_noalloc(const mce_csr* g, mce_rank rank, const mce_opts* opts, mce_result* out,
                       mce_clique_buf* cliques, const mce_per_vertex* per_vertex) {
  if (!g || !out) {
    set_error("NULL graph or result");
    return MCE_EINVAL;
  }
  mce_opts o = opts ? *opts : default_opts();
  int dev;
  MCE_TRY(current_device(&dev));
  std::lock_guard<std::mutex> lk(g_mu[dev]);
  void* base;
  MCE_TRY(scratch_of(dev, &base));
  Carver c{(uint8_t*)base, MCE_NOALLOC_SCRATCH_BYTES, 0};
  CarverScope scope(&c);
  Workspace ws;  // every buffer of this call is carved from the scratch
  return static_impl(g, rank, o, out, cliques, per_vertex, ws, true);
}

int mce_rank_metric(const mce_csr* g, mce_rank rank, uint64_t* metric, void* hip_stream) {
  if (!g || !metric) {
    set_error("NULL graph or output");
    return MCE_EINVAL;
  }
  int dev;
  MCE_TRY(current_device(&dev));
  std::lock_guard<std::mutex> lk(g_mu[dev]);
  Workspace& ws = g_ws[dev];
  hipStream_t s = (hipStream_t)hip_stream;
  const uint64_t* rp;
  const uint32_t* col;
  uint64_t nnz;
  MCE_TRY(stage_csr(g, ws, s, &rp, &col, &nnz));
  if (g->n == 0) return MCE_OK;
  MCE_TRY(compute_metric(rank, g->n, rp, col, metric, ws, s));
  MCE_TRY_HIP(hipStreamSynchronize(s));
  return MCE_OK;
}

int mce_features(const mce_csr* g, float* feat, void* hip_stream) {
  if (!g || !feat) {
    set_error("NULL graph or output");
    return MCE_EINVAL;
  }
  int dev;
  MCE_TRY(current_device(&dev));
  std::lock_guard<std::mutex> lk(g_mu[dev]);
  Workspace& ws = g_ws[dev];
  hipStream_t s = (hipStream_t)hip_stream;
  const uint64_t* rp;
  const uint32_t* col;
  uint64_t nnz;
  MCE_TRY(stage_csr(g, ws, s, &rp, &col, &nnz));
  const uint64_t n = g->n;
  if (n == 0) return MCE_OK;
  MCE_TRY(ws.core.ensure(n * sizeof(uint64_t)));
  MCE_TRY(ws.tri.ensure(n * sizeof(uint64_t)));
  MCE_TRY(compute_metric(MCE_RANK_DEGENERACY, n, rp, col, ws.core.as<uint64_t>(), ws, s));
  MCE_TRY_HIP(launch_triangles(n, rp, col, ws.tri.as<uint64_t>(), s));
  MCE_TRY_HIP(launch_features(n, rp, col, ws.core.as<uint64_t>(), ws.tri.as<uint64_t>(), feat, s));
  MCE_TRY_HIP(hipStreamSynchronize(s));
  return MCE_OK;
}

}  // extern "C"
