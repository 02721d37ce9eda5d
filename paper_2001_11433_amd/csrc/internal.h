// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <functional>

#include "../../include/mce.h"

namespace mce {

void set_error(const char* fmt, ...);

#define MCE_TRY_HIP(expr)                                                              \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::mce::set_error("%s:%d: %s: %s", __FILE__, __LINE__, #expr, hipGetErrorString(e_)); \
      return (e_ == hipErrorOutOfMemory) ? MCE_ENOMEM : MCE_EDEVICE;                   \
    }                                                                                  \
  } while (0)

#define MCE_TRY(expr)        \
  do {                       \
    int rc_ = (expr);        \
    if (rc_ != MCE_OK) return rc_; \
  } while (0)

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kMaxCand = 8192;  // |cand| per subproblem: 128 words of 64 bits
constexpr uint32_t kBlockWords = 1024;  // one donated-task record
// K list of a search wave in LDS: enough for subproblems whose cliques stay
// below 512 vertices.
constexpr uint32_t kKLds = 512;
// K list capacity of a search wave when a subproblem's cliques can reach 512
// vertices (its LDS list is shorter): any clique within the envelope
// (|K| <= 2 + kMaxCand) plus the compact search's depth margin.
constexpr uint32_t kKBig = kMaxCand + 72;

// Control block of one enumeration launch (uint64 words).
enum {
  // the words that waves poll or update with atomics during the search sit
  // on cache lines of their own (16 words = 128 bytes apart)
  CTL_HEAD = 0,      // next queue slot to claim
  CTL_TAIL = 16,     // next queue slot to fill
  CTL_PENDING = 32,  // tasks queued or running
  CTL_FREE = 48,     // free list of pool blocks: (tag << 32) | first free block
  CTL_TICKETS = 64,  // donation tickets handed out
  CTL_CLQ = 80,      // packed clique-output counter: (cliques << 32) | verts
  CTL_HAND = 88,     // handoff requests: (records << 32) | 64-byte units (may exceed the capacity)
  CTL_HANDOK = 112,  // handoff records written
  // totals, added once per wave at exit (and rare flags)
  CTL_FLAGS = 96,    // bit 0: DFS stack overflow; bit 1: clique counter overflow
  CTL_DONATED = 97,  // donations that reached the queue
  CTL_COUNT = 98,    // maximal cliques
  CTL_HASH = 99,     // sum of clique hashes
  CTL_NODES = 100,   // search nodes
  CTL_OPS = 101,     // algorithmic 32-bit integer operations
  CTL_OPS_EXEC = 102,   // the same at the executed row width
  CTL_LDS_BYTES = 103,  // algorithmic LDS bytes
  CTL_DIAG = 104,    // 8 diagnostic counters (see mce_result.diag)
  CTL_WORDS = 128
};

// Per-subproblem tables, indexed by subproblem id.
struct SubTab {
  const uint64_t* off;   // word offset of the subproblem's bit rows in the arena
  const uint64_t* goff;  // offset of its vertex-id table
  const uint32_t* p;     // |cand| at the root
  const uint32_t* x;     // number of fini vertices that have a cand neighbour
  const uint32_t* r0;    // root clique vertex
  const uint32_t* r1;    // second root clique vertex (edge subproblems) or kNone
};

struct EnumArgs {
  SubTab sub;
  const uint64_t* arena;
  const uint32_t* gids;
  uint64_t* queue;
  uint64_t qcap;
  uint64_t* ctl;
  uint64_t* pool;        // pool_blocks blocks of kBlockWords words (donated task records)
  uint32_t* pool_next;   // free-list links
  uint64_t pool_blocks;
  uint64_t max_tickets;
  uint64_t* stacks;
  uint64_t stack_words;  // per wave
  uint32_t frame_cap;
  uint32_t frame_words;  // max frame size over all subproblems
  uint32_t donate_interval;
  uint32_t pad;
  uint64_t* nodes_v;     // per-subproblem outputs (nullable)
  uint64_t* count_v;
  uint64_t* hash_v;
  uint64_t* cl_off;      // clique output (nullable)
  uint32_t* cl_vert;
  uint64_t cap_cliques, cap_verts;
  uint64_t* hand;        // arena of re-based nodes handed to the compact kernel (nullable)
  uint64_t hand_units;   // its size in 64-byte units
  uint32_t* hand_idx;    // record index -> first unit
  uint64_t hand_cap;     // records (at most 2^26, so the packed request counter cannot carry into
                         // a record that passes both checks)
  uint32_t* kbig;        // per-wave K lists of kKBig entries (gridDim.x of them), for subproblems with
                         // |cand| + |K at the root| + 2 > 512; null when no subproblem needs them
  uint64_t* hist;        // clique-size histogram (nullable), hist_len entries, last = hist_len - 1 or more
  uint64_t hist_len;
  uint32_t emit_extra;   // nonzero when cliques are written out or tallied by size (cl_vert or hist)
  uint32_t lds_rows;     // 64-bit words of the per-wave LDS row cache of k_enum (0 = none)
};

// Largest per-wave LDS row cache (keeps k_enum's LDS below 64 KiB per workgroup).
constexpr uint32_t kLdsRowsMax = 4096;

// Sizes below this are tallied per wave in LDS and flushed at exit; larger
// ones go to the histogram with device atomics.
constexpr uint32_t kHistLds = 64;

// A node is handed off only when its K list has at most kHandK vertices.
constexpr uint32_t kHandK = 64;

// Bump allocator over a fixed device region (the scratch array of the
// allocation-free entry point).  While one is installed on the calling thread
// (CarverScope), DevBuf::ensure and the temp-storage helpers take their memory
// from it instead of calling hipMalloc; nothing taken is ever freed.
struct Carver {
  uint8_t* base;
  uint64_t cap, used;
  void* take(uint64_t b) {
    const uint64_t at = (used + 255) & ~255ULL;
    if (at > cap || b > cap - at) return nullptr;
    used = at + b;
    return base + at;
  }
};
Carver*& active_carver();  // the calling thread's, or null
struct CarverScope {
  Carver* prev;
  explicit CarverScope(Carver* c) : prev(active_carver()) { active_carver() = c; }
  ~CarverScope() { active_carver() = prev; }
};
// Takes `b` bytes from the active carver (MCE_ENOTSUP with a message when the
// scratch is exhausted).
int carve(void** p, uint64_t b);

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool carved = false;  // taken from a Carver: never freed
  int ensure(size_t b) {
    if (b <= bytes && p) return MCE_OK;
    if (active_carver()) {
      void* q = nullptr;
      int rc = carve(&q, std::max<size_t>(b, 256));
      if (rc != MCE_OK) return rc;
      p = q;
      bytes = std::max<size_t>(b, 256);
      carved = true;
      return MCE_OK;
    }
    if (p) {
      if (!carved) (void)hipFree(p);
      p = nullptr;
      bytes = 0;
      carved = false;
    }
    size_t want = std::max<size_t>(b, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      set_error("hipMalloc(%zu bytes) failed: %s", want, hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? MCE_ENOMEM : MCE_EDEVICE;
    }
    bytes = want;
    return MCE_OK;
  }
  void release() {
    if (p && !carved) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    carved = false;
  }
  template <class T>
  T* as() const {
    return (T*)p;
  }
};


// Buffers of one persistent enumeration launch (queue, control block, task
// pool, DFS stacks).  Each incremental state owns one, so sessions on
// different streams never share them.
struct EnumWork {
  DevBuf queue, ctl, pool, pool_next, stacks, hand, hand_idx, hkeys, hkeys2, hvals, hvals2, kbig;
  void* sort_tmp = nullptr;
  size_t sort_bytes = 0;
  void release() {
    for (DevBuf* b : {&queue, &ctl, &pool, &pool_next, &stacks, &hand, &hand_idx, &hkeys, &hkeys2, &hvals, &hvals2,
                      &kbig})
      b->release();
    if (sort_tmp) (void)hipFree(sort_tmp);
    sort_tmp = nullptr;
    sort_bytes = 0;
    hand_want_recs = hand_want_units = 0;
  }
  uint64_t hand_want_recs = 0, hand_want_units = 0;  // what the last run asked for
};

// One persistent enumeration over a table of subproblems.
struct EnumJob {
  SubTab sub;
  const uint64_t* arena;
  const uint32_t* gids;
  uint64_t nq;             // root tasks
  const uint32_t* order;   // their subproblem ids, in queue order
  const uint32_t* split = nullptr;  // root chunks per subproblem id (1 = run whole); null = none
  uint64_t max_p, max_frame;
  bool excl;               // edge subproblems with excluded edges
  uint64_t *nodes_v, *count_v, *hash_v;
  uint64_t* hist = nullptr;  // clique-size histogram (nullable), zeroed by the caller
  uint64_t hist_len = 0;
  uint64_t* cl_off;
  uint32_t* cl_vert;
  uint64_t cap_cliques, cap_verts;
  const mce_opts* opts;
  std::function<int(uint32_t attempt, uint64_t* ctl_dev)> before_launch;
  // initial handoff arena in 64-byte units when no earlier run sized it
  // (0 = a small default)
  uint64_t hand_initial_units = 0;
  // donation pool blocks and queue tickets (0 = the defaults: 2^16 blocks of
  // 8 KiB, max(2^24, 4 * nq) tickets)
  uint64_t pool_blocks = 0, max_tickets = 0;
  bool timing = true;  // device-time events around the compact launch
  // written by run_enum: compact-kernel time and the nodes handed to it
  double hand_ms = 0;
  uint64_t handed = 0;
};

// Runs the job (restarting with deeper DFS stacks after an overflow) and
// copies the control block to `ctl` (CTL_WORDS words).
int run_enum(EnumJob& j, EnumWork& w, hipStream_t s, uint64_t* ctl, uint32_t* retries);

// Persistent waves of an enumeration launch under these options.
uint32_t enum_grid(const mce_opts& opts);

// rank.hip
hipError_t launch_validate(uint64_t n, const uint64_t* rp, const uint32_t* col, uint32_t* bad, hipStream_t s);
hipError_t launch_degree(uint64_t n, const uint64_t* rp, uint64_t* metric, hipStream_t s);
// MCE_RANK_TTT_ROOT: metric 0 for the children of the whole-graph root, bit 63
// for the root pivot's neighbours (no subproblem of their own); `best` is one
// u64 of scratch.
hipError_t launch_root_metric(uint64_t n, const uint64_t* rp, const uint32_t* col, uint64_t* metric, uint64_t* best,
                              hipStream_t s);
// Level-synchronous peeling (see rank.hip): core number or peel round
// (MCE_RANK_PEEL) of every vertex.  Scratch: deg_scratch and list hold n
// entries each, ctl 8 words.
int run_core_numbers(uint64_t n, const uint64_t* rp, const uint32_t* col, uint64_t* core, uint32_t* deg_scratch,
                     uint32_t* list, uint64_t* ctl, hipStream_t s);
int run_peel_rounds(uint64_t n, const uint64_t* rp, const uint32_t* col, uint64_t* round, uint32_t* deg_scratch,
                    uint32_t* list, uint64_t* ctl, hipStream_t s);
hipError_t launch_triangles(uint64_t n, const uint64_t* rp, const uint32_t* col, uint64_t* tri, hipStream_t s);
hipError_t launch_features(uint64_t n, const uint64_t* rp, const uint32_t* col, const uint64_t* core,
                           const uint64_t* tri, float* feat, hipStream_t s);

// mlp.hip
hipError_t launch_mlp_forward_bf16(const float* prm, const uint16_t* prm16, const float* feat, uint64_t n, float* out,
                                   hipStream_t s);

// build.hip
struct BuildBufs {
  uint32_t* p;       // [n]
  uint32_t* x;       // [n]
  uint32_t* xmark;   // [ceil(2m/32)] fini vertices with a cand neighbour, by CSR position
  uint32_t* lidx;    // [2m] local index of each CSR position in its row's subproblem
  uint64_t* words;   // [n] arena words per subproblem (scan input/output)
  uint64_t* gwords;  // [n]
  uint64_t* stats;   // [8]: 0 max p, 1 max frame words, 2 nontrivial count, 3 count, 4 hash, 5 nodes
};
hipError_t launch_sizes(uint64_t n, const uint64_t* rp, const uint32_t* col, const uint64_t* metric,
                        BuildBufs b, uint64_t* nodes_v, uint64_t* count_v, uint64_t* hash_v, hipStream_t s);
hipError_t launch_mark(uint64_t n, const uint64_t* rp, const uint32_t* col, const uint64_t* metric, BuildBufs b,
                       hipStream_t s);
hipError_t launch_words(uint64_t n, const uint64_t* rp, BuildBufs b, hipStream_t s);
hipError_t launch_build(uint64_t n, const uint64_t* rp, const uint32_t* col, const uint64_t* metric, BuildBufs b,
                        const uint64_t* off, const uint64_t* goff, uint64_t* arena, uint32_t* gids, hipStream_t s);
hipError_t launch_queue_keys(uint64_t n, const uint64_t* rp, const uint32_t* p, mce_sched sched,
                             const uint64_t* tri, const float* cost, uint64_t* keys, uint32_t* vals,
                             uint64_t* count, hipStream_t s);
hipError_t launch_queue_fill(uint64_t nq, const uint32_t* vals, const uint32_t* split, uint64_t* queue,
                             hipStream_t s);
// Root chunks per subproblem from predicted log search nodes (mce_opts.split).
// `total` is one double of scratch.
hipError_t launch_split_plan(uint64_t n, const uint32_t* p, const float* cost, uint32_t waves, uint32_t split_max,
                             double* total, uint32_t* split, hipStream_t s);
int device_exclusive_scan(const uint64_t* in, uint64_t* out, uint64_t n, void*& tmp, size_t& tmp_bytes,
                          hipStream_t s);
// Temp storage of at least `need` bytes in (tmp, tmp_bytes): carved while a
// Carver is active, else grown with hipMalloc.
int ensure_temp(void*& tmp, size_t& tmp_bytes, size_t need);
// Zero `bytes` (a multiple of 4) at p with a fill kernel.
hipError_t dev_zero(void* p, uint64_t bytes, hipStream_t s);
int device_sort_desc(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, uint64_t n,
                     void*& tmp, size_t& tmp_bytes, hipStream_t s, uint64_t** keys_out, uint32_t** vals_out,
                     int end_bit = 64);

// enum.hip
hipError_t launch_enum(const EnumArgs& a, uint32_t grid, bool exclusion, hipStream_t s);
// The compact kernel over `nh` handed-off records already in the queue.
hipError_t launch_compact(const EnumArgs& a, uint32_t grid, bool exclusion, hipStream_t s);
hipError_t launch_queue_fill_hand(uint64_t nh, const uint32_t* order, uint64_t* queue, hipStream_t s);
// Sort keys of the handoff records: candidate count, then fini count.
hipError_t launch_hand_keys(uint64_t nh, const uint64_t* hand, const uint32_t* hand_idx, uint32_t by_sub, uint64_t* keys,
                            uint32_t* vals, hipStream_t s);
hipError_t launch_finish_offsets(uint64_t* off, uint64_t n_cliques, uint64_t n_verts, hipStream_t s);
hipError_t launch_pool_init(uint32_t* next, uint64_t blocks, hipStream_t s);

}  // namespace mce
