/*
 * mce.h - C ABI of the MI355X (gfx950) maximal clique enumeration library.
 *
 * The library implements the shared-memory method of Das, Sanei-Mehri and
 * Tirthapura, "Shared-Memory Parallel Maximal Clique Enumeration from Static
 * and Dynamic Graphs", as GPU kernels:
 *   - mce_static: every maximal clique of a simple undirected graph.  The
 *     problem is split into one subproblem per vertex v (Algorithm 4,
 *     ParMCE): K = {v}, cand = neighbours of higher rank, fini = the rest;
 *     each subproblem is searched by pivoted backtracking (Algorithm 1, TTT;
 *     its unrolled form, Algorithm 3, gives independent children, which the
 *     GPU work queue uses to split large subproblems).
 *   - imce_*: incremental maintenance under batches of edge additions
 *     (Section 5): the new maximal cliques of G+H (Algorithms 5, 6 and 8) and
 *     the cliques of G they subsume (Algorithm 7).
 *
 * Conventions
 *   - A graph is a CSR over vertex ids 0..n-1: row_ptr[n+1] (uint64),
 *     col[row_ptr[n]] (uint32).  Rows are sorted ascending, the adjacency is
 *     symmetric, and there are no self-loops or repeated entries (a simple
 *     undirected graph, Section 3).  An isolated vertex v forms the maximal
 *     clique {v}; n = 0 has no maximal cliques.
 *   - `on_device` != 0 means the pointer is HIP device memory of the current
 *     device; 0 means host memory.  Input arrays are borrowed for the call.
 *   - Every call runs on `opts->hip_stream` (NULL = the default stream) and
 *     returns after the results are complete.
 *   - Return values: MCE_OK (0) or a negative MCE_E* code; mce_strerror()
 *     names it and mce_last_error() gives the calling thread's last detailed
 *     message.  On error the output structs are unspecified unless stated.
 *   - The clique-set hash of a set S of cliques is
 *         H(S) = sum over c in S of hc(c)            (mod 2^64)
 *         hc(c) = mix(sum over v in c of mix(v) + |c| * 0x9E3779B97F4A7C15)
 *     with mix the splitmix64 output function (add 0x9E3779B97F4A7C15, then
 *     x ^= x>>30; x *= 0xBF58476D1CE4E5B9; x ^= x>>27; x *= 0x94D049BB133111EB;
 *     x ^= x>>31).  It does not depend on the order of cliques or of vertices.
 *   - The pivot of a search node is, among the vertices u of cand u fini that
 *     maximise |cand n Gamma(u)|, the one with the smallest id; the children
 *     are visited in ascending id.  With these two choices the recursion tree,
 *     and so the node count, is fully determined.
 */
#ifndef MCE_MI355X_H
#define MCE_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCE_OK 0
#define MCE_EINVAL (-1)  /* bad argument: malformed CSR, id >= n, self-loop in a batch, NULL pointer */
#define MCE_ENOMEM (-2)  /* device allocation failed */
#define MCE_ENOSPC (-3)  /* a caller clique buffer is too small; required sizes written back */
#define MCE_EDEVICE (-4) /* HIP runtime error */
#define MCE_ENOTSUP (-5) /* input outside the supported envelope (see mce_static) */
#define MCE_ECANCELED (-6) /* a submitted batch was dropped because an earlier one failed (imce_submit) */

typedef struct {
  uint64_t n;               /* number of vertices */
  const uint64_t* row_ptr;  /* n+1 entries, row_ptr[0] = 0 */
  const uint32_t* col;      /* row_ptr[n] entries */
  int on_device;
} mce_csr;

/* Rank used to give each clique to exactly one subproblem (Section 4.2):
 * rank(v) = (metric(v), id(v)) compared lexicographically, metric = degree,
 * core number (degeneracy), or number of triangles through v.  Subproblem v
 * reports exactly the cliques in which v has the lowest rank. */
typedef enum {
  MCE_RANK_DEGREE = 0,
  MCE_RANK_DEGENERACY = 1,
  MCE_RANK_TRIANGLE = 2,
  /* No per-vertex ownership: Algorithm 3 (ParTTT) applied to the root of
   * Algorithm 1 on the whole graph (K = {}, cand = V, fini = {}).  The root's
   * pivot u is a vertex of largest degree (smallest id on ties) and every
   * q in ext = V \ Gamma(u), in ascending id, becomes a task with
   * cand = Gamma(q) minus the earlier ext vertices and fini = Gamma(q) n the
   * earlier ext vertices (Algorithm 3's child formula).  The root counts as
   * one search node; per-vertex outputs describe the root's children.
   * mce_rank_metric writes 0 for the children and 2^63 for u's neighbours. */
  MCE_RANK_TTT_ROOT = 3,
  /* metric = peel round: the degeneracy ordering (Eppstein, Loeffler and
   * Strash) taken in synchronous rounds.  Level k starts at 0; a round
   * removes at once every remaining vertex whose remaining degree is <= k and
   * gives it the round's index; a round that would remove nobody instead
   * raises k to the smallest remaining degree and is not counted.  Every
   * vertex then has at most core(v) neighbours of higher rank, so no cand set
   * exceeds the degeneracy.  The rounds depend on the graph only. */
  MCE_RANK_PEEL = 4
} mce_rank;

/* Order in which subproblems enter the work queue (largest key first).  It
 * changes only the schedule, never the cliques, hashes or node counts. */
typedef enum {
  MCE_SCHED_DEGREE = 0,   /* vertex degree */
  MCE_SCHED_TRIANGLE = 1, /* triangles through the vertex */
  MCE_SCHED_COST = 2,     /* caller-supplied per-vertex float cost, any real value (e.g. a learned
                             model's predicted log search nodes) */
  MCE_SCHED_ID = 3,       /* ascending vertex id */
  MCE_SCHED_MLP = 4       /* the learned cost model, evaluated inside the call: the features of
                             mce_features (core numbers and triangles reused when the rank already
                             computed them) and the bfloat16 forward of mce_mlp_forward_bf16, on a
                             second stream while the subproblems are built; the predicted log search
                             nodes order the queue as MCE_SCHED_COST would, and drive `split` */
} mce_sched;

typedef struct {
  mce_sched sched;
  int validate;             /* != 0: check the CSR on the device first (MCE_EINVAL if malformed) */
  void* hip_stream;         /* hipStream_t; NULL = default stream */
  const float* sched_cost;  /* MCE_SCHED_COST: device array of n costs, larger = scheduled earlier */
  /* tuner overrides, 0 = library default */
  uint32_t waves_per_cu;    /* persistent enumeration waves per compute unit */
  uint32_t donate_interval; /* search nodes between checks for idle waves */
  uint32_t frame_cap;       /* initial DFS frames per wave (grows on demand) */
  /* Root splitting, MCE_SCHED_COST only; 0 = off.  sched_cost[v] is then read
   * as the natural log of subproblem v's predicted search nodes.  A subproblem
   * predicted above one wave's share of the total (the total over the launch's
   * waves) has its root's children dealt out at launch, in up to `split`
   * chunks of consecutive children (Algorithm 3's child formula makes each
   * chunk a self-contained task).  Never changes results. */
  uint32_t split;
  /* Nodes re-based onto the compact 64 + 64 universe are handed to a second,
   * low-register kernel with more waves per SIMD.  Its waves per CU (0 =
   * library default), or inline_compact != 0 to search them in the first
   * kernel instead.  Neither changes results. */
  uint32_t compact_waves_per_cu;
  uint32_t inline_compact;
  /* Order of the handed-off nodes in the compact kernel's queue: 0 = as
   * produced, 1 = largest candidate set first, 2 = grouped by subproblem
   * (records that gather rows of the same subproblem are claimed together,
   * so the rows are read from L2 rather than from HBM).  Never changes
   * results. */
  uint32_t compact_order;
  /* Bit rows of a wide subproblem (over 64 candidates) in LDS: per-wave row
   * cache of this many 64-bit words (0 = none, at most 4096).  A subproblem
   * whose rows over its candidate columns fit ((|cand| + |relevant fini|) *
   * ceil(|cand|/64) words) is searched from LDS, a wider one from device
   * memory (the width classes of the search).  Never changes results. */
  uint32_t lds_row_words;
  /* Device memory for the search's handoff records, in MiB (0 = 16384, at
   * most 65536).  A node re-based for the compact kernel is written there as
   * one small record (its subproblem, K and candidate masks; no row data);
   * once the budget is used up, further nodes are searched in place by the
   * first kernel, with the same results, more slowly.  This bounds the call's
   * memory whatever the number of search nodes. */
  uint32_t hand_mb;
  /* MCE_SCHED_MLP: the cost model's parameter block (device memory,
   * mce_mlp_param_count() floats, layout as for mce_mlp_forward; its mu and
   * sigma are used) and its bfloat16 copy from mce_mlp_to_bf16.  Both are
   * read only; NULL for every other schedule. */
  const float* sched_model;
  const uint16_t* sched_model_bf16;
} mce_opts;

typedef struct {
  uint64_t count;       /* number of maximal cliques */
  uint64_t set_hash;    /* H(all maximal cliques) */
  uint64_t nodes_total; /* search nodes (TTT invocations, subproblem roots included) */
  uint64_t donated;     /* subtrees handed to idle waves */
  uint64_t subproblems; /* subproblems that needed a search (|cand| > 0) */
  uint64_t max_cand;    /* largest |cand| of a subproblem */
  uint64_t alg_ops;     /* algorithmic 32-bit integer operations of the search: per node
                           3*s*w + 2*|ext|*w + 2*s, s = |cand u fini| at the node, w =
                           ceil((|cand| + |relevant fini|)/32) of its subproblem's root (the
                           32-bit words of one bit row); leaves count none */
  double rank_ms, build_ms, enum_ms; /* device time of ranking, subproblem build + queue, enumeration */
  uint32_t retries;     /* enumeration restarts after a DFS stack overflow */
  uint32_t pad;
  /* diagnostics of the enumeration kernel: [0] re-based nodes, [1] nodes
     searched in compact form, [2..5] shader clock cycles summed over waves
     spent in wide nodes, re-basing, compact nodes and waiting for work, [6]
     cycles spent donating, [7] (tasks << 32) | donation attempts */
  uint64_t diag[8];
  double compact_ms;    /* device time of the compact kernel (included in enum_ms) */
  uint64_t handed;      /* re-based nodes it searched (the rest were searched in place) */
  uint64_t exec_ops;    /* alg_ops at the row width the kernels execute: w = 2 * ceil(|cand|/64)
                           of the subproblem for a wide node, w = 2 for a node re-based onto the
                           compact 64 + 64 universe */
  uint64_t lds_bytes;   /* algorithmic LDS bytes of the search: per node 4 * w * (s + |ext|), w
                           and s as in alg_ops (the compact kernel keeps its rows in registers) */
  uint64_t arena_bytes; /* the subproblems' bit rows and vertex ids the search reads: its
                           algorithmic device-memory bytes (each read once) */
} mce_result;

/* Clique output in CSR form: clique i is vert[off[i] .. off[i+1]), vertices
 * ascending; the order of cliques is unspecified.  The library writes
 * n_cliques / n_verts (the required sizes) always, and the arrays only when
 * both fit (off needs n_cliques+1 entries); otherwise the call returns
 * MCE_ENOSPC after finishing all other outputs.  n_verts must stay below
 * 2^32 per call. */
typedef struct {
  uint64_t cap_cliques, cap_verts;
  uint64_t* off;
  uint32_t* vert;
  int on_device;
  uint64_t n_cliques, n_verts;
} mce_clique_buf;

/* Optional outputs (any pointer may be NULL).  nodes / count / hash: device
 * arrays of n entries, the search nodes, cliques and H(cliques) of
 * subproblem v; node counts are the labels of the learned cost model.
 * size_hist: device array of hist_len >= 2 entries, overwritten with the
 * clique-size distribution the paper reports per graph (Section 6.1):
 * size_hist[k] = number of maximal cliques with k vertices, cliques of
 * hist_len - 1 or more vertices counted in the last entry. */
typedef struct {
  uint64_t* nodes;
  uint64_t* count;
  uint64_t* hash;
  uint64_t* size_hist;
  uint64_t hist_len;
  /* MCE_SCHED_MLP: the predicted cost of every vertex's subproblem (device
   * array of n floats, the values that ordered the queue); NULL = not wanted */
  float* sched_cost;
} mce_per_vertex;

/* All maximal cliques of `g` (Algorithm 4 over Algorithm 1).
 * opts may be NULL (defaults), cliques and per_vertex may be NULL.
 * Supported envelope: n < 2^32, |cand| of every subproblem <= 8192 (else
 * MCE_ENOTSUP; cliques up to 8193 vertices are then found), and for
 * materialised output n_verts < 2^32. */
int mce_static(const mce_csr* g, mce_rank rank, const mce_opts* opts, mce_result* out,
               mce_clique_buf* cliques, const mce_per_vertex* per_vertex);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mce_static
 * with the same arguments, results and errors, except that
 *   - every work buffer is carved from one fixed scratch array of
 *     MCE_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from its
 *     first use on that GPU until the process ends; a call whose buffers do
 *     not fit returns MCE_ENOTSUP and mce_last_error() says how much it asked
 *     (host-resident inputs and outputs are staged through the scratch too);
 *   - no device memory is allocated or freed and no HIP events are created:
 *     rank_ms, build_ms, enum_ms and compact_ms are 0;
 *   - the tables for handing subtrees between waves are smaller (the results
 *     are the same).
 * All calls on one GPU share its scratch, which keeps the last call's
 * contents; the library runs them one at a time per GPU (together with
 * mce_static) and clears what each call needs, so calls from several threads
 * are serialised rather than racing. */
#define MCE_NOALLOC_SCRATCH_BYTES (256ULL << 20)
int mce_static_noalloc(const mce_csr* g, mce_rank rank, const mce_opts* opts, mce_result* out,
                       mce_clique_buf* cliques, const mce_per_vertex* per_vertex);

/* Per-vertex rank metric (Section 4.2) into the device array metric[n]. */
int mce_rank_metric(const mce_csr* g, mce_rank rank, uint64_t* metric, void* hip_stream);

/* Cost-model features of every vertex into the device array feat[n*4]
 * (row-major, float): log1p of degree, core number, triangles through v, and
 * the number of length-2 walks from v (sum over neighbours u of d(u)-1). */
int mce_features(const mce_csr* g, float* feat, void* hip_stream);

/* --- incremental maintenance (Section 5) -------------------------------- */

typedef struct imce_state imce_state; /* opaque: device graph, clique count and set hash */

typedef struct {
  uint64_t n_applied;  /* batch edges added (after canonicalisation) */
  uint64_t n_skipped;  /* batch edges already in G or repeated in the batch */
  uint64_t n_new;      /* |Lambda_new| = |C(G+H) \ C(G)| */
  uint64_t n_del;      /* |Lambda_del| = |C(G) \ C(G+H)| */
  uint64_t hash_new, hash_del; /* H(Lambda_new), H(Lambda_del) */
  uint64_t count, set_hash;    /* |C(G+H)| and H(C(G+H)) after the batch */
  double new_ms, sub_ms, ms;   /* device time: new cliques, subsumed cliques, whole batch */
  uint64_t nodes;              /* search nodes of the batch's edge subproblems */
  uint64_t handed;             /* re-based nodes searched by the compact kernel */
  double compact_ms;           /* device time of the compact kernel (inside new_ms) */
} imce_result;

/* Copies `g` to state-owned device memory and enumerates C(g) once (degree
 * ranking) to initialise the count and set hash.  `initial` may be NULL. */
int imce_create(const mce_csr* g, const mce_opts* opts, imce_state** out, mce_result* initial);

/* Adds the batch H = {(src[i], dst[i])}.  Every pair must have two distinct
 * ids < n, else MCE_EINVAL and the state is unchanged.  Pairs already in G or
 * repeated in the batch are skipped (n_skipped); the survivors, in input
 * order, are e_1..e_rho of Algorithm 5.  new_cl / del_cl (nullable) receive
 * Lambda_new / Lambda_del.  On any error the state is unchanged (the batch is
 * applied atomically).
 * Supported envelope (else MCE_ENOTSUP): every batch edge has at most 4096
 * common neighbours in G+H; a new clique holds at most 256 batch edges and
 * splits into at most 1024 subsets free of batch edges (Algorithm 7); a new
 * clique of more than 64 vertices has at most 64 vertices that are ends of
 * batch edges inside it. */
int imce_add_edges(imce_state* st, const uint32_t* src, const uint32_t* dst, uint64_t rho, int on_device,
                   imce_result* out, mce_clique_buf* new_cl, mce_clique_buf* del_cl);

/* Deletes the batch H = {(src[i], dst[i])} (Section 5.3: the reduction of a
 * deletion to the incremental case on G - H, since G = (G - H) + H).  The
 * cliques of G that hold an edge of H stop being maximal (del_cl, n_del,
 * hash_del; Algorithms 5 and 8 run on G), and those of their subsets free of
 * H edges that are maximal in G - H become maximal (new_cl, n_new, hash_new;
 * Algorithm 7 with its membership test in the form "maximal in G - H").
 * Canonicalisation as in imce_add_edges except that pairs that are not edges
 * of G (and repeats) are skipped.  Same errors, envelope and all-or-nothing
 * commit as imce_add_edges. */
int imce_remove_edges(imce_state* st, const uint32_t* src, const uint32_t* dst, uint64_t rho, int on_device,
                      imce_result* out, mce_clique_buf* new_cl, mce_clique_buf* del_cl);

/* Pipelined updates: the subsumed-clique pass of one batch (Algorithm 7) runs
 * on the device while the next batch's new-clique search (Algorithms 5 and 8)
 * runs, which is what a stream of batches of one session can overlap.
 * imce_submit runs a batch's canonicalisation, the graph update and the
 * new-clique search, starts its subsumed pass on a second stream of the state
 * and returns; remove != 0 makes it a deletion batch (as imce_remove_edges).
 * imce_collect waits for the oldest submitted batch and returns its result and
 * cliques exactly as imce_add_edges / imce_remove_edges would have.  At most
 * two submitted batches may be uncollected (else MCE_EINVAL); imce_add_edges
 * and imce_remove_edges are refused (MCE_EINVAL) while any is.  Errors:
 *   - imce_submit fails like imce_add_edges's first steps and then leaves the
 *     state and the pending batch untouched;
 *   - a failed subsumed pass is returned by imce_collect of that batch; the
 *     graph, count and hash go back to before that batch, and a batch
 *     submitted after it is dropped (its imce_submit returns MCE_ECANCELED);
 *   - MCE_ENOSPC from imce_collect (caller buffers too small, sizes written
 *     back) keeps the batch to be collected again; the batch is applied.
 * The calls of one state must not overlap (one caller thread at a time). */
int imce_submit(imce_state* st, const uint32_t* src, const uint32_t* dst, uint64_t rho, int on_device, int remove);
int imce_collect(imce_state* st, imce_result* out, mce_clique_buf* new_cl, mce_clique_buf* del_cl);

/* Device memory the state holds now (graph buffers, work buffers, tables),
 * and an estimate of what a batch of rho edges may add to it (from the
 * library's own sizing rules; the edge-subproblem rows at the largest bytes
 * per edge seen so far), in bytes: what the admission decision of a serving
 * loop budgets. */
int imce_device_bytes(const imce_state* st, uint64_t* bytes);
int imce_batch_bytes(const imce_state* st, uint64_t rho, uint64_t* bytes);

/* Current graph: n and the number of stored adjacency entries (2m). */
int imce_info(const imce_state* st, uint64_t* n, uint64_t* nnz, uint64_t* count, uint64_t* set_hash);

void imce_destroy(imce_state* st);

/* --- learned cost model (orders the queue only, never changes results) ----
 * A 4 -> 64 -> 64 -> 1 ReLU MLP from the mce_features columns to log(search
 * nodes of the vertex's subproblem).  Parameters are one float block of
 * mce_mlp_param_count() entries, row-major: W1[64][4], b1[64], W2[64][64],
 * b2[64], w3[64], b3, then mu[4], sigma[4] (inputs are standardised as
 * (x - mu) / sigma).  All pointers are device memory; n is the number of
 * vertices (feat is n x 4, row-major). */
uint32_t mce_mlp_param_count(void);
/* FP32 prediction: out[i] = MLP(feat[i]). */
int mce_mlp_forward(const float* params, const float* feat, uint64_t n, float* out, void* hip_stream);
/* BF16 prediction: weights (params_bf16, from mce_mlp_to_bf16), inputs and
 * hidden activations rounded to bfloat16, FP32 accumulation; mu/sigma are
 * read from the FP32 block `params`. */
int mce_mlp_forward_bf16(const uint16_t* params_bf16, const float* params, const float* feat, uint64_t n, float* out,
                         void* hip_stream);
/* Gradient of the mean squared error (1/n) sum (MLP(feat[i]) - target[i])^2
 * with respect to the trainable parameters (all but mu/sigma) into grad
 * (mce_mlp_param_count() floats, overwritten) and the loss into loss[0]. */
int mce_mlp_grad(const float* params, const float* feat, const float* target, uint64_t n, float* grad, float* loss,
                 void* hip_stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the trainable
 * parameters; m and v are zero-initialised moment buffers; step >= 1. */
int mce_mlp_adam(float* params, float* m, float* v, const float* grad, float lr, uint32_t step, void* hip_stream);
/* mu/sigma of the parameter block from the feature columns. */
int mce_mlp_fit_norm(float* params, const float* feat, uint64_t n, void* hip_stream);
/* Round-to-nearest-even bfloat16 copy of the parameter block. */
int mce_mlp_to_bf16(const float* params, uint16_t* params_bf16, void* hip_stream);
/* Training targets: target[i] = log(max(nodes[i], 1)). */
int mce_mlp_labels(const uint64_t* nodes, uint64_t n, float* target, void* hip_stream);

const char* mce_strerror(int code);
const char* mce_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MCE_MI355X_H */
