/*
 * kclique.h -- exact k-clique counting on one AMD Instinct MI355X (gfx950).
 *
 * The library implements the k-clique listing method of "Efficient k-clique
 * Listing with Set Intersection Speedup" (Yuan et al.): Pre-Core and Pre-List
 * preprocessing (Sec. 5, Alg. 3 and Alg. 4), an acyclic orientation by degree
 * (SDegree, Sec. 6, Alg. 5) or by degeneracy with a per-root greedy color
 * ordering and bitmap intersections (BitCol, Sec. 7, Alg. 6), and a recursive
 * listing whose last level is counted.  Every result is an exact unsigned
 * 64-bit integer; no rounding is involved.
 *
 * Graph input (every entry point): a simple undirected graph in CSR form.
 *   n         number of vertices (0 <= n < 2^31)
 *   row_ptr   int32[n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] < 2^31
 *   col_idx   int32[row_ptr[n]], the neighbours of v are
 *             col_idx[row_ptr[v] .. row_ptr[v+1]), strictly ascending, in
 *             [0, n), never v itself; the graph is symmetric (w in N(v) iff
 *             v in N(w)).  Every undirected edge therefore appears twice.
 * Unless the options mark the input trusted, the library checks all of this
 * on the device and returns KC_EINVAL on any violation.
 *
 * k: k >= 1.  k = 1 gives n, k = 2 gives the number of edges, k > n gives 0.
 * (The paper treats k >= 3; the two linear cases follow Sec. 8.)
 *
 * Ownership: the caller owns every buffer.  The library keeps no pointer after
 * returning.  Its device scratch memory comes either from a caller-owned
 * workspace (kc_options.workspace, sized by kclique_workspace_size) or, when
 * none is given, from stream-ordered allocations freed before the call
 * returns; the one exception is a prepared batch (kclique_plan_*), which holds
 * its device memory until it is destroyed.  Calls that share a stream are
 * serialised by it; calls on different streams are independent (they must not
 * share a workspace).
 *
 * Errors: every function returns a kc_status.  On a non-zero status the
 * outputs are unspecified.  No C++ exception crosses this interface.
 */
#ifndef KCLIQUE_H
#define KCLIQUE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KC_OK = 0,
  KC_EINVAL = -1,        /* malformed graph, k < 1, unknown order/schedule/option */
  KC_ENOMEM = -2,        /* device allocation failed */
  KC_EOVERFLOW = -3,     /* a count does not fit in 64 bits (e.g. C(201,20)) */
  KC_EDEVICE = -4,       /* a HIP runtime call failed or no device */
  KC_EUNSUPPORTED = -5,  /* a local subgraph exceeds the supported size: 2048 local vertices (BitCol); above
                            1024 (512 with per-vertex output) only for k <= 5; SDegree candidate lists
                            that do not fit LDS only when counting (no per-vertex or listing output) */
  KC_EWORKSPACE = -6     /* the caller's workspace is smaller than the call needs */
} kc_status;

/* Orientation / algorithm. */
#define KC_ORDER_DEGREE 0 /* SDegree: degree order, sorted-list merge joins (Alg. 5) */
#define KC_ORDER_COLOR 1  /* BitCol: degeneracy order + per-root color order, bitmaps (Alg. 6) */
#define KC_ORDER_CORE 2   /* SDegree's merge joins (Alg. 5) on the degeneracy order: Sec. 6.2 notes that
                             SDegree can take any vertex order; out-degrees are then bounded by core numbers */
#define KC_ORDER_DEGREE_REDUCED 3 /* SDegree with the out-neighbour reduction (Sec. 7.2): Alg. 5 runs on each
                                     root's DAG G_u induced by N+(u), whose out-lists are N+(x) restricted to
                                     N+(u); its pruning uses the out-degree in G_u and its logged work is
                                     |C| + |L_x| per join.  Roots of more than 4096 out-neighbours give
                                     KC_EUNSUPPORTED (the reduced lists hold 16-bit positions of N+(u)
                                     in a per-workgroup pool of d+(d+ - 1)/2 entries). */
#define KC_ORDER_CORE_REDUCED 4   /* the same on the degeneracy order */

/* Ablations (kc_options.disable, bit mask; Sec. 9.2 and 9.4 compare the
 * method with and without its preprocessing and pruning).  None changes a
 * result, only the work done. */
#define KC_NO_PRECORE 1 /* skip Pre-Core (Alg. 3) */
#define KC_NO_PRELIST 2 /* skip Pre-List (Alg. 4) */
#define KC_NO_PRUNE 4   /* SDegree: no d+ <= l-2 skip and no |C'| > l-2 test (children with any member are
                           entered); BitCol: no color(v) < l skip (Sec. 7.1; its size test stays) */

/* Root schedule of the persistent listing kernel (does not change results). */
#define KC_SCHED_DEGREE 0  /* roots ordered and split by DAG out-degree */
#define KC_SCHED_LEARNED 1 /* roots ordered and split by the MLP's predicted work */

/* Number of floats in an MLP parameter block (see kc_mlp_* below). */
#define KC_MLP_IN 4
#define KC_MLP_HIDDEN 64
#define KC_MLP_NPARAMS (KC_MLP_IN * KC_MLP_HIDDEN + KC_MLP_HIDDEN + KC_MLP_HIDDEN * KC_MLP_HIDDEN + KC_MLP_HIDDEN + KC_MLP_HIDDEN + 1)

/* Timings and counters of the last call (filled when kc_options.stats is set). */
typedef struct {
  double total_ms;        /* device time of the whole call (events on its stream) */
  double prep_ms;         /* validation, Pre-Core, Pre-List, orientation */
  double stage_ms;        /* BitCol: local subgraph staging, coloring, encoding */
  double sched_ms;        /* features, MLP inference, binning, task generation */
  double list_ms;         /* the persistent listing kernel(s) */
  int32_t list_launches;  /* listing kernel launches in the call */
  int32_t n_roots;        /* roots with d+ >= k-1 */
  int64_t n_tasks;        /* work items in the queue(s) */
  int32_t max_out_degree; /* largest d+ among roots */
  int32_t max_core;       /* degeneracy (COLOR order only) */
  uint64_t prelist_count; /* cliques reported by Pre-List */
  uint64_t nodes;         /* calls of the listing procedure */
  uint64_t isect;         /* set intersections (merge joins or BitJoins) */
  uint64_t work;          /* SDegree: sum of |C|+d+ per join; BitCol: sum of ceil(s/32) words per BitJoin */
  uint64_t staged_words;  /* BitCol: 32-bit words of encoded bitmaps written */
  uint64_t stage_bytes;   /* BitCol: algorithmic bytes read while staging: 4*(d+_u + sum of d+_v) */
  uint64_t isect_wide;    /* BitCol: of `isect`, BitJoins done as one whole-wave step on full-width bitmaps */
  uint64_t isect_compressed; /* BitCol: of `isect`, BitJoins on re-encoded 64-bit rows (see `compress`) */
  /* per listing launch (BitCol: bitmap word class 1,2,4,8,12,16,24,32,48,64; SDegree: candidate-list
   * class of at most 64, 256, 1024, 4096, 16384, 65536 entries) */
  double class_ms[10];     /* device time of that class's persistent listing kernel */
  uint64_t class_work[10]; /* its work, as `work` above */
  int64_t class_tasks[10]; /* its queue length */
} kc_stats;

typedef struct {
  int32_t device_ptrs;    /* 1: row_ptr, col_idx and every output are device pointers */
  void* stream;           /* hipStream_t; NULL = the default stream */
  int32_t trusted_input;  /* 1: skip the O(m log d) CSR validation */
  int32_t schedule;       /* KC_SCHED_DEGREE (default) or KC_SCHED_LEARNED */
  const float* mlp_params;/* LEARNED: device pointer, KC_MLP_NPARAMS floats */
  const float* mlp_norm;  /* LEARNED: device pointer, 8 floats: feature mean[4], std[4] (of log1p features) */
  int32_t waves_per_root; /* BitCol waves sharing one root's bitmaps: 0 = auto (16 for roots of more than 512
                             out-neighbours, 8 above 128, 4 above 64, else 1), 1, 4, 8 or 16 (others round
                             down; 16 applies to the 24- and 32-word classes when counting, where one
                             workgroup per CU is all the LDS holds, and means 8 elsewhere) */
  int32_t chunk;          /* tasks taken per queue access: 0 = auto */
  int32_t split;          /* heavy-root splitting: 0 = auto, -1 = never, 1/2 = force that depth for heavy roots */
  float split_threshold;  /* 0 = auto: schedule key above which roots are split */
  int32_t compress;       /* BitCol node re-encoding: the largest candidate set re-encoded into rows
                             of one 64-bit word (sets <= 64) or, when counting without per-vertex
                             output, two words (sets of 65..128).  0 = auto (128 when counting, 64
                             per-vertex), -1 = off, else capped at those values */
  int32_t compress_level; /* BitCol: re-encode only nodes of level >= this (0 = auto) */
  int32_t class_streams;  /* BitCol: listing kernels of the word classes 1 = one after another on `stream`,
                             2 = concurrently on streams of their own, 0 = auto (1 for the learned
                             schedule, 2 for the degree schedule) */
  int32_t disable;        /* ablation bit mask of KC_NO_PRECORE, KC_NO_PRELIST, KC_NO_PRUNE (0 = the method) */
  int32_t split_policy;   /* BitCol: which roots are split into depth-1 / depth-2 work items, given each
                             root's work estimate (the schedule's key).  0 = the schedule's own (2 for
                             LEARNED, 1 for DEGREE); 1 = fixed counts: per word class the slots/4
                             roots of highest key split twice, the next 4 x slots once (slots = 4 per
                             CU); 2 = shares: a root whose estimate exceeds 1/(8 slots) of its class's
                             estimated total splits once, 64 such shares twice.  DEGREE with policy 2
                             isolates what the MLP's estimates add over log C(d+, k-1). */
  /* optional per-vertex logs, device pointers of n entries (NULL = off):
   * the root's listing work (as kc_stats.work) and its features */
  uint64_t* root_work;
  uint64_t* root_isect;
  float* root_features;   /* n x 4: d+_u, core(u), colors of G_u, |E_u| (BitCol only) */
  uint64_t* root_count;   /* cliques attributed to each vertex: those listed from it as a root, plus the
                             Pre-List cliques of a clique component at its smallest vertex (sums to the total) */
  const int32_t* vertex_k;/* device pointer, n entries, or NULL: a k per vertex (constant on every
                             connected component; the k argument must be their maximum).  Used to count
                             many graphs with different k in one call. */
  const uint8_t* root_mask;/* device pointer, n entries, or NULL (= every vertex): a share of the roots.
                             Only vertices u with root_mask[u] != 0 are listed from as roots (Theorem 1
                             gives each k-clique exactly one root, its first vertex in the orientation),
                             and the Pre-List cliques of a clique component (Alg. 4) are reported when
                             the mask is set at the component's smallest vertex.  Preprocessing and the
                             orientation still see the whole graph, so over masks that partition the
                             vertices the counts, per-vertex values and listed rows add up to those of
                             the unmasked call.  Requires device_ptrs and k >= 3 (else KC_EINVAL,
                             KC_EUNSUPPORTED); not for batched calls and plans (KC_EINVAL). */
  void* workspace;        /* device memory owned by the caller, or NULL: the call takes all its scratch
                             memory from it (no device allocation by the library); its contents on
                             entry are irrelevant and on return unspecified.  At least the size
                             kclique_workspace_size reports for the same arguments and options. */
  size_t workspace_bytes;
  kc_stats* stats;        /* host pointer or NULL */
} kc_options;

/* Zero-filled options = defaults. */
void kc_options_init(kc_options* opt);

/* Number of k-cliques (Sec. 3.1: all k-cliques of G).  row_ptr, col_idx and
 * count_out are host pointers.  order: KC_ORDER_DEGREE or KC_ORDER_COLOR. */
int kclique_count(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k, int32_t order,
                  uint64_t* count_out);

/* Per-vertex participation: per_vertex_out[v] = number of k-cliques that
 * contain v (host array of n entries); count_out (nullable) = total.  The
 * per-vertex values sum to k times the total.  Each clique found by the
 * listing (the emit points of Alg. 5 and Alg. 6) or by Pre-List (Alg. 4,
 * C(n_c - 1, k - 1) per member of a clique component) is credited to each of
 * its k vertices. */
int kclique_list_per_vertex(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k, int32_t order,
                            uint64_t* per_vertex_out, uint64_t* count_out);

/* Full form of both calls (Sec. 3.1; Alg. 3-6).  per_vertex_out may be NULL
 * (count only).  With opt->device_ptrs the graph and outputs live in device
 * memory. */
int kclique_count_ex(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k, int32_t order,
                     const kc_options* opt, uint64_t* count_out, uint64_t* per_vertex_out);

/* Listing (Sec. 3.1: report every k-clique of G).  Each k-clique is written
 * exactly once (Theorem 1) as a row of k int32 vertex ids -- the emit steps of
 * Alg. 5 (SDegree, R + {u, v} at l = 2) and Alg. 6 (BitCol, R + {v, w} at
 * l = 2), and, for the clique components Pre-List removes (Alg. 4), each of
 * their k-subsets.  cliques_out holds `capacity` rows, row-major (capacity x k
 * int32; device memory if opt->device_ptrs, else host); the order of the
 * rows and of the ids inside a row is unspecified.  *count_out receives the
 * total number of k-cliques and *written_out the rows written,
 * min(total, capacity): when the total exceeds the capacity the rows written
 * are some `capacity` of the cliques (the count is still exact).  k >= 1 (k =
 * 1: one row per vertex; k = 2: one row (u, v), u < v, per edge).  Options as
 * for kclique_count_ex; the schedule, the per-root logs and vertex_k do not
 * apply (vertex_k gives KC_EINVAL). */
int kclique_list(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k, int32_t order,
                 const kc_options* opt, int32_t* cliques_out, int64_t capacity, int64_t* written_out,
                 uint64_t* count_out);

/* Scratch memory a kclique_count_ex call with the same arguments and options
 * needs when it takes it from kc_options.workspace; per_vertex = 1 when that
 * call passes per_vertex_out.  The workspace fields and the per-root log
 * pointers of `opt` are ignored here (nothing of the caller's is written).
 * The amount depends on the graph itself -- the staged bitmaps of Sec. 7.3
 * and the work items follow the out-degrees of the oriented graph after
 * Pre-Core and Pre-List -- so the query runs the call's preparation
 * (validation, Sec. 5 preprocessing, orientation, staging, scheduling) on the
 * device, with scratch it allocates and frees itself, and stops before the
 * listing.  *bytes receives the size (a multiple of 256).  Errors as for
 * kclique_count_ex (a malformed graph gives KC_EINVAL here already). */
int kclique_workspace_size(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k, int32_t order,
                           int32_t per_vertex, const kc_options* opt, size_t* bytes);

/* Allocation-free variant of kclique_count_ex, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): arguments, results and errors as for
 * kclique_count_ex, but the call's scratch is a fixed 256 MiB array inside the
 * library's device code (held by each GPU the library runs on until the
 * process ends), and the call allocates nothing and creates no stream or
 * event (class_streams is taken as 1; opt->stats and opt->workspace are
 * ignored).  A call that needs more scratch than 256 MiB (see
 * kclique_workspace_size) returns KC_EWORKSPACE.  Calls on one GPU share the
 * array: calls that overlap on one GPU race and must be serialised by the
 * caller (one stream, or host synchronisation). */
int kclique_count_noalloc(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k, int32_t order,
                          const kc_options* opt, uint64_t* count_out, uint64_t* per_vertex_out);

/* Many independent graphs in one call (each counted as in Sec. 3.1, all in
 * one preprocessing pass and one listing launch per bitmap class, as the
 * disjoint union with a k per vertex): graph g has n[g] vertices, its rows
 * start at row_ptr_cat[row_off[g]] (n[g]+1 entries, local offsets starting at
 * 0) and its columns at col_idx_cat[col_off[g]] (local vertex ids).  k[g] per
 * graph.  counts_out[g] receives graph g's count.  Pointers follow
 * opt->device_ptrs for the concatenated arrays and counts_out; n, row_off,
 * col_off and k are always host arrays. */
int kclique_count_batched(int32_t num_graphs, const int32_t* n, const int64_t* row_off, const int64_t* col_off,
                          const int32_t* row_ptr_cat, const int32_t* col_idx_cat, const int32_t* k, int32_t order,
                          const kc_options* opt, uint64_t* counts_out);

/* ---- prepared batches, replayed as a HIP graph --------------------------
 * For callers that count the same batch repeatedly, or launch it from a loop
 * that cannot afford the per-call host work: the preparation (validation,
 * Pre-Core, Pre-List, orientation, staging, coloring, encoding, scheduling;
 * Sec. 5-7) runs once, and the listing phase with the per-graph sums is
 * captured into a HIP graph that every execution replays.  BitCol order only
 * (KC_ORDER_COLOR; otherwise KC_EUNSUPPORTED).  Arguments as for
 * kclique_count_batched; the options' schedule, MLP, waves, chunking,
 * splitting and re-encoding apply (class_streams is forced to 1; per-root
 * logs and statistics are not produced).  The plan owns its device memory
 * (the union graph, the staged bitmaps, the queues) until kclique_plan_destroy,
 * and the caller's graph arrays are not read after kclique_plan_batched
 * returns.  A plan belongs to the device that was current when it was made. */
typedef struct kc_plan kc_plan;

int kclique_plan_batched(int32_t num_graphs, const int32_t* n, const int64_t* row_off, const int64_t* col_off,
                         const int32_t* row_ptr_cat, const int32_t* col_idx_cat, const int32_t* k, int32_t order,
                         const kc_options* opt, kc_plan** plan_out);

/* Replays the plan on `stream` (NULL = default stream) and writes the
 * per-graph counts to counts_out (device memory if the plan was made with
 * device_ptrs, else host).  Returns when the counts are written.  Calls on
 * one plan must not overlap (they share its buffers).  KC_EOVERFLOW as for
 * kclique_count_batched. */
int kclique_plan_execute(kc_plan* plan, void* stream, uint64_t* counts_out);

/* Releases the plan's device memory and graph. */
int kclique_plan_destroy(kc_plan* plan);

/* ---- learned scheduling: MLP 4 -> 64 -> 64 -> 1, ReLU, FP32 -------------
 * Parameter block layout (KC_MLP_NPARAMS floats, row-major):
 *   W1[64][4], b1[64], W2[64][64], b2[64], W3[64] (1 x 64), b3[1].
 * y = W3 relu(W2 relu(W1 x + b1) + b2) + b3.  All pointers are device
 * pointers; calls are ordered on `stream` (NULL = default stream). */

/* y[i] = MLP(x[i]) for i < rows; x is rows x 4 (row-major). */
int kc_mlp_forward(const float* params, const float* x, int32_t rows, float* y, void* stream);

/* One training step on a minibatch: mean squared error between MLP(x) and
 * target; grad (KC_MLP_NPARAMS) receives d loss / d params, loss_out (one
 * float, device) the loss.  Then, if lr > 0, one Adam step (Kingma and Ba)
 * with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 updates params in place using
 * the moment buffers m, v (KC_MLP_NPARAMS each) and the 1-based step t.
 * workspace: device scratch of at least kc_mlp_workspace_size(rows) bytes
 * owned by the caller, or NULL (the library allocates and frees it).
 * Gradients are summed in a fixed order: identical inputs give identical
 * bits. */
int kc_mlp_train_step(float* params, const float* x, const float* target, int32_t rows, float* grad, float* loss_out,
                      float* m, float* v, int32_t t, float lr, void* workspace, size_t workspace_bytes,
                      void* stream);

/* Scratch bytes kc_mlp_train_step needs for a minibatch of `rows` rows. */
int kc_mlp_workspace_size(int32_t rows, size_t* bytes);

const char* kc_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* KCLIQUE_H */
