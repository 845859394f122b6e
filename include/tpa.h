/*
 * tpa.h -- C ABI of the MI355X (gfx950) implementation of TPA's hot path.
 *
 * Method: Yoon, Jung, Kang, "TPA: Fast, Scalable, and Accurate Method for
 * Approximate Random Walk with Restart on Billion Scale Graphs".
 *   RWR:        r = (1-c) A~^T r + c q                      (Section 2.2)
 *   CPI:        x(0) = c q,  x(i) = (1-c) A~^T x(i-1),  r = sum_i x(i)
 *                                                      (Section 2.3, Alg. 1)
 *   TPA:        r_TPA = r_family + r~_neighbor + r~_stranger    (Section 3)
 *     r_family    = x(0) + ... + x(S-1)          (online, per seed, Alg. 3)
 *     r~_neighbor = ((1-c)^S - (1-c)^T) / (1 - (1-c)^S) * r_family
 *                                               (Section 3.2, Lemma 2)
 *     r~_stranger = the PageRank terms x'(T) + x'(T+1) + ..., with
 *                   x'(0) = (c/n) 1           (preprocessing, Alg. 2, 3.1)
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers on the current HIP device
 *     unless the argument's comment says "host".  The caller owns them.
 *   - Work is enqueued on `stream` and returns without synchronising,
 *     except where a comment says "synchronous" (graph construction,
 *     export of sizes).  A NULL stream is the default stream.
 *   - Nothing throws across the ABI.  Each call returns a tpa_status; the
 *     text of the last failure on the calling thread is available from
 *     tpa_last_error_message().  A failed call leaves the handle usable.
 *   - A tpa_graph_t owns its device arrays (both orientations of A~, the
 *     stranger vector, work schedules and workspace).  It may be used by
 *     one stream at a time; after tpa_preprocess it is read-only for
 *     queries, which share the handle's workspace (serialise queries on
 *     one stream, or use one handle per stream).
 *   - Computation is FP32 with FP32 accumulation (compensated summation for
 *     the stranger tail); node ids are int32, edge offsets int64.  Results
 *     are deterministic: the same call on the same inputs gives the same
 *     bits (no floating-point atomics).
 */
#ifndef TPA_H
#define TPA_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tpa_status {
    TPA_OK = 0,
    TPA_ERR_INVALID_ARG = -1,      /* bad size, pointer, parameter or node id   */
    TPA_ERR_NOT_PREPROCESSED = -2, /* query/backward before tpa_preprocess      */
    TPA_ERR_PARAM_MISMATCH = -3,   /* query (c, T) differs from preprocess      */
    TPA_ERR_OUT_OF_MEMORY = -4,    /* device allocation failed                  */
    TPA_ERR_HIP = -5,              /* a HIP runtime call failed                 */
    TPA_ERR_INDEX_OVERFLOW = -6,   /* node count does not fit int32 ids         */
    TPA_ERR_CAPTURE = -7           /* would allocate while the stream captures  */
} tpa_status;

typedef struct tpa_graph *tpa_graph_t;

/* ------------------------------------------------------------------------
 * Graph construction (synchronous on `stream`).
 *
 * Every constructor produces the row-normalised adjacency A~ of Section 2
 * (Table 1): duplicate edges are merged, each node without an out-edge gets
 * a self-loop (so every row of A~ sums to 1, as Theorem 1 and Lemma 2
 * require), and A~_uv = 1/outdeg(u) in FP32 (IEEE division).  Both A~ (rows
 * = sources) and A~^T (rows = destinations) are stored, columns ascending,
 * int64 row offsets, int32 column ids.
 * ---------------------------------------------------------------------- */

/* R-MAT graph on `n_nodes` nodes (n_nodes <= 2^scale; 0 means 2^scale):
 * raw sample e draws `scale` quadrants, most significant bit first, level l
 * from the top 32 bits of the (e*scale + l)-th output of SplitMix64 seeded
 * with `seed`; quadrant probabilities (a, b, c, 1-a-b-c) map to (u bit,
 * v bit) = (0,0), (0,1), (1,0), (1,1).  Samples with an endpoint >= n_nodes
 * are rejected; `samples` accepted samples are kept.
 * Errors: INVALID_ARG (scale outside 1..31, samples < 0, bad probabilities,
 * n_nodes > 2^scale), OUT_OF_MEMORY, HIP. */
tpa_status tpa_graph_rmat(int scale, int64_t n_nodes, int64_t samples, uint64_t seed,
                          double a, double b, double c, hipStream_t stream,
                          tpa_graph_t *out);

/* Graph from an edge list src[i] -> dst[i], i < m, node ids in [0, n).
 * `device_ptrs` != 0: src/dst are device pointers; 0: host pointers.
 * Errors: INVALID_ARG (n < 1, m < 0, null pointer, id out of range -- the
 * range check is synchronous), INDEX_OVERFLOW (n > 2^31 - 1), OOM, HIP. */
tpa_status tpa_graph_from_edges(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                                int device_ptrs, hipStream_t stream, tpa_graph_t *out);

/* Block-diagonal packing of `count` graphs into one (node ids of graph g
 * are offset by the node counts of graphs 0..g-1).  Each block keeps its
 * own PageRank restart c/n_g in tpa_preprocess, so queries on the packed
 * graph equal queries on each graph alone.  The inputs stay valid and are
 * not modified; edge logits are not carried over.
 * Errors: INVALID_ARG (count < 1, null handle), INDEX_OVERFLOW, OOM, HIP. */
tpa_status tpa_graph_pack(const tpa_graph_t *graphs, int count, hipStream_t stream,
                          tpa_graph_t *out);

tpa_status tpa_graph_destroy(tpa_graph_t g);

/* Sizes (host outputs; any may be NULL). nblocks is 1 unless packed. */
tpa_status tpa_graph_info(tpa_graph_t g, int64_t *n, int64_t *m, int64_t *nblocks);

/* Device memory the handle holds, in bytes (host output): both CSR
 * orientations and per-node arrays, the gather layout's arrays, the work
 * schedules, the query workspace, kept iterates and tpa_backward's cached
 * buffers (the requested sizes, before allocator rounding).  Query graphs
 * (tpa_query_graph_create) hold their own workspace and are not counted.
 * Errors: INVALID_ARG (NULL). */
tpa_status tpa_graph_device_bytes(tpa_graph_t g, size_t *bytes);

/* A counter (host output) that changes whenever the graph's weights or its
 * preprocessed state change: each tpa_graph_set_logits and each
 * tpa_preprocess call moves it on.  A caller that keeps results derived
 * from one state (for example a forward pass awaiting its derivative)
 * compares it to tell whether the handle still holds that state.
 * Errors: INVALID_ARG (NULL). */
tpa_status tpa_graph_version(tpa_graph_t g, uint64_t *version);

/* Host copy of the block offsets (nblocks + 1 entries). */
tpa_status tpa_graph_blocks(tpa_graph_t g, int64_t *offsets_host);

/* Copy one orientation out: transpose = 0 gives A~ (rows = sources),
 * 1 gives A~^T (rows = destinations).  row_ptr int64[n+1], col int32[m],
 * w float[m] (the current weights); any of them may be NULL. */
tpa_status tpa_graph_export(tpa_graph_t g, int transpose, int64_t *row_ptr, int32_t *col,
                            float *w, hipStream_t stream);

/* mask[u] = 1 where the builder added a self-loop (u had no out-edge). */
tpa_status tpa_graph_padded(tpa_graph_t g, uint8_t *mask, hipStream_t stream);

/* Per-edge logits theta (float[m], A~ order): A~_uv becomes the softmax of
 * theta over u's out-edges.  NULL restores 1/outdeg.  Invalidates the
 * stranger vector (tpa_preprocess must run again).  Errors: INVALID_ARG,
 * OOM, HIP. */
tpa_status tpa_graph_set_logits(tpa_graph_t g, const float *theta, hipStream_t stream);

/* ------------------------------------------------------------------------
 * TPA.
 * ---------------------------------------------------------------------- */

/* Preprocessing phase (Algorithm 2, Section 3.1): r~_stranger = sum of
 * x'(i) for T <= i <= K, x'(0) = (c/n_g) on every node of block g.  K is
 * the first i with c(1-c)^i < eps -- Algorithm 1's L1 break evaluated with
 * Lemma 2's closed form ||x'(i)||_1 = c(1-c)^i per block -- so K = 116 at
 * c = 0.15, eps = 1e-9.  tpa_preprocess uses eps = 1e-9 (the paper's
 * setting, Section 4.1).  Errors: INVALID_ARG (c outside (0,1), T < 0,
 * eps <= 0), OOM, HIP. */
tpa_status tpa_preprocess(tpa_graph_t g, double c, int T, hipStream_t stream);
tpa_status tpa_preprocess_ex(tpa_graph_t g, double c, int T, double eps, hipStream_t stream);

/* The neighbor scale of Section 3.2 (host output): r~_neighbor = scale *
 * r_family with scale = ((1-c)^S - (1-c)^T) / (1 - (1-c)^S), the ratio of
 * the norms Lemma 2 gives; tpa_query's combine multiplies the family part
 * by 1 + scale.  Errors: INVALID_ARG (NULL, c outside (0,1), S < 1,
 * T < S). */
tpa_status tpa_neighbor_scale(double c, int S, int T, double *scale);

/* Parameters of the last tpa_preprocess (host outputs, any may be NULL):
 * c, T, eps and K, the last iteration of the stranger chain (the first i
 * with c (1-c)^i < eps).  Errors: INVALID_ARG (NULL graph),
 * NOT_PREPROCESSED. */
tpa_status tpa_preprocess_info(tpa_graph_t g, double *c, int *T, double *eps, int64_t *K);

/* Copy r~_stranger (float[n]) out.  Errors: NOT_PREPROCESSED. */
tpa_status tpa_stranger(tpa_graph_t g, float *out, hipStream_t stream);

/* Online phase (Algorithm 3) for k seed nodes: out[j*n + v] = r_TPA of
 * seed seeds[j] at node v (seed-major float[k][n]).  r_family is computed
 * in Horner form y <- c q + (1-c) A~^T y (S-1 steps; same sum), the neighbor
 * scale uses Lemma 2's closed form, and the combine
 * out = (1 + scale) y + r~_stranger is fused into the last step.
 * Requires S >= 1, T >= S, and (c, T) equal to tpa_preprocess's.
 * Seeds must lie in [0, n); the check runs on the device: an out-of-range
 * seed makes its output row all NaN and sets the sticky error returned by
 * tpa_get_device_error.  On a packed graph this computes over the whole
 * packed node set (use tpa_query_packed for per-block seeds).
 * Errors: INVALID_ARG, NOT_PREPROCESSED, PARAM_MISMATCH, OOM, HIP,
 * CAPTURE (workspace would have to grow during stream capture: call
 * tpa_reserve first). */
tpa_status tpa_query(tpa_graph_t g, const int32_t *seeds, int64_t k, double c, int S, int T,
                     float *out, hipStream_t stream);

/* tpa_query for callers that cannot allocate device memory (code under HIP
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results as tpa_query (bitwise), but the workspace is
 * a fixed device array inside the library, 64 MiB per device, held from the
 * first call on a device until the process ends, and no call here allocates
 * or frees device memory.  The work schedule of the seed tile tpa_query
 * would use must exist already: tpa_preprocess builds the single-seed one;
 * for k > 1 call tpa_reserve(g, k) (or one tpa_query of k seeds) first.
 * The workspace a query needs is tpa_query_workspace_size's figure without
 * the dense-restart tile: about 16 bytes per node for one seed and 8*kt
 * more per node for a seed tile of kt columns, and for a tile whose second
 * step may be pushed (tpa_set_tile_push_limit) its push buffer: 8*kt bytes
 * per node, about 400 KB of plan and m/8 bytes of pieces, cleared per
 * call.  Every call on one device
 * shares the array (the state the previous call left is cleared where it
 * must start at zero), so calls that overlap on one device, from any
 * stream, thread or graph, race and must be serialised by the caller.
 * Errors: as tpa_query, and INVALID_ARG when the schedule is missing or the
 * workspace would exceed the 64 MiB (the message gives the size needed). */
tpa_status tpa_query_noalloc(tpa_graph_t g, const int32_t *seeds, int64_t k, double c, int S, int T,
                             float *out, hipStream_t stream);

/* Online phase on a block-diagonal graph with `per_block` seed slots per
 * block: seeds[b*per_block + j] is a node of block b; out[j*n + v] is the
 * r_TPA of block(v)'s j-th seed at node v (float[per_block][n]).  One
 * SpMM over all blocks.  Errors as tpa_query; a seed outside its block
 * counts as out of range. */
tpa_status tpa_query_packed(tpa_graph_t g, const int32_t *seeds, int per_block, double c,
                            int S, int T, float *out, hipStream_t stream);

/* Online phase for dense restart vectors: q[j*n + v] is restart vector j
 * (seed-major float[k][n]; Algorithm 1's q, e.g. 1/|set| over a seed set).
 * x(0) = c q_j, same steps and combine as tpa_query; out as tpa_query.  On a
 * packed graph, column j holds every block's j-th restart vector.  Errors
 * as tpa_query (no seed check). */
tpa_status tpa_query_dense(tpa_graph_t g, const float *q, int64_t k, double c, int S, int T,
                           float *out, hipStream_t stream);

/* Reverse-mode derivative (an extension of the method) of
 *   L = sum_j sum_v grad_out[j*n + v] * r_TPA_j[v]
 * with r_TPA_j from seeds (k seed nodes; packed != 0: seeds[b*k + j] per
 * block as tpa_query_packed) or from dense restart vectors q [k][n] (pass
 * exactly one).  Both CPI chains are differentiated: the family chain per
 * restart vector (x(0) = c q_j, S-1 steps) and the PageRank stranger chain
 * (x'(0) = c/n_g per block, K steps, its iterates checkpointed every
 * `checkpoint_every` steps and recomputed per segment; negative = one
 * segment, every iterate kept; 0 = automatic: every iterate kept when the
 * K+1 vectors take at most a third of the free device memory, else
 * checkpoints every ceil(sqrt(K)) steps).  Outputs (device, either may be
 * NULL):
 *   grad_logits float[m], A~ order: dL/dtheta for row-softmax weights
 *               A~_uv = softmax_u(theta); with 1/outdeg weights it is the
 *               derivative at theta = 0;
 *   grad_q      float[k][n]: dL/dq_j = c * lambda_j(0).
 * Requires tpa_preprocess with the same (c, T) (K comes from its eps).
 * Its work buffers stay on the handle for the next call (up to 8 GiB in
 * all; buffers beyond that are allocated and freed per call), so repeated
 * calls of one shape allocate nothing; they are freed with the graph.
 * Synchronises `stream` before returning; calls on one handle must not
 * overlap.  With tpa_set_keep_iterates on and checkpoint_every = 0 the
 * stranger chain is read from the iterates kept by tpa_preprocess.
 * Errors: INVALID_ARG, NOT_PREPROCESSED, PARAM_MISMATCH, OOM, HIP. */
tpa_status tpa_backward(tpa_graph_t g, const int32_t *seeds, const float *q, int64_t k, int packed,
                        double c, int S, int T, const float *grad_out, float *grad_logits,
                        float *grad_q, int checkpoint_every, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Captured queries (HIP graphs).  tpa_query_graph_create records the whole
 * launch sequence of a query (seeds: as tpa_query / tpa_query_packed when
 * packed != 0; or dense q as tpa_query_dense) into a HIP graph with its own
 * workspace (allocated here, synchronously); tpa_query_graph_launch replays
 * it on `stream`.  The seeds / q / out buffers are fixed at capture; their
 * contents may change between replays.  Re-create after
 * tpa_graph_set_logits, tpa_preprocess with other parameters or
 * tpa_set_tuning.  The graph handle must outlive the capture, and a replay
 * must not overlap other queries on the same handle.  Errors: INVALID_ARG,
 * NOT_PREPROCESSED, PARAM_MISMATCH, OOM, HIP. */
typedef struct tpa_query_graph *tpa_query_graph_t;
tpa_status tpa_query_graph_create(tpa_graph_t g, const int32_t *seeds, const float *q, int64_t k,
                                  int packed, double c, int S, int T, float *out, hipStream_t stream,
                                  tpa_query_graph_t *out_graph);
tpa_status tpa_query_graph_launch(tpa_query_graph_t qg, hipStream_t stream);
tpa_status tpa_query_graph_destroy(tpa_query_graph_t qg);

/* Autotuner: times tpa_query on the caller's k seeds (device) for every
 * candidate seed tile (8..64, and 1 when k <= 4) and group edge budget
 * (128, 256, 512, and 1024 for seed tiles), keeps candidates whose first min(k, 8) outputs agree
 * with the single-vector path within L1 <= 1e-5 per seed, and stores the
 * fastest with tpa_set_tuning.  scratch_out is a float[k][n] device buffer
 * it may overwrite.  Outputs (host, nullable): best seed tile, edge budget,
 * milliseconds per query call.  Synchronous.  Errors: INVALID_ARG,
 * NOT_PREPROCESSED, OOM, HIP. */
tpa_status tpa_autotune(tpa_graph_t g, const int32_t *seeds, int64_t k, double c, int S, int T,
                        float *scratch_out, int *best_tile, int *best_edges_per_item, double *best_ms,
                        hipStream_t stream);

/* Pre-allocate the query workspace for up to k seeds (or per_block slots),
 * so that later queries allocate nothing (e.g. under stream capture). */
tpa_status tpa_reserve(tpa_graph_t g, int64_t k);

/* Bytes of device workspace a query of k columns (seeds, per_block slots or
 * dense restart vectors) needs under the current tuning: the size that
 * tpa_reserve(g, k) holds on the handle and that a captured query allocates
 * for itself.  It may build the work schedule (synchronously).  Errors:
 * INVALID_ARG (NULL, k < 0), HIP. */
tpa_status tpa_query_workspace_size(tpa_graph_t g, int64_t k, size_t *bytes);

/* Query tuning: seed-tile width kt (seeds per SpMM pass: 1, 2, 4, 8, 16,
 * 32 or 64; 0 = automatic: the next power of two up to 16 for k <= 32
 * columns, 64 above) and the edge budget of a wave work item that
 * groups short rows (64..1024, a multiple of 64; 0 = automatic, 512 for
 * both the single vector and seed tiles; the single-vector step caps it at
 * 512).  Longer rows are one wave item up to 2x (seed tiles) or 4x (single
 * vector) the budget, then block items or chunks.  Applies to later calls. */
tpa_status tpa_set_tuning(tpa_graph_t g, int seed_tile, int edges_per_item);
tpa_status tpa_get_tuning(tpa_graph_t g, int *seed_tile, int *edges_per_item);

/* Direction of the second family step of a single-seed query (seed tile 1,
 * unpacked graph, S >= 4).  x(1) lives on the seed's out-neighbours, so
 * x(2) can be pushed over the out-edges of F = out(s) + {s} instead of
 * pulled over all m edges (the same sum; Section 2.3's CPI step).  The
 * choice is made on the device per query: push when the frontier's edge
 * count W = sum of outdeg over F is at most `max_edges` and F has at most
 * 2048 nodes.  max_edges = -1
 * restores the default (m/8, at least 1024), 0 always pulls.  The pushed
 * sums are exact fixed-point additions of FP32 terms, so results are
 * reproducible but may differ from the pulled step in the last bits.
 * The pull that follows a push (step 3 after a pushed step 2 when it is
 * not pushed itself, see tpa_set_third_push_limit; step 2 after the pushed
 * step 1 of a seed tile of 1 or 64) skips the gathers of rows the push
 * left zero, using a bitmap the push fills; the skipped terms are exact
 * zeros, so the sums are unchanged.  max_edges = 0 also turns this skip
 * off.
 * Errors: INVALID_ARG (NULL graph, max_edges < -1). */
tpa_status tpa_set_push_limit(tpa_graph_t g, int64_t max_edges);

/* Direction of the second family step of a seed tile (2..64 one-hot
 * columns, unpacked graph, S >= 4), the tile form of the single seed's
 * pushed step (Section 2.3's CPI step, over the columns' frontiers).
 * Column j's x(1) lives on F_j = out(s_j) + {s_j}; the device plans the
 * tile (one entry per node of every F_j) and pushes step 2 over their
 * out-edges when the plan has at most 16384 entries and the tile's
 * frontier edge count W = sum over j of sum over F_j of outdeg is at most
 * `max_edges`; it pulls otherwise.  The pushed step also replaces the
 * pushed first step (y1 is folded into the plan).  max_edges = -1 restores
 * the default (m/4, at least 2048), 0 always pulls.  The pushed sums are
 * exact fixed-point additions of FP32 terms (reproducible, and within FP32
 * rounding of the pulled step).  The push needs a buffer of 8 bytes per
 * node and column (allocated on the handle at the first such query, or by
 * tpa_reserve; not under stream capture; none above 32 GiB or a quarter of
 * the free device memory, when tiles pull).  Captured query graphs hold
 * their own buffer; tpa_query_noalloc takes it from its fixed array.
 * Errors: INVALID_ARG (NULL graph, max_edges < -1). */
tpa_status tpa_set_tile_push_limit(tpa_graph_t g, int64_t max_edges);
tpa_status tpa_get_tile_push_limit(tpa_graph_t g, int64_t *max_edges);

/* Direction of the third family step of a single-seed query whose second
 * step was pushed (S >= 5, so that step 3 is not the last).  x(2) lives on
 * the rows the push reached; the device lists them (with their out-edges,
 * W3 in all) from the step's bitmap and pushes step 3 over those edges
 * when W3 <= `max_edges` (Section 2.3's CPI step, as for step 2), else it
 * pulls the step with the frontier skip.  max_edges = -1 restores the
 * default: m/20 on graphs of at least 2^28 edges, where a pulled step
 * costs far more than the list, push and conversion launches, and always
 * pull on smaller ones; 0 always pulls; tpa_set_push_limit(g, 0) turns this
 * push off as well.  Pushed sums are exact fixed-point additions
 * of FP32 terms (reproducible, within FP32 rounding of the pull).
 * Errors: INVALID_ARG (NULL graph, max_edges < -1). */
tpa_status tpa_set_third_push_limit(tpa_graph_t g, int64_t max_edges);
tpa_status tpa_get_third_push_limit(tpa_graph_t g, int64_t *max_edges);

/* Keep the stranger chain's iterates (Algorithm 2's x'(0) .. x'(K-1), node
 * order, K x n floats) on the handle at the next tpa_preprocess, so that
 * tpa_backward with checkpoint_every = 0 reads them instead of recomputing
 * the chain (the same values).  They are taken only when they fit in a
 * quarter of the free device memory at preprocessing; tpa_graph_set_logits
 * drops them until the next tpa_preprocess.  keep = 0 (the default) frees
 * them (after a device synchronisation).  Errors: INVALID_ARG (NULL). */
tpa_status tpa_set_keep_iterates(tpa_graph_t g, int keep);

/* Memory order of the vectors a CPI step gathers (internal work buffers).
 * hub_first = 1: node v's
 * entries sit at the rank of v by descending out-degree (ties by id), so
 * the most gathered entries, those of high out-degree sources, share cache
 * lines, and each row of A~^T is summed in ascending rank, so the lanes
 * that read the first edges of neighbouring rows hit the same lines.  The
 * re-sorted column ids and each entry's position in its original row are
 * two more int32[m] arrays (plus int32[n] ranks); graphs with logit
 * weights also keep their weights in that order (float[m], refreshed by
 * tpa_preprocess after tpa_graph_set_logits).  Built by tpa_preprocess, or
 * here when the graph is already preprocessed.  hub_first = 0 keeps node
 * order, A~^T's own edge order and no extra memory.  The two orders give
 * the same sums up to FP32 rounding (each row is added in a different
 * order).  hub_first = 2 (the default) is order 1 plus, for the
 * single-vector step (one seed, preprocessing, tpa_cpi, the adjoint's
 * forward chain), one more int32[m] copy of the column ids in which the
 * edges of each work item that sums several short rows (at most 512 edges)
 * are sorted by rank across the rows, so each 64-edge load reads fewer
 * cache lines; every entry carries its position in the item, where its
 * product is added, so the sums are bitwise those of order 1.  The copy
 * is built with the work schedule (by tpa_preprocess, the first
 * single-seed query or tpa_reserve; not during stream capture, where the
 * kernels read the order-1 ids instead) when the graph has fewer than
 * 2^23 nodes and the copy takes at most a quarter of the free device
 * memory.  tpa_backward's single-vector adjoint step gets one more such
 * copy of A~'s destination ids (sorted by node id within its items, the
 * gradients again bitwise those of order 1), built at its first call.  Leaving layout 2 stops its use but keeps the copy (query
 * graphs captured before may read it) until tpa_graph_destroy; coming
 * back uses it again.  Synchronous when it builds.  Errors: INVALID_ARG
 * (layout not 0, 1 or 2), OOM, HIP. */
tpa_status tpa_set_gather_layout(tpa_graph_t g, int hub_first);
tpa_status tpa_get_gather_layout(tpa_graph_t g, int *hub_first);

/* XCD-sliced sweeps (Section 3.3's preprocessing CPI, Algorithm 2; the same
 * chain recomputed by tpa_backward; the dense family pulls of single-seed
 * queries).  The chip deals the workgroups of a launch to its 8 XCDs in turn
 * and each XCD caches in an L2 of its own, so a cache line gathered by
 * blocks on several XCDs is fetched into each of their L2s.  In the sliced
 * sweep every row of A~^T with more than 32 edges is summed as 8 runs, one
 * per slice of the hub-first gather rows (rows below 8192 by row mod 8, the
 * others by blocks of 1024 rows), and slice x's runs run on XCD x, so that
 * each L2 holds its own eighth of the gathered vector: rows up to a group
 * item's budget (512 edges by default) in band items that hold one slice's
 * runs of up to 63 such rows, longer rows in chunks; finish passes add each
 * row's run sums in slice order and apply the epilogue.  Shorter rows are
 * summed whole.  It needs one more int32[m] copy of the hub-first column
 * ids (rearranged: short rows, then the bands, then the long rows), int64
 * row offsets and the work items, built at the first preprocessing that
 * takes them (synchronous; when the copy takes at most a quarter of the
 * free device memory, and never under stream capture).  Single-seed queries
 * on the handle's own workspace then use it for their dense pulls (not
 * captured query graphs, nor tpa_query_noalloc).  Only graphs with 1/outdeg
 * weights in the hub-first gather layout take it.  The same mode slices the
 * adjoint steps of the stranger chain in tpa_backward (1/outdeg graphs):
 * rows of A~ longer than a group item are summed per slice of the lambda
 * rows they gather (their edges partitioned within the row, in one more
 * int32[m] copy of the gathered ids, dropped and rebuilt when a later
 * adjoint buffer does not fit), and the edge gradient, accumulated in that
 * order over the chain, is put back in A~'s order after it (a float[m]
 * temporary).  mode: 0 off, 1 (the default) from 2^23 nodes, 2 on every
 * such graph.  The results agree with the unsliced sweeps up to FP32
 * rounding (the split rows are added in another order).
 * tpa_get_sliced_sweep reports the mode and, in *active (may be NULL),
 * whether the forward sliced schedule is built and in use for the graph's
 * current work-item shape.  Errors: INVALID_ARG (mode not 0, 1 or 2, NULL
 * handle). */
tpa_status tpa_set_sliced_sweep(tpa_graph_t g, int mode);
tpa_status tpa_get_sliced_sweep(tpa_graph_t g, int *mode, int *active);
tpa_status tpa_get_push_limit(tpa_graph_t g, int64_t *max_edges);

/* Sticky device-side error (synchronises `stream`): TPA_ERR_INVALID_ARG if
 * any query since the last call saw an out-of-range seed, else TPA_OK.
 * Clears the flag. */
tpa_status tpa_get_device_error(tpa_graph_t g, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Exact RWR and the accuracy harness (Section 2.3 Algorithm 1, Theorem 1;
 * Section 4's error and top-k recall measurements).
 *
 * tpa_cpi: Algorithm 1 for one restart vector, r = sum of x(i) over
 * s_iter <= i <= t_iter with x(0) = c q, x(i) = (1-c) A~^T x(i-1), x(0)
 * included when s_iter = 0, stopping after the first i whose ||x(i)||_1 is
 * below eps.  The restart is either a seed (seed >= 0, q NULL: q = e_seed)
 * or a dense vector q (float[n], seed = -1).  t_iter = -1 means no last
 * iteration (only the eps test).  The norm test uses Lemma 2's closed form
 * c (1-c)^i ||q||_1 (exact for q >= 0; an upper bound otherwise, so the
 * loop never stops early), with ||q||_1 = 1 for a seed and reduced on the
 * device for dense q.  s_iter = 0, t_iter = -1 gives exact RWR up to the
 * truncation (Theorem 1); [0, S-1], [S, T-1] and [T, -1] give the exact
 * family, neighbor and stranger parts.  out: float[n], the summed window
 * (Kahan-compensated FP32).  Needs no preprocessing (it builds the gather
 * layout of tpa_set_gather_layout if that is on and not built yet).
 * Synchronous (it allocates and frees its work vectors).  Errors: INVALID_ARG (not exactly
 * one of seed >= 0 and q, seed >= n, c outside (0,1), s_iter < 0,
 * t_iter < -1, t_iter < s_iter, eps < 0, eps = 0 with t_iter = -1), OOM,
 * HIP. */
tpa_status tpa_cpi(tpa_graph_t g, int32_t seed, const float *q, double c, int s_iter, int t_iter, double eps,
                   float *out, hipStream_t stream);

/* tpa_cpi for k restarts at once, on seed tiles of the automatic width
 * (the batched form of the same CPI steps): seeds int32[k] (device, q NULL)
 * or dense restart vectors q float[k][n] (device, seed-major, seeds NULL).
 * Row j of out float[k][n] is restart j's window sum over s_iter <= i <=
 * t_iter, each restart with its own last iteration (min of t_iter and the
 * first i with c (1-c)^i ||q_j||_1 < eps).  A seed outside [0, n) gives an
 * all-NaN row and sets the sticky error of tpa_get_device_error.
 * Synchronous (it allocates and frees its work tiles: five [n][kt] float
 * tiles with dense q, four with seeds).  k = 0 does nothing.  Errors:
 * INVALID_ARG (k < 0; for k > 0, not exactly one of seeds and q, or out
 * NULL; the tpa_cpi parameter checks), OOM, HIP. */
tpa_status tpa_cpi_batch(tpa_graph_t g, const int32_t *seeds, const float *q, int64_t k, double c, int s_iter,
                         int t_iter, double eps, float *out, hipStream_t stream);

/* The k largest entries of each row of vals (row-major [rows][n]), ordered
 * by value descending and, among equal values, index ascending; NaN ranks
 * below every number.  idx_out int32[rows][k], val_out float[rows][k].
 * 1 <= k <= min(n, 1024).  Rows are cut into segments of max(4096, 16k)
 * entries, each keeping its k best, until one segment is left; when that
 * takes more than one pass the candidate lists live in a device buffer
 * allocated and freed here, and the call synchronises the stream.  Errors:
 * INVALID_ARG (sizes, NULL), INDEX_OVERFLOW (n or rows above 2^31 - 1, or
 * rows times segments above 2^31 - 1), OOM, CAPTURE (a buffer would be
 * allocated during stream capture), HIP. */
tpa_status tpa_topk(const float *vals, int64_t rows, int64_t n, int k, int32_t *idx_out, float *val_out,
                    hipStream_t stream);

/* Per-row L1 distance out[r] = sum_v |a x[r][v] - y[r][v]| (row-major
 * [rows][n] FP32 inputs, double[rows] output), summed in FP64 in a fixed
 * order (deterministic).  Synchronous (it frees a scratch buffer).
 * Errors: INVALID_ARG (negative sizes, NULL), INDEX_OVERFLOW (more than
 * 65535 rows), OOM, HIP. */
tpa_status tpa_row_l1(const float *x, const float *y, int64_t rows, int64_t n, double a, double *out,
                      hipStream_t stream);

/* ------------------------------------------------------------------------
 * Kernel timing (a tracing aid, process-wide).  While enabled, HIP events
 * bracket one in every `sample_period` launches of each CPI step-kernel
 * variant, on the launch's stream; variants are numbered
 *   code = 16*log2(kt) + 4*mode + 2*first + weighted
 * (mode 0 = online family step, 1 = preprocessing stranger step, 2 =
 * plain step keeping its iterate, 3 = adjoint step; first = the gather-free
 * first step from one-hot seeds, or for mode 3 = with the edge gradient;
 * weighted = explicit edge weights), except the last family step of a
 * single seed and of seed tiles of 16 and 64, which is 112 + 2*t +
 * weighted (t = 0, 1, 2 for kt = 1, 16, 64), and a pull launched under a
 * device-side gate (a step the device may have pushed instead; its launch
 * then does nothing), which is 118 + weighted; codes 120 and 121 are the
 * gated launch of a single seed's second family step, which converts the
 * pushed sums or pulls (uniform, explicit weights), 122 a seed tile's push
 * plan, 123 its push, 124 the launch that pushes a single seed's first two
 * steps, 125 a pushed tile's conversion, 126 the frontier list and push of
 * a single seed's third step, and 127 the long-row finish pass.
 * tpa_profile_read synchronises the
 * recorded events, adds their durations into per-code totals and returns
 * them (launches timed, milliseconds).  tpa_profile_reset clears the
 * totals.  Errors: INVALID_ARG (capacity outside 1..2^20, sample_period
 * < 1, code outside 0..127), OOM, HIP. */
tpa_status tpa_profile_enable(int enable, int capacity, int sample_period);
tpa_status tpa_profile_read(int code, int64_t *launches, double *total_ms);
tpa_status tpa_profile_reset(void);

const char *tpa_status_string(tpa_status s);
const char *tpa_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* TPA_H */
