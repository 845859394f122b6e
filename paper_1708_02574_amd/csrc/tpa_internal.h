// Internal declarations shared by the HIP sources of libtpa.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "tpa.h"

namespace tpa {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);

#define TPA_TRY_HIP(expr)                                                        \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess) {                                                  \
            ::tpa::set_error(std::string(#expr) + ": " + hipGetErrorString(e_)); \
            return e_ == hipErrorOutOfMemory ? TPA_ERR_OUT_OF_MEMORY : TPA_ERR_HIP; \
        }                                                                        \
    } while (0)

#define TPA_TRY(expr)                    \
    do {                                 \
        tpa_status s_ = (expr);          \
        if (s_ != TPA_OK) return s_;     \
    } while (0)

tpa_status fail(tpa_status s, const std::string &msg);

// Device allocation that reports OOM as a status (refuses during capture).
tpa_status dmalloc(void **p, size_t bytes, hipStream_t stream);
template <class T>
tpa_status dalloc(T **p, size_t count, hipStream_t stream) {
    return dmalloc(reinterpret_cast<void **>(p), count * sizeof(T), stream);
}
void dfree(void *p);

// ---------------------------------------------------------------- schedule
// A wave work item over the rows of A~^T.
//   kind 0 (group) : rows [row0, row0+nrows), nrows <= 63, with nnz <= EW
//                    edges starting at e0
//   kind 1 (row)   : the single row row0, nnz edges starting at e0
//   kind 2 (chunk) : a chunk [e0, e0+nnz) of a long row; its sum goes to
//                    partial slot <item index>; a finish pass adds each long
//                    row's partials in chunk order
//   kind 3 (block) : the single row row0 shared by the 4 waves of a block
//                    (the item is repeated in the block's 4 slots); the
//                    waves' quarter sums are added in LDS in wave order
struct Item {
    int64_t e0;
    int32_t row0;
    uint32_t meta;  // nrows [0,7) | nnz [7,24) | kind [24,26)
};
constexpr uint32_t kItemGroup = 0, kItemRow = 1, kItemChunk = 2, kItemBlock = 3;
__host__ __device__ inline uint32_t item_meta(uint32_t nrows, uint32_t nnz, uint32_t kind) {
    return nrows | (nnz << 7) | (kind << 24);
}
__host__ __device__ inline uint32_t item_nrows(uint32_t m) { return m & 127u; }
__host__ __device__ inline uint32_t item_nnz(uint32_t m) { return (m >> 7) & 0x1ffffu; }
__host__ __device__ inline uint32_t item_kind(uint32_t m) { return (m >> 24) & 3u; }

struct LongRow {
    int32_t row, nchunks, first_item, pad;
};

// Group items in gather order: the single-vector step keeps a group item's
// products in a kGroupEdges-float LDS slice.  In a schedule's colg copy of
// the hub-first column ids, each group item's edges are re-sorted by gather
// row (ties by position) and each entry carries, above its kGroupSlotShift
// row bits, its position in the item: the LDS slot its product goes to, so
// the rows are still summed in the same order.  Graphs of at least
// kGroupSlotMaxN nodes do not fit and keep the row order.
constexpr int kGroupEdges = 512;
constexpr int kGroupSlotShift = 23;
constexpr int64_t kGroupSlotMaxN = int64_t(1) << kGroupSlotShift;
constexpr uint32_t kGroupRowMask = (1u << kGroupSlotShift) - 1u;

// Shape of a schedule: group items hold <= ew edges; rows of ew+1..el edges
// are one wave item each; rows of el+1..eb edges are block items; longer
// rows are cut into chunks of `chunk` edges.
struct SchedShape {
    int ew, el, chunk, eb;
    bool operator<(const SchedShape &o) const {
        if (ew != o.ew) return ew < o.ew;
        if (el != o.el) return el < o.el;
        if (chunk != o.chunk) return chunk < o.chunk;
        return eb < o.eb;
    }
};

struct Schedule {
    int ew = 0;                  // edge budget of a group item
    int ds = 0;                  // group rows with <= ds edges are summed per lane
    int el = 0;                  // rows with > el edges are chunked
    int chunk = 0;               // chunk length
    int eb = 0;                  // rows of el+1..eb edges are block items
    Item *items = nullptr;       // device; chunk items first
    int64_t n_items = 0;
    int64_t n_chunk_items = 0;
    LongRow *longs = nullptr;    // device
    int64_t n_long = 0;
    // device, m: colg_src (the graph's t_colz, or a.col for a schedule over
    // A~) with group items in gather order (see kGroupEdges), built by
    // ensure_group_order; null when absent.
    // The step launchers use colg only while colg_src is set (layout 2).
    int32_t *colg = nullptr;
    const int32_t *colg_src = nullptr;
    const int32_t *colg_from = nullptr;  // the ids colg was built from (reused only for those)
    // XCD-sliced schedules: chunk items carry their partial slot in row0,
    // and n_chunk_items counts the slots; band items and the short-row
    // offsets (see gather_slice); rows of longs8 have 8 consecutive slots
    bool chunk_slot_in_item = false;
    int64_t *rowptr_x = nullptr;  // device, n+1
    int32_t *xrel = nullptr;      // device
    LongRow *longs8 = nullptr;    // device
    int64_t n_long8 = 0;
    void release();
};

// XCD-sliced single-vector sweep.  The workgroups of a launch are dealt to
// the chip's 8 XCDs round-robin (block b runs on XCD b % 8), and each XCD
// has an L2 of its own, so gathers of one cache line from blocks on
// different XCDs fetch it into every L2.  Rows of A~^T longer than a group
// item are cut into one run per source slice (their edges stably
// partitioned by the slice of the gather row, rank order kept within a
// slice), and slice x's chunks are placed in blocks that run on XCD x: each
// XCD's L2 then holds the lines of its own eighth of the gathered vector.
// The hub rows (below 8192, gathered everywhere and cached by every XCD)
// alternate by row so that the slices carry equal work; the others go by
// blocks of 1024 rows.  Used from kSliceMinN nodes (1/outdeg graphs in the
// hub-first layout): below that the whole vector stays in the caches.
//
// Rows of up to kSliceShortRow edges are not split.  Medium rows (up to a
// group item) are split into 8 runs as well: a band item holds slice x's
// runs of up to 63 consecutive medium rows, laid out one after the other in
// the sliced ids, so each band reads like a group item.  The sliced ids hold
// the short rows first (row order), then the bands (slice-major per band),
// then the long rows (slice-major per row).  rowptr_x gives each row's
// offset in the short section with bit kRowxForeignBit set on medium and
// long rows (no edges there; their epilogue is the finish pass's), and a
// band item's row0 indexes xrel: [first partial slot, run offsets 0..R].
// Medium row k (in row order, M of them) keeps slice x's sum in slot
// x * M + k; the long rows' chunk slots follow from 8 M.
constexpr int kSliceCount = 8;
constexpr int64_t kSliceMinN = int64_t(1) << 23;
constexpr int kSliceShortRow = 32;
constexpr uint32_t kItemBandBit = 1u << 26;
constexpr int kRowxForeignBit = 62;
constexpr int64_t kRowxMask = (int64_t(1) << kRowxForeignBit) - 1;
__host__ __device__ inline int gather_slice(int32_t r) { return r < 8192 ? (r & 7) : ((r >> 10) & 7); }

// XCD-sliced adjoint sweep over the rows of A~ (the stranger chain's
// single-vector step with the edge gradient, 1/outdeg graphs): rows longer
// than a group item have their edges stably partitioned in place, within
// the row, by the slice of the lambda row they gather, and each slice run
// is summed in chunk items on its XCD; the other rows keep A~'s order in
// group items.  The edge gradient accumulates in that order over the chain
// and is put back in A~'s order after it (the segments of the partition are
// kept for that).
struct SlicedAdj {
    Schedule s;                     // chunk items carry their partial slot in row0
    int32_t *col = nullptr;         // device, m: the gathered ids, long rows partitioned
    const int32_t *from = nullptr;  // the ids it was built from
    int32_t *slot_row = nullptr;    // device: the row of each partial slot
    int64_t *seg_e0 = nullptr;      // device: counting segments of the long rows
    int32_t *seg_len = nullptr;
    int64_t *seg_out = nullptr;     // device, [nseg][8]: where each slice's edges of a segment go
    int64_t nseg = 0;
    int ew = 0;
    bool none = false;              // built for ew and from: no long rows
    void release();
};

struct Csr {
    int64_t *rowptr = nullptr;  // n+1
    int32_t *col = nullptr;     // m
    float *w = nullptr;         // m, only when weights are not 1/outdeg
};

}  // namespace tpa

namespace tpa {
// Smallest graph whose adjoint keeps lambda in in-degree rank order.  Below
// it lambda (at most 32 MB) stays in the caches in node order and the row
// lookup of every store costs more than it saves (adjoint of 64 seeds on
// R-MAT graphs: +2 % at 2^20 and 2^22 nodes; -14 % at 2^24, -43 % per step
// at 2^27).
constexpr int64_t kLamRankMinN = int64_t(1) << 23;

// Device buffer of a seed tile's pushed second step (laid out for up to
// kt_cap columns by tile_push_at; zeroed when allocated).
struct TileBuf {
    void *base = nullptr;
    size_t bytes = 0;
    int kt_cap = 0;
};
}  // namespace tpa

struct tpa_graph {
    int device = 0;
    int64_t n = 0, m = 0;
    int64_t max_outdeg = 0;                 // largest row of A~
    int bits = 1;                           // bits of a node id (key packing)
    int64_t nblocks = 1;
    std::vector<int64_t> block_off;         // host, nblocks+1
    int32_t *node_block = nullptr;          // device, n (only when nblocks > 1)
    float *restart_pr = nullptr;            // device, n: 1/n_block(v) (packed only)

    tpa::Csr a;                             // A~   (rows = sources)
    tpa::Csr t;                             // A~^T (rows = destinations)
    int64_t *t2a = nullptr;                 // A~^T entry -> A~ entry (lazy)
    // gather layout of the CPI work vectors: node v's entries sit at row
    // zperm[v] (rank of v by descending out-degree, ties by id); t_colz holds
    // zperm[t.col] with each row of A~^T re-sorted in ascending rank, t_locz
    // each entry's position in its original row, and t_wz the per-edge
    // weights in that order (logit weights; rebuilt at preprocessing)
    int32_t *zperm = nullptr;               // n
    int32_t *zinv = nullptr;                // n: node at each gather row (zperm's inverse)
    int32_t *t_colz = nullptr;              // m
    int32_t *t_locz = nullptr;              // m
    float *t_wz = nullptr;                  // m, weighted graphs
    bool t_wz_valid = false;
    int gather_layout = 2;                  // 2 = hub-first order, group items in gather
                                            // order; 1 = hub-first order; 0 = node order
    // adjoint gather layout (layout 2, n >= kLamRankMinN, unpacked): the adjoint's
    // lambda vectors keep node v's entry at row lrank[v], the rank of v by
    // descending in-degree (ties by id), so the entries a pull over A~
    // gathers most share cache lines; a_colr holds lrank[a.col] in A~'s own
    // edge order (the sums and the edge gradient keep their order).  Built
    // at the first tpa_backward.
    int32_t *lrank = nullptr;               // n
    int32_t *a_colr = nullptr;              // m
    // XCD-sliced sweep of the stranger chain (preprocessing and the
    // adjoint's recomputation): t_colx is t_colz with the edges of each row
    // longer than a group item partitioned by source slice, sched_x its
    // schedule (built for group edge budget sched_x_ew; sched_x_none: that
    // budget leaves no such rows)
    int sliced_sweep = 1;                   // 0 off, 1 from kSliceMinN nodes, 2 always
    int32_t *t_colx = nullptr;              // m
    tpa::Schedule sched_x;
    int sched_x_ew = 0;
    bool sched_x_none = false;
    tpa::SlicedAdj sax;                     // the adjoint's (same mode)
    float *inv_deg = nullptr;               // 1/outdeg(u), FP32
    uint8_t *padded = nullptr;
    bool weighted = false;                  // weights from logits (a.w, t.w set)

    // preprocessing state
    bool preprocessed = false;
    // changes whenever the weights or the preprocessed state change
    // (tpa_graph_set_logits, tpa_preprocess)
    uint64_t version = 1;
    // stranger-chain iterates x'(0..K-1), node order, [K][n], kept by
    // tpa_preprocess when keep_iterates is on (for tpa_backward)
    bool keep_iterates = false;
    float *xiter = nullptr;
    int64_t xiter_K = 0;  // iterates held (0: none)
    size_t xiter_cap = 0;  // floats allocated at xiter
    // tpa_backward's work buffers, kept for the next call (slot i = the
    // call's i-th buffer; at most kAdjCacheBytes in all)
    std::vector<std::pair<void *, size_t>> adj_cache;
    double c = 0.0, eps = 0.0;
    int T = 0;
    int64_t K = 0;
    float *str = nullptr;                   // r~_stranger, n

    // schedules over the rows of A~^T (forward) and of A~ (adjoint), by shape
    std::map<tpa::SchedShape, tpa::Schedule> sched_t;
    std::map<tpa::SchedShape, tpa::Schedule> sched_a;

    // query workspace
    float *ws = nullptr;
    size_t ws_bytes = 0;
    // pushed-tile state of eager queries (the fixed-point y2 tile and the
    // plan), laid out for kt_cap columns; all-zero accumulator between queries
    tpa::TileBuf tbuf;
    int32_t *dev_err = nullptr;             // sticky device error flag

    // tuning
    int seed_tile = 0;                      // 0 = automatic
    int edges_per_item = 0;                 // 0 = automatic
    int64_t push_limit = -1;                // -1 = automatic, 0 = never push
    int64_t tile_push_limit = -1;           // seed tiles: -1 = automatic, 0 = never push
    int64_t third_push_limit = -1;          // step 3 of a single seed: -1 = automatic, 0 = never push
};

namespace tpa {

int64_t stranger_last_iteration(double c, double eps);
double family_alpha(double c, int S, int T);
int choose_kt(const tpa_graph *g, int64_t k);
SchedShape choose_shape(const tpa_graph *g, int kt);
// Query driver; ws == nullptr uses (and grows) the handle's workspace.
// no_alloc: allocate nothing (the work schedule must exist already and the
// group-ordered ids are used only if built; ws must be given).
// tb: the pushed-tile buffer to use (null: the handle's own, allocated on
// demand outside capture; under no_alloc, none); seed tiles push step 2
// only with a buffer of at least kt columns.
tpa_status run_query(tpa_graph *g, const int32_t *seeds, const float *q, int64_t k, bool packed, double c,
                     int S, int T, float *out, hipStream_t st, float *ws, size_t ws_bytes, bool no_alloc = false,
                     TileBuf *tb = nullptr);
// Whether a query of kt columns from seed lists may push its tile's step 2,
// and the bytes of its buffer (0 when it may not: tile width 1, a packed
// graph, S < 4, pushes off, or a buffer above the size limit).
size_t tile_buf_bytes(const tpa_graph *g, int kt, bool packed, int S);
bool tile_push_applies(const tpa_graph *g, int kt, bool packed, int S);
// Allocate and zero a pushed-tile buffer of `bytes` for kt columns.
tpa_status tile_buf_alloc(TileBuf *tb, size_t bytes, int kt, hipStream_t st);
void tile_buf_free(TileBuf *tb);
size_t query_workspace_bytes(tpa_graph *g, int64_t k, bool dense, hipStream_t st);
// Zero the push state at the front of a fresh query workspace.
tpa_status clear_push_state(const tpa_graph *g, void *ws, hipStream_t st);
tpa_status build_from_keys(tpa_graph *g, uint64_t *keys, int64_t nkeys, hipStream_t stream);
// Work schedule over the rows of A~^T (over_a = false) or of A~ (true).
tpa_status get_schedule(tpa_graph *g, SchedShape shape, hipStream_t stream, const Schedule **out,
                        bool over_a = false);
// The cached schedule of that shape, or null (never builds one).
const Schedule *find_schedule(const tpa_graph *g, SchedShape shape, bool over_a = false);
tpa_status ensure_t2a(tpa_graph *g, hipStream_t stream);
// Build zperm, t_colz and t_locz (synchronises `stream`); no-op when present.
tpa_status ensure_zlayout(tpa_graph *g, hipStream_t stream);
// Give a single-vector schedule its group-ordered column ids (colg) when
// the graph's layout asks for them and they fit; a no-op otherwise, also
// under stream capture (the step kernels then read the row-ordered ids,
// with the same sums).  over_a: a schedule over the rows of A~ (the
// adjoint), whose ids are A~'s destinations; else over A~^T, from t_colz.
// Synchronous when it builds.
tpa_status ensure_group_order(tpa_graph *g, const Schedule *s, hipStream_t stream, bool over_a = false);
// Stop using every schedule's colg (after the layout leaves group order);
// the arrays stay allocated until the handle is destroyed.
void drop_group_order(tpa_graph *g);
// Build t_wz from the current weights when the graph is weighted.
tpa_status ensure_wz(tpa_graph *g, hipStream_t stream);
// Build lrank and a_colr (synchronises `stream`); a no-op when present.
tpa_status ensure_lam_layout(tpa_graph *g, hipStream_t stream);
// The XCD-sliced schedule and column ids of the single-vector sweep over
// A~^T when the graph takes one (else *s = nullptr, *col = nullptr); built
// on first use (synchronous), never under stream capture.
tpa_status ensure_sliced_sweep(tpa_graph *g, hipStream_t stream, const Schedule **s, const int32_t **col);
// The same when already built for the current shape, else null (never builds).
const Schedule *find_sliced_sweep(const tpa_graph *g, const int32_t **col);
// The XCD-sliced adjoint sweep for gathered ids `src` (A~'s destinations in
// lambda's row order) when the graph takes one, else *out = nullptr; built
// on first use (synchronous), never under stream capture.
tpa_status ensure_sliced_adj(tpa_graph *g, const int32_t *src, hipStream_t stream, const SlicedAdj **out);
// Edge gradient of the long rows from the sliced order (gx) back to A~'s (G).
tpa_status launch_unslice(const SlicedAdj &sa, const float *gx, float *G, hipStream_t stream);
tpa_status graph_alloc_common(tpa_graph *g, hipStream_t stream);
void graph_release(tpa_graph *g);
int key_bits(int64_t n);

}  // namespace tpa
