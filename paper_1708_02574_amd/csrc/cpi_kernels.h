// Launch interface of the CPI step kernels (cpi_kernels.hip).
#pragma once

#include "tpa_internal.h"

namespace tpa {

enum StepMode : int { kFamily = 0, kStranger = 1, kPlain = 2 };

// One CPI step y = (1-c) A~^T x over a seed tile of kt columns (node-major
// [n][kt] vectors), pulled over the rows of A~^T, plus the step's epilogue:
//   family   (Horner form): y = c*[v == seed] + (1-c)*sum; the next gathered
//            vector is y * (1/outdeg) (uniform weights) or y (explicit
//            weights); on the last step out = alpha*y + r~_stranger instead.
//   stranger : x = (1-c)*sum; next gathered vector as above; when
//            `accumulate` is set r~_stranger += x (Kahan-compensated).
//   plain    : x = (1-c)*sum, stored in xs_out when set (the iterates the
//            adjoint needs), next gathered vector as above.
// The family restart c*q is c*[v == seed] for seed lists, or c*Q[j][v] for
// dense restart vectors (seed-major Q, qdense set).
struct StepParams {
    const int64_t *rowptr = nullptr;
    const int32_t *col = nullptr;
    const float *w = nullptr;          // per-edge weights in A~^T order, or null
    const float *inv = nullptr;        // 1/outdeg (uniform weights)
    const float *zin = nullptr;        // gathered vector [n][kt]
    float *zout = nullptr;             // next gathered vector [n][kt]
    const int32_t *zperm = nullptr;    // row of node v in zin/zout (null: v); col is
                                       // then given in those rows, except on first steps
    int col_slots = 0;                 // kt == 1: col is a schedule's colg (group items in
                                       // gather order with LDS slots); set by the launchers
    float *partials = nullptr;         // [chunk items][kt] chunk sums of long rows
    int chunk_slot_in_item = 0;        // kt == 1: a chunk item's partial slot is its row0
                                       // (XCD-sliced schedules); set by the launchers
    const int64_t *rowptr_x = nullptr; // XCD-sliced schedules: short-row offsets and band
    const int32_t *xrel = nullptr;     // tables (set by the launchers)
    float omc = 0.f;                   // 1 - c
    float c = 0.f;
    int kt = 1;
    // family
    const int32_t *seeds = nullptr;    // tile seeds (caller memory; validated on the last step)
    const int32_t *node_block = nullptr;
    int seed_stride = 0;               // seeds per block (packed graphs)
    int ncols = 0;                     // active columns of this tile
    int last = 0;
    float alpha = 0.f;
    const float *str = nullptr;
    float *out = nullptr;              // seed-major [*, n]
    int64_t n = 0;
    int64_t out_col0 = 0;
    int32_t *err = nullptr;            // sticky error flag (invalid seed)
    const float *qdense = nullptr;     // dense restart vectors, seed-major [*, n] (tile offset applied)
    const float *qT = nullptr;         // the tile's c*q node-major [n][kt] (zero past ncols), when
                                       // qdense is set on a family query
    float *xs_out = nullptr;           // plain mode: iterate store [n][kt]
    // plain mode, batched window sums: column j adds x(iter) into tacc
    // (Kahan, compensation tcomp; both node-major [n][kt]) when
    // s_iter <= iter <= klast[j]
    float *tacc = nullptr;
    float *tcomp = nullptr;
    const int32_t *klast = nullptr;
    int iter = 0;
    int s_iter = 0;
    // stranger
    float *acc = nullptr;
    float *comp = nullptr;
    int accumulate = 0;
    // frontier skip (pull steps after a push): bit r of `bits` clear means
    // row r of zin is all zero, so its gathers are skipped (their terms are
    // exact zeros, so the sums are unchanged); applies when bits is set and
    // bits_on is null or *bits_on != 0
    const uint32_t *bits = nullptr;
    const int32_t *bits_on = nullptr;
    // set: the launch does nothing when *skip_on != 0 (the pulled step 2 and
    // the pushed step 1 of a seed tile whose step 2 the device pushed)
    const int32_t *skip_on = nullptr;
};

// Device state of the pushed first two family steps of a single seed
// (kt == 1).  acc holds y2 in gathered form (scaled by 1/outdeg for uniform
// weights), indexed by gather row, as fixed point (2^62 units); it is all
// zero between queries.  ctrl = {W, |F|} and flag record the push decision
// of the query's step 2 (the plan itself lives in each block's LDS).
struct PushPlan {
    unsigned long long *acc = nullptr;  // [n] by gather row, zero between queries
    uint32_t *bits = nullptr;           // [ceil(n/32)]: rows of the pushed vector that may be non-zero
    int64_t nwords = 0;
    int64_t *ctrl = nullptr;            // {W, |F|, W3, pieces3}
    int32_t *flag = nullptr;            // 1: step 2 is pushed (the gated step converts acc)
    int64_t wmax = 0;                   // push only when W <= wmax
    // The third step after a pushed second one: the rows of y2's support
    // (bits) become a list of pieces of at most kTilePiece out-edges of A~
    // (node << 32 | offset of the first edge), W3 = their out-edges in all.
    // Step 3 is pushed into acc (cleared by the step-2 conversion) when W3 <=
    // wmax3 and the pieces fit (flag3 = 1), and pulled otherwise.
    int64_t *pieces3 = nullptr;         // [qmax3]
    int64_t qmax3 = 0;
    int64_t wmax3 = 0;                  // 0: step 3 is always pulled
    int32_t *flag3 = nullptr;
    // 1: step 3 was pushed and y3's support is small (W3 <= n/16, and each
    // row of the support takes at least one of those edges), so step 4
    // skips the gathers of the rows the bitmap marks zero; with a larger
    // support the per-edge bitmap reads cost more than the gathers saved
    int32_t *flag4 = nullptr;
};

// Bytes of the push state (kept at the front of the query workspace; the
// third step's pieces only when that step may be pushed), and of its leading
// part that must be zero before the first query (acc, ctrl, flags, bits; the
// pieces need no clearing).
size_t push_plan_bytes(int64_t n, int64_t m, bool third);
size_t push_plan_clear_bytes(int64_t n);
// wmax3 > 0 requires the pieces (push_plan_bytes with third).
PushPlan push_plan_at(void *base, int64_t n, int64_t m, int64_t wmax, int64_t wmax3);

// Device state of the pushed first two family steps of a seed tile (kt >= 2,
// one-hot seeds, unpacked graph).  Column j's x(1) lives on F_j = out(s_j)
// + {s_j}; one block plans the push on the device: an entry per node of
// every F_j (its y1 in gathered form, its A~ edges) and the entries' edges
// cut into pieces of kTilePiece.  When the plan fits (at most kTilePlanMax
// entries, at most qmax pieces) and the tile's frontier edges W = sum over
// j of sum over F_j of outdeg number at most wmax, the flag is set and the
// pieces are pushed into acc.  acc holds y2 in gathered form, by gather row,
// [n][kt] in 2^62 fixed point, all zero between queries; mark[r] is set (a
// plain byte store, no atomic) for every row r the push reached.
constexpr int kTilePlanMax = 16384;
constexpr int kTilePiece = 256;
struct TilePush {
    unsigned long long *acc = nullptr;  // [n][kt] by gather row
    uint8_t *mark = nullptr;            // [n] by gather row, cleared by the plan launch
    int64_t *ent_e0 = nullptr;          // [kTilePlanMax] first A~ edge of the entry's node
    int64_t *ent_e1 = nullptr;          // end of its edges
    float *ent_y = nullptr;             // its y1 value, gathered form
    int32_t *ent_col = nullptr;         // its column j
    int64_t *pieces = nullptr;          // [qmax] entry << 32 | offset of the piece's first edge
    int64_t *ctrl = nullptr;            // {W, pieces pushed (0 when pulled), entries}
    int32_t *flag = nullptr;            // 1: step 2 of the tile is pushed
    int64_t qmax = 0;
    int64_t wmax = 0;
};

// Bytes of the tile push state for kt columns, and its layout from base
// (256-byte aligned).
size_t tile_push_bytes(int64_t n, int64_t m, int kt);
TilePush tile_push_at(void *base, int64_t n, int64_t m, int kt, int64_t wmax);

// Step 3 of a single seed after a pushed step 2 (p.zin = y2 gathered, p.zout
// = y3 gathered): the frontier list and the push (nothing unless step 2 was
// pushed and the frontier is small enough), then the conversion of every
// row from acc, or (launched with p.skip_on = pp.flag3 by the caller) the
// frontier-skipped pull.
tpa_status launch_push_third(const StepParams &p, const tpa_graph *g, const PushPlan &pp, hipStream_t st);
tpa_status launch_convert_third(const StepParams &p, const PushPlan &pp, hipStream_t st);

// Steps 1 and 2 of a seed tile, pushed when the device's plan allows:
// clears mark, plans (flag, ctrl, the restart terms c e_s of y2 in acc) and
// pushes the plan's pieces (nothing when the flag is clear).  The caller
// launches the pushed first step (launch_push_first) between the plan and
// the push with p.skip_on = tp.flag, so it runs only when step 2 is pulled.
tpa_status launch_tile_plan(const StepParams &p, const tpa_graph *g, const TilePush &tp, hipStream_t st);
tpa_status launch_tile_push(const StepParams &p, const tpa_graph *g, const TilePush &tp, hipStream_t st);

// Step 2 of a pushed tile: p.zout = y2 as the next gathered vector, every
// row written (the rows the push reached from acc, which is cleared, the
// others zero).  Nothing when the flag is clear; the pulled step 2 is then
// launched with p.skip_on = tp.flag.
tpa_status launch_tile_convert(const StepParams &p, const TilePush &tp, hipStream_t st);

tpa_status launch_step(const Schedule &s, int mode, bool first, const StepParams &p, hipStream_t st);

// x'(0) for the stranger chain: zout = c*r0*(1/outdeg or 1), acc = c*r0 if
// T == 0 else 0, comp = 0, where r0 = 1/n or 1/n_block(v); zout rows follow
// zperm when set.
tpa_status launch_stranger_init(const tpa_graph *g, float c, int include_x0, float *zout, float *acc,
                                float *comp, const int32_t *zperm, hipStream_t st);

// z0 = c*Q^T tile (node-major, scaled by 1/outdeg for uniform weights) and,
// when x0 is set, the unscaled x(0) = c*Q tile; columns >= ncols are zero.
// Reads p.qT when set, else the seed-major p.qdense.
tpa_status launch_dense_init(const StepParams &p, float *z0, float *x0, hipStream_t st);

// qT = c*Q^T for the tile's dense restarts (node-major [n][kt], columns >=
// ncols zero), through an LDS-tiled transpose: every step's epilogue then
// reads its restart term with the row's other columns.
tpa_status launch_dense_transpose(const StepParams &p, float *qT, hipStream_t st);

// x(0) = c*e_seed tile for seed lists (node-major), columns >= ncols zero.
tpa_status launch_onehot_init(const StepParams &p, float *x0, hipStream_t st);

// z[0..n) = 0 with a fill kernel (capturable, unlike a memset node).
tpa_status launch_fill_zero(float *z, int64_t n, hipStream_t st);

// out[(col0 + j) * n + v] = tile[v * kt + j] for j < ncols (seed-major rows
// from a node-major tile).  With seeds, a column whose seed lies outside
// [0, n) becomes NaN and raises the sticky error flag *err.
tpa_status launch_tile_to_rows(const float *tile, int kt, int ncols, int64_t n, const int32_t *seeds, float *out,
                               int64_t col0, int32_t *err, hipStream_t st);

// First family step from seeds (any tile width) pushed over each seed's
// out-edges of A~: zout = y1 scaled as the gathered vector (one wave per
// (block, column) seed).  Without bits every other entry of zout is zeroed
// by a fill.  With bits, it is cleared, receives the rows of zout that may
// be non-zero, and only those rows are zeroed and written: the others are
// left as they were, for a pull that skips them.
tpa_status launch_push_first(const StepParams &p, const tpa_graph *g, int64_t nblocks, uint32_t *bits,
                             int64_t nwords, hipStream_t st);

// Single seed (kt == 1, unpacked): the first two family steps in one
// launch.  x(1) is kept on F = out(s) + {s}; when F fits the plan (at most
// 2048 nodes) and its out-edges number W <= wmax, step 2 is pushed over
// them into acc (fixed point, order-independent, so bitwise reproducible,
// with the restart term c e_s) and the flag is set; otherwise y1 is written
// densely to p.zout (p holds the first step's parameters) for the pulled
// step 2 and the flag is cleared.
tpa_status launch_push_steps12(const StepParams &p, const tpa_graph *g, const PushPlan &pp, hipStream_t st);

// The second family step proper (p.zin = dense y1, p.zout = y2 as the next
// gathered vector): with the flag set every row is converted from acc (and
// acc cleared) and bits receives the rows of y2 that are non-zero; with it
// clear the step is pulled over A~^T as usual.
tpa_status launch_gated_step(const Schedule &s, const StepParams &p, const PushPlan &pp, hipStream_t st);

// S == 1: out = alpha*c*[v == seed] + r~_stranger (no CPI step).
// A seed outside [0, n) (or outside its block on a packed graph) gives a
// NaN output column and raises the sticky error flag, here and on the last
// CPI step.
tpa_status launch_combine_only(const StepParams &p, hipStream_t st);


}  // namespace tpa
