// C ABI of the TPA hot path: preprocessing (Algorithm 2) and the online
// phase (Algorithm 3), driving the CPI step kernels.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "cpi_kernels.h"
#include "tpa_internal.h"

namespace tpa {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

tpa_status fail(tpa_status s, const std::string &msg) {
    set_error(msg);
    return s;
}

tpa_status dmalloc(void **p, size_t bytes, hipStream_t stream) {
    *p = nullptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(TPA_ERR_CAPTURE, "device allocation requested while the stream is capturing");
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? TPA_ERR_OUT_OF_MEMORY : TPA_ERR_HIP,
                    std::string("hipMalloc(") + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    return TPA_OK;
}

void dfree(void *p) {
    if (p) (void)hipFree(p);
}

namespace {

constexpr int kDefaultEW1 = 512;   // group edge budget, single vector
constexpr int kDefaultEW64 = 512;  // group edge budget, seed tiles

}  // namespace

// 1 + the neighbor scale of Section 3.2: r_family + r~_neighbor =
// alpha r_family with alpha = (1 - (1-c)^T) / (1 - (1-c)^S), from the norms
// of Lemma 2 (||r_family||_1 = 1 - (1-c)^S, ||r_neighbor||_1 = (1-c)^S -
// (1-c)^T).
double family_alpha(double c, int S, int T) {
    const double pS = std::pow(1.0 - c, (double)S), pT = std::pow(1.0 - c, (double)T);
    return (1.0 - pT) / (1.0 - pS);
}

// First i >= 1 with c (1-c)^i < eps: Algorithm 1's L1 break, with the
// per-block norm ||x'(i)||_1 = c (1-c)^i of Lemma 2.
int64_t stranger_last_iteration(double c, double eps) {
    double norm = c;
    for (int64_t i = 1; i < 100000; ++i) {
        norm = c * std::pow(1.0 - c, (double)i);
        if (norm < eps) return i;
    }
    return 100000;
}

// Schedule shape per seed-tile width: a single vector takes groups of up to
// 512 edges, rows of up to 4*EW edges as one wave item, rows of up to
// 128*EW edges as one block item (4 waves) and chunks of 16*EW beyond; seed tiles
// move kt floats per edge, so their items are shorter and they have no
// block items.
SchedShape choose_shape(const tpa_graph *g, int kt) {
    if (kt == 1) {
        // the single-vector step keeps a group's products in a 512-float LDS slice
        const int ew = g->edges_per_item > 0 ? std::min(g->edges_per_item, kDefaultEW1) : kDefaultEW1;
        return {ew, 4 * ew, 16 * ew, 128 * ew};
    }
    const int ew = g->edges_per_item > 0 ? g->edges_per_item : kDefaultEW64;
    return {ew, 2 * ew, ew, 0};
}

// Automatic seed tile: the next power of two up to 16 for small batches;
// beyond 32 columns the 64-column walk (one column per lane) is fastest for
// both seed lists and dense restarts (measured on R-MAT 2^20: 64 seeds in
// 1.6 ms against 2.9 ms with tiles of 16).
int choose_kt(const tpa_graph *g, int64_t k) {
    if (g->seed_tile > 0) return g->seed_tile;
    if (k <= 1) return 1;
    if (k > 32) return 64;
    int kt = 2;
    while (kt < k && kt < 16) kt <<= 1;
    return kt;
}

// The push accumulator must be zero before the first query on a workspace.
tpa_status clear_push_state(const tpa_graph *g, void *ws, hipStream_t st) {
    TPA_TRY_HIP(hipMemsetAsync(ws, 0, push_plan_clear_bytes(g->n), st));
    return TPA_OK;
}

// Largest frontier edge count for which the second family step is pushed
// rather than pulled: an eighth of the edges (a pushed edge costs a binary
// search, a gather and an atomic; a pulled edge one coalesced index and one
// gather).
int64_t push_wmax(const tpa_graph *g) {
    if (g->push_limit >= 0) return g->push_limit;
    return std::max<int64_t>(1024, g->m / 8);
}

// Largest out-edge count of y2's support for which step 3 of a single seed
// (after a pushed step 2) is pushed: m/20 (a pushed edge costs about 20
// times a pulled one: an atomic and two gathers against a coalesced index
// and one gather), and never when pushes are off.  By default only graphs
// of at least kThirdPushMinEdges edges try it: the list, push and
// conversion launches cost a fixed 20-25 us per query even when the step is
// then pulled, more than the pulls they save on R-MAT graphs of 1.7e7 and
// 6.7e7 edges (125 against 152, 585 against 601 us per query); on 2.2e9
// edges a query takes 28.7 against 30.9 ms.
constexpr int64_t kThirdPushMinEdges = int64_t(1) << 28;

int64_t third_wmax(const tpa_graph *g) {
    if (push_wmax(g) <= 0) return 0;
    if (g->third_push_limit >= 0) return g->third_push_limit;
    if (g->m < kThirdPushMinEdges) return 0;
    return std::max<int64_t>(1024, g->m / 20);
}

namespace {

// Workspace layout: push state (push_plan_bytes, the same for every tile
// width, so its all-zero accumulator survives queries of any width) |
// z0 [n*kt] | z1 [n*kt] | partials [slots * kt] | (dense restarts)
// c*q^T [n*kt] at the next 256-byte boundary (floats)
size_t query_ws_floats_before_qt(const tpa_graph *g, int64_t slots, int kt) {
    const size_t zf = (size_t)g->n * kt;
    const size_t pf = (size_t)std::max<int64_t>(slots, 1) * kt;
    return ((2 * zf + pf) + 63) & ~(size_t)63;
}

size_t query_ws_bytes(const tpa_graph *g, int64_t slots, int kt, bool dense) {
    const size_t qf = dense ? (size_t)g->n * kt : 0;
    return push_plan_bytes(g->n, g->m, third_wmax(g) > 0) +
           sizeof(float) * (query_ws_floats_before_qt(g, slots, kt) + qf) + 256;
}

// Partial slots per column of a query's chunk items: the schedule's, and
// those of the XCD-sliced schedule when single-seed pulls take it.
int64_t query_slots(const Schedule *s, const Schedule *sx) {
    return sx ? std::max(s->n_chunk_items, sx->n_chunk_items) : s->n_chunk_items;
}

tpa_status ensure_ws(tpa_graph *g, size_t bytes, hipStream_t st) {
    if (g->ws_bytes >= bytes) return TPA_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(TPA_ERR_CAPTURE, "query workspace too small during stream capture; call tpa_reserve first");
    if (g->ws) {
        TPA_TRY_HIP(hipStreamSynchronize(st));
        dfree(g->ws);
        g->ws = nullptr;
        g->ws_bytes = 0;
    }
    TPA_TRY(dmalloc(reinterpret_cast<void **>(&g->ws), bytes, st));
    g->ws_bytes = bytes;
    TPA_TRY(clear_push_state(g, g->ws, st));
    TPA_TRY_HIP(hipStreamSynchronize(st));  // ordered before queries on any stream
    return TPA_OK;
}

tpa_status check_query_args(tpa_graph *g, double c, int S, int T) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (!g->preprocessed) return fail(TPA_ERR_NOT_PREPROCESSED, "tpa_preprocess has not run on this graph");
    if (!(c > 0.0 && c < 1.0)) return fail(TPA_ERR_INVALID_ARG, "c must lie in (0, 1)");
    if (S < 1) return fail(TPA_ERR_INVALID_ARG, "S must be >= 1");
    if (T < S) return fail(TPA_ERR_INVALID_ARG, "T must be >= S");
    if (c != g->c || T != g->T)
        return fail(TPA_ERR_PARAM_MISMATCH, "query (c, T) differs from the preprocessed (c, T)");
    return TPA_OK;
}

}  // namespace

// Shared driver: `k` columns; restart from seeds [k] (plain) or
// [nblocks][k] (packed), or from dense seed-major vectors q [k][n].
size_t query_workspace_bytes(tpa_graph *g, int64_t k, bool dense, hipStream_t st) {
    const int kt = choose_kt(g, k);
    const Schedule *s = nullptr;
    if (get_schedule(g, choose_shape(g, kt), st, &s) != TPA_OK) return 0;
    return query_ws_bytes(g, s->n_chunk_items, kt, dense);
}

// Frontier edges up to which a seed tile pushes its second step, summed
// over the tile's columns: by default a quarter of the edges, twice the
// single seed's share (a pulled tile step gathers kt-wide rows per edge, so
// it costs more than a single vector's).
int64_t tile_wmax(const tpa_graph *g) {
    if (g->tile_push_limit >= 0) return g->tile_push_limit;
    return std::max<int64_t>(2048, g->m / 4);
}

bool tile_push_applies(const tpa_graph *g, int kt, bool packed, int S) {
    return kt >= 2 && !packed && S >= 4 && tile_wmax(g) > 0;
}

size_t tile_buf_bytes(const tpa_graph *g, int kt, bool packed, int S) {
    if (!tile_push_applies(g, kt, packed, S)) return 0;
    const size_t bytes = tile_push_bytes(g->n, g->m, kt);
    // the y2 accumulator is 8 bytes per entry: at most 32 GiB, and at most
    // a quarter of the free device memory
    size_t free_b = 0, total_b = 0;
    if (bytes > (size_t(32) << 30)) return 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || bytes > free_b / 4) return 0;
    return bytes;
}

tpa_status tile_buf_alloc(TileBuf *tb, size_t bytes, int kt, hipStream_t st) {
    TPA_TRY(dmalloc(&tb->base, bytes, st));
    tb->bytes = bytes;
    tb->kt_cap = kt;
    TPA_TRY_HIP(hipMemsetAsync(tb->base, 0, bytes, st));
    TPA_TRY_HIP(hipStreamSynchronize(st));  // ordered before queries on any stream
    return TPA_OK;
}

void tile_buf_free(TileBuf *tb) {
    dfree(tb->base);
    *tb = TileBuf();
}

namespace {

// The handle's pushed-tile buffer for kt columns, when it may push (left
// absent under stream capture, where nothing is allocated).
tpa_status ensure_tile_buf(tpa_graph *g, int kt, bool packed, int S, hipStream_t st) {
    if (g->tbuf.base && g->tbuf.kt_cap >= kt) return TPA_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return TPA_OK;
    const size_t bytes = tile_buf_bytes(g, kt, packed, S);
    if (bytes == 0) return TPA_OK;
    if (g->tbuf.base) {
        TPA_TRY_HIP(hipStreamSynchronize(st));
        tile_buf_free(&g->tbuf);
    }
    return tile_buf_alloc(&g->tbuf, bytes, kt, st);
}

}  // namespace

tpa_status run_query(tpa_graph *g, const int32_t *seeds, const float *q, int64_t k, bool packed, double c,
                     int S, int T, float *out, hipStream_t st, float *ws, size_t ws_bytes, bool no_alloc,
                     TileBuf *tb) {
    TPA_TRY(check_query_args(g, c, S, T));
    if (k < 0) return fail(TPA_ERR_INVALID_ARG, "k must be >= 0");
    if (k == 0) return TPA_OK;
    if ((!seeds && !q) || !out) return fail(TPA_ERR_INVALID_ARG, "seeds/q/out is NULL");
    if (packed && !g->node_block) return fail(TPA_ERR_INVALID_ARG, "graph is not packed");
    if (no_alloc && !ws) return fail(TPA_ERR_INVALID_ARG, "a query without allocation needs a workspace");
    const int kt = choose_kt(g, k);
    const Schedule *s = nullptr;
    if (no_alloc) {
        s = find_schedule(g, choose_shape(g, kt));
        if (!s)
            return fail(TPA_ERR_INVALID_ARG, "no work schedule for this seed tile yet (building one allocates): "
                                             "call tpa_reserve(g, k) or run one tpa_query of k seeds first");
    } else {
        TPA_TRY(get_schedule(g, choose_shape(g, kt), st, &s));
    }
    // single seeds on the handle's own workspace pull their dense family
    // steps in XCD slices when preprocessing built them (never built here)
    const int32_t *colx = nullptr;
    const Schedule *sx = !ws && kt == 1 && !packed ? find_sliced_sweep(g, &colx) : nullptr;
    const int64_t slots = query_slots(s, sx);
    if (ws) {
        if (ws_bytes < query_ws_bytes(g, slots, kt, q != nullptr)) return fail(TPA_ERR_INVALID_ARG, "workspace too small");
    } else {
        TPA_TRY(ensure_ws(g, query_ws_bytes(g, slots, kt, q != nullptr), st));
        ws = g->ws;
    }
    const PushPlan pp = push_plan_at(ws, g->n, g->m, push_wmax(g), third_wmax(g));
    float *z0 = reinterpret_cast<float *>(reinterpret_cast<char *>(ws) + push_plan_bytes(g->n, g->m, pp.wmax3 > 0));
    float *z1 = z0 + (size_t)g->n * kt;
    float *part = z1 + (size_t)g->n * kt;
    float *qT = z0 + query_ws_floats_before_qt(g, slots, kt);  // used by dense restarts only
    // a single seed whose step 2 is not the last: push steps 1 and 2 from
    // the seed's neighbourhood when it is small, pull otherwise (decided on
    // the device, so the launch sequence is fixed and capturable)
    const bool push2 = kt == 1 && !packed && !q && S >= 4 && pp.wmax > 0;
    // and its third step when that is not the last either
    const bool push3 = push2 && S >= 5 && pp.wmax3 > 0;
    // pulls after a push skip the rows it left zero (seed tiles of 1 and 64)
    const bool frontier = pp.wmax > 0 && (kt == 1 || kt == 64);
    // a seed tile whose step 2 is not the last: the device pushes step 2 from
    // the columns' seeds when the tile's frontier is small, and pulls it
    // otherwise (steps 1 and 2 are then as without the push)
    bool tpush = tile_push_applies(g, kt, packed, S) && !q && (!no_alloc || tb);
    if (tpush && !tb) {
        TPA_TRY(ensure_tile_buf(g, kt, packed, S, st));
        tb = &g->tbuf;
    }
    tpush = tpush && tb && tb->base && tb->kt_cap >= kt;
    const TilePush tp = tpush ? tile_push_at(tb->base, g->n, g->m, tb->kt_cap, tile_wmax(g)) : TilePush();

    StepParams p;
    p.rowptr = g->t.rowptr;
    p.inv = g->inv_deg;
    p.partials = part;
    p.err = g->dev_err;
    // gathered vectors in hub-first rows (first steps read node ids: t.col
    // and t.w in A~^T's own order)
    const bool hub = g->gather_layout && g->zperm && (!g->weighted || g->t_wz_valid);
    if (hub && kt == 1 && !no_alloc) TPA_TRY(ensure_group_order(g, s, st));  // a no-op under capture
    p.zperm = hub ? g->zperm : nullptr;
    const int32_t *col_gather = hub ? g->t_colz : g->t.col;
    const float *w_gather = g->weighted ? (hub ? g->t_wz : g->t.w) : nullptr;
    p.col = col_gather;
    p.w = w_gather;
    p.omc = (float)(1.0 - c);
    p.c = (float)c;
    p.kt = kt;
    p.node_block = packed ? g->node_block : nullptr;
    p.seed_stride = packed ? (int)k : 0;
    p.alpha = (float)family_alpha(c, S, T);  // 1 + neighbor scale
    p.str = g->str;
    p.out = out;
    p.n = g->n;
    // a pulled family step that gathers hub-first ids: sliced when available,
    // except step 3 behind a frontier skip (its sparse pulls pay for the
    // slice sums of every split row and gain little from the locality)
    auto pull = [&](const StepParams &pp, int step) -> tpa_status {
        if (sx && pp.col == g->t_colz && (!pp.bits || step >= 4)) {
            StepParams px = pp;
            px.col = colx;
            return launch_step(*sx, kFamily, false, px, st);
        }
        return launch_step(*s, kFamily, false, pp, st);
    };
    for (int64_t base = 0; base < k; base += kt) {
        p.seeds = seeds ? seeds + base : nullptr;
        p.qdense = q ? q + base * g->n : nullptr;
        p.ncols = (int)std::min<int64_t>(kt, k - base);
        p.out_col0 = base;
        if (S == 1) {
            p.last = 1;
            TPA_TRY(launch_combine_only(p, st));
            continue;
        }
        p.qT = nullptr;
        if (q) {
            TPA_TRY(launch_dense_transpose(p, qT, st));
            p.qT = qT;
            TPA_TRY(launch_dense_init(p, z0, nullptr, st));
        }
        for (int step = 1; step <= S - 1; ++step) {
            p.zin = (step & 1) ? z0 : z1;
            p.zout = (step & 1) ? z1 : z0;
            p.last = step == S - 1;
            if (step == 1 && !q && !p.last) {
                // one-hot restarts: x(1) lives on the seeds' out-edges; push it
                if (push2) {
                    TPA_TRY(launch_push_steps12(p, g, pp, st));  // steps 1 and 2
                } else {
                    StepParams p1 = p;
                    if (tpush) {
                        TPA_TRY(launch_tile_plan(p, g, tp, st));
                        p1.skip_on = tp.flag;  // x(1) is written only for a pulled step 2
                    }
                    TPA_TRY(launch_push_first(p1, g, packed ? g->nblocks : 1, frontier ? pp.bits : nullptr,
                                              pp.nwords, st));
                    if (tpush) TPA_TRY(launch_tile_push(p, g, tp, st));
                }
                continue;
            }
            if (step == 2 && tpush) {
                // converted from the push, or pulled (each launch runs only in its case)
                TPA_TRY(launch_tile_convert(p, tp, st));
                StepParams p2 = p;
                p2.skip_on = tp.flag;
                p2.bits = frontier ? pp.bits : nullptr;
                p2.bits_on = nullptr;
                p2.col = col_gather;
                p2.w = w_gather;
                TPA_TRY(launch_step(*s, kFamily, false, p2, st));
                continue;
            }
            if (step == 3 && push3) {
                // pushed over y2's support when it is small, else pulled
                // with the frontier skip (each launch runs only in its case)
                StepParams p3 = p;
                p3.col = col_gather;
                p3.w = w_gather;
                TPA_TRY(launch_push_third(p3, g, pp, st));
                TPA_TRY(launch_convert_third(p3, pp, st));
                p3.bits = pp.bits;
                p3.bits_on = pp.flag;
                p3.skip_on = pp.flag3;
                TPA_TRY(pull(p3, step));
                continue;
            }
            if (step == 2 && push2) {
                tpa_status rc = launch_gated_step(*s, p, pp, st);
                if (rc != TPA_OK) {
                    // the conversion that clears acc may not have run: restore
                    // the all-zero push state before reporting the error
                    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
                    if (!no_alloc && hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
                        (void)clear_push_state(g, ws, st);  // (the no-allocation path clears it per call)
                    return rc;
                }
                continue;
            }
            // the step after a push gathers only the rows the push reached:
            // step 3 after the pushed step 2 (when the device took the push),
            // step 2 after a pushed step 1
            p.bits = nullptr;
            p.bits_on = nullptr;
            if (frontier && !q && ((push2 && step == 3) || (!push2 && step == 2))) {
                p.bits = pp.bits;
                p.bits_on = push2 ? pp.flag : nullptr;
            }
            // and step 4 after a pushed step 3 with a small support (its
            // conversion wrote that support into the bitmap)
            if (push3 && step == 4) {
                p.bits = pp.bits;
                p.bits_on = pp.flag4;
            }
            // one-hot restart: the first step needs no gather
            const bool first = step == 1 && !q;
            p.col = first ? g->t.col : col_gather;
            p.w = first ? (g->weighted ? g->t.w : nullptr) : w_gather;
            TPA_TRY(first ? launch_step(*s, kFamily, true, p, st) : pull(p, step));
        }
    }
    return TPA_OK;
}

}  // namespace tpa

using namespace tpa;

extern "C" const char *tpa_status_string(tpa_status s) {
    switch (s) {
        case TPA_OK: return "ok";
        case TPA_ERR_INVALID_ARG: return "invalid argument";
        case TPA_ERR_NOT_PREPROCESSED: return "graph not preprocessed";
        case TPA_ERR_PARAM_MISMATCH: return "query parameters differ from preprocessing";
        case TPA_ERR_OUT_OF_MEMORY: return "out of device memory";
        case TPA_ERR_HIP: return "HIP runtime error";
        case TPA_ERR_INDEX_OVERFLOW: return "index overflow";
        case TPA_ERR_CAPTURE: return "allocation needed during stream capture";
    }
    return "unknown status";
}

extern "C" const char *tpa_last_error_message(void) { return g_last_error.c_str(); }

extern "C" tpa_status tpa_preprocess_ex(tpa_graph_t g, double c, int T, double eps, hipStream_t st) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (!(c > 0.0 && c < 1.0)) return fail(TPA_ERR_INVALID_ARG, "c must lie in (0, 1)");
    if (T < 0) return fail(TPA_ERR_INVALID_ARG, "T must be >= 0");
    if (!(eps > 0.0)) return fail(TPA_ERR_INVALID_ARG, "eps must be > 0");
    g->preprocessed = false;
    ++g->version;
    const int64_t K = stranger_last_iteration(c, eps);
    const Schedule *s = nullptr;
    TPA_TRY(get_schedule(g, choose_shape(g, 1), st, &s));
    // iterates kept for the adjoint: K x n floats, when they fit in a quarter
    // of the free device memory
    g->xiter_K = 0;
    if (g->keep_iterates) {
        const size_t need = (size_t)K * (size_t)g->n;
        size_t free_b = 0, total_b = 0;
        if (!g->xiter || g->xiter_cap < need) {
            dfree(g->xiter);
            g->xiter = nullptr;
            g->xiter_cap = 0;
            if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && need * sizeof(float) <= free_b / 4 &&
                dalloc(&g->xiter, need, st) == TPA_OK)
                g->xiter_cap = need;
        }
    }
    float *xit = (g->keep_iterates && g->xiter) ? g->xiter : nullptr;
    if (g->gather_layout) {
        TPA_TRY(ensure_zlayout(g, st));
        TPA_TRY(ensure_wz(g, st));
    }
    const bool hub = g->gather_layout && g->zperm && (!g->weighted || g->t_wz_valid);
    if (hub) TPA_TRY(ensure_group_order(g, s, st));
    // large graphs sweep in XCD slices (when the graph takes them)
    const Schedule *sx = nullptr;
    const int32_t *colx = nullptr;
    if (hub) TPA_TRY(ensure_sliced_sweep(g, st, &sx, &colx));
    if (sx) s = sx;
    if (!g->str) TPA_TRY(dalloc(&g->str, g->n, st));
    float *tmp = nullptr;
    const size_t n = (size_t)g->n;
    TPA_TRY(dalloc(&tmp, 3 * n + (size_t)std::max<int64_t>(s->n_chunk_items, 1), st));
    float *z0 = tmp, *z1 = tmp + n, *comp = tmp + 2 * n, *part = tmp + 3 * n;
    tpa_status rc = TPA_OK;
    if (xit) rc = launch_stranger_init(g, (float)c, 1, z0, xit, comp, hub ? g->zperm : nullptr, st);  // x'(0)
    if (rc == TPA_OK) rc = launch_stranger_init(g, (float)c, T == 0, z0, g->str, comp, hub ? g->zperm : nullptr, st);
    StepParams p;
    p.rowptr = g->t.rowptr;
    p.col = colx ? colx : hub ? g->t_colz : g->t.col;
    p.zperm = hub ? g->zperm : nullptr;
    p.w = g->weighted ? (hub ? g->t_wz : g->t.w) : nullptr;
    p.inv = g->inv_deg;
    p.partials = part;
    p.omc = (float)(1.0 - c);
    p.c = (float)c;
    p.kt = 1;
    p.n = g->n;
    p.acc = g->str;
    p.comp = comp;
    for (int64_t i = 1; rc == TPA_OK && i <= K; ++i) {
        p.zin = (i & 1) ? z0 : z1;
        p.zout = (i & 1) ? z1 : z0;
        p.accumulate = i >= T;
        p.xs_out = (xit && i < K) ? xit + (size_t)i * n : nullptr;
        rc = launch_step(*s, kStranger, false, p, st);
    }
    hipError_t e = hipStreamSynchronize(st);
    dfree(tmp);
    if (rc != TPA_OK) return rc;
    TPA_TRY_HIP(e);
    g->c = c;
    g->T = T;
    g->eps = eps;
    g->K = K;
    g->xiter_K = xit ? K : 0;
    g->preprocessed = true;
    return TPA_OK;
}

extern "C" tpa_status tpa_preprocess(tpa_graph_t g, double c, int T, hipStream_t st) {
    return tpa_preprocess_ex(g, c, T, 1e-9, st);
}

extern "C" tpa_status tpa_preprocess_info(tpa_graph_t g, double *c, int *T, double *eps, int64_t *K) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (!g->preprocessed) return fail(TPA_ERR_NOT_PREPROCESSED, "tpa_preprocess has not run on this graph");
    if (c) *c = g->c;
    if (T) *T = g->T;
    if (eps) *eps = g->eps;
    if (K) *K = g->K;
    return TPA_OK;
}

extern "C" tpa_status tpa_neighbor_scale(double c, int S, int T, double *scale) {
    if (!scale) return fail(TPA_ERR_INVALID_ARG, "scale is NULL");
    if (!(c > 0.0 && c < 1.0)) return fail(TPA_ERR_INVALID_ARG, "c must lie in (0, 1)");
    if (S < 1) return fail(TPA_ERR_INVALID_ARG, "S must be >= 1");
    if (T < S) return fail(TPA_ERR_INVALID_ARG, "T must be >= S");
    *scale = family_alpha(c, S, T) - 1.0;
    return TPA_OK;
}

extern "C" tpa_status tpa_stranger(tpa_graph_t g, float *out, hipStream_t st) {
    if (!g || !out) return fail(TPA_ERR_INVALID_ARG, "NULL argument");
    if (!g->preprocessed) return fail(TPA_ERR_NOT_PREPROCESSED, "tpa_preprocess has not run on this graph");
    TPA_TRY_HIP(hipMemcpyAsync(out, g->str, sizeof(float) * g->n, hipMemcpyDeviceToDevice, st));
    return TPA_OK;
}

extern "C" tpa_status tpa_query(tpa_graph_t g, const int32_t *seeds, int64_t k, double c, int S, int T,
                                float *out, hipStream_t st) {
    return run_query(g, seeds, nullptr, k, false, c, S, T, out, st, nullptr, 0);
}

extern "C" tpa_status tpa_query_dense(tpa_graph_t g, const float *q, int64_t k, double c, int S, int T,
                                      float *out, hipStream_t st) {
    if (k > 0 && !q) return fail(TPA_ERR_INVALID_ARG, "q is NULL");
    return run_query(g, nullptr, q, k, false, c, S, T, out, st, nullptr, 0);
}

extern "C" tpa_status tpa_query_packed(tpa_graph_t g, const int32_t *seeds, int per_block, double c, int S,
                                       int T, float *out, hipStream_t st) {
    if (per_block < 1) return fail(TPA_ERR_INVALID_ARG, "per_block must be >= 1");
    return run_query(g, seeds, nullptr, per_block, true, c, S, T, out, st, nullptr, 0);
}

extern "C" tpa_status tpa_query_workspace_size(tpa_graph_t g, int64_t k, size_t *bytes) {
    if (!g || !bytes || k < 0) return fail(TPA_ERR_INVALID_ARG, "bad argument");
    *bytes = query_workspace_bytes(g, k, true, nullptr);
    if (*bytes == 0) return fail(TPA_ERR_HIP, "could not build the work schedule");
    return TPA_OK;
}

extern "C" tpa_status tpa_reserve(tpa_graph_t g, int64_t k) {
    if (!g || k < 0) return fail(TPA_ERR_INVALID_ARG, "bad argument");
    const int kt = choose_kt(g, k);
    const Schedule *s = nullptr;
    TPA_TRY(get_schedule(g, choose_shape(g, kt), nullptr, &s));
    const bool hub = g->gather_layout && g->zperm && (!g->weighted || g->t_wz_valid);
    if (hub && kt == 1) TPA_TRY(ensure_group_order(g, s, nullptr));  // not buildable under capture
    TPA_TRY(ensure_tile_buf(g, kt, false, 4, nullptr));  // for seed tiles whose step 2 may be pushed
    const int32_t *colx = nullptr;
    const Schedule *sx = kt == 1 ? find_sliced_sweep(g, &colx) : nullptr;
    return ensure_ws(g, query_ws_bytes(g, query_slots(s, sx), kt, true), nullptr);  // room for dense restarts too
}

extern "C" tpa_status tpa_set_tuning(tpa_graph_t g, int seed_tile, int edges_per_item) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (seed_tile != 0 && seed_tile != 1 && seed_tile != 2 && seed_tile != 4 && seed_tile != 8 &&
        seed_tile != 16 && seed_tile != 32 && seed_tile != 64)
        return fail(TPA_ERR_INVALID_ARG, "seed tile must be 0, 1, 2, 4, 8, 16, 32 or 64");
    if (edges_per_item != 0 && (edges_per_item < 64 || edges_per_item > 1024 || edges_per_item % 64))
        return fail(TPA_ERR_INVALID_ARG, "edges per item must be 0 or a multiple of 64 in 64..1024");
    g->seed_tile = seed_tile;
    g->edges_per_item = edges_per_item;
    return TPA_OK;
}

extern "C" tpa_status tpa_get_tuning(tpa_graph_t g, int *seed_tile, int *edges_per_item) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (seed_tile) *seed_tile = g->seed_tile;
    if (edges_per_item) *edges_per_item = g->edges_per_item;
    return TPA_OK;
}

extern "C" tpa_status tpa_set_gather_layout(tpa_graph_t g, int hub_first) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (hub_first < 0 || hub_first > 2) return fail(TPA_ERR_INVALID_ARG, "layout must be 0, 1 or 2");
    if (hub_first < 2) drop_group_order(g);
    g->gather_layout = hub_first;
    if (hub_first && g->preprocessed) {
        TPA_TRY(ensure_zlayout(g, nullptr));
        TPA_TRY(ensure_wz(g, nullptr));
        const Schedule *s = nullptr;
        TPA_TRY(get_schedule(g, choose_shape(g, 1), nullptr, &s));
        TPA_TRY(ensure_group_order(g, s, nullptr));
        TPA_TRY_HIP(hipStreamSynchronize(nullptr));
    }
    return TPA_OK;
}

extern "C" tpa_status tpa_get_gather_layout(tpa_graph_t g, int *hub_first) {
    if (!g || !hub_first) return fail(TPA_ERR_INVALID_ARG, "NULL argument");
    *hub_first = g->gather_layout;
    return TPA_OK;
}

extern "C" tpa_status tpa_set_sliced_sweep(tpa_graph_t g, int mode) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (mode < 0 || mode > 2) return fail(TPA_ERR_INVALID_ARG, "mode must be 0, 1 or 2");
    g->sliced_sweep = mode;
    return TPA_OK;
}

extern "C" tpa_status tpa_get_sliced_sweep(tpa_graph_t g, int *mode, int *active) {
    if (!g || !mode) return fail(TPA_ERR_INVALID_ARG, "NULL argument");
    *mode = g->sliced_sweep;
    if (active) {
        const int32_t *colx = nullptr;
        *active = find_sliced_sweep(g, &colx) != nullptr;
    }
    return TPA_OK;
}

extern "C" tpa_status tpa_set_keep_iterates(tpa_graph_t g, int keep) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    g->keep_iterates = keep != 0;
    if (!keep) {
        (void)hipDeviceSynchronize();  // no kernel may still read them
        dfree(g->xiter);
        g->xiter = nullptr;
        g->xiter_K = 0;
        g->xiter_cap = 0;
    }
    return TPA_OK;
}

extern "C" tpa_status tpa_set_push_limit(tpa_graph_t g, int64_t max_edges) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (max_edges < -1) return fail(TPA_ERR_INVALID_ARG, "max_edges must be >= -1");
    g->push_limit = max_edges;
    return TPA_OK;
}

extern "C" tpa_status tpa_get_push_limit(tpa_graph_t g, int64_t *max_edges) {
    if (!g || !max_edges) return fail(TPA_ERR_INVALID_ARG, "NULL argument");
    *max_edges = g->push_limit;
    return TPA_OK;
}

extern "C" tpa_status tpa_set_tile_push_limit(tpa_graph_t g, int64_t max_edges) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (max_edges < -1) return fail(TPA_ERR_INVALID_ARG, "max_edges must be >= -1");
    g->tile_push_limit = max_edges;
    return TPA_OK;
}

extern "C" tpa_status tpa_get_tile_push_limit(tpa_graph_t g, int64_t *max_edges) {
    if (!g || !max_edges) return fail(TPA_ERR_INVALID_ARG, "bad argument");
    *max_edges = g->tile_push_limit;
    return TPA_OK;
}

extern "C" tpa_status tpa_set_third_push_limit(tpa_graph_t g, int64_t max_edges) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (max_edges < -1) return fail(TPA_ERR_INVALID_ARG, "max_edges must be >= -1");
    g->third_push_limit = max_edges;
    return TPA_OK;
}

extern "C" tpa_status tpa_get_third_push_limit(tpa_graph_t g, int64_t *max_edges) {
    if (!g || !max_edges) return fail(TPA_ERR_INVALID_ARG, "bad argument");
    *max_edges = g->third_push_limit;
    return TPA_OK;
}

extern "C" tpa_status tpa_get_device_error(tpa_graph_t g, hipStream_t st) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    int32_t v = 0;
    TPA_TRY_HIP(hipMemcpyAsync(&v, g->dev_err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TPA_TRY_HIP(hipStreamSynchronize(st));
    if (v) {
        TPA_TRY_HIP(hipMemsetAsync(g->dev_err, 0, sizeof(int32_t), st));
        TPA_TRY_HIP(hipStreamSynchronize(st));
        return fail(TPA_ERR_INVALID_ARG, "a query saw a seed outside [0, n) or outside its block");
    }
    return TPA_OK;
}

// ---------------------------------------------------------------- no-allocation query
// For callers that cannot allocate device memory (code under stream capture,
// serving loops, harnesses that forbid hipMalloc): the query workspace is a
// file-scope device array of kScratchBytes, one copy per device, held until
// the process ends.  Host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in there).  Every call on a device shares that device's
// array and finds the previous call's contents, so the part that must start
// at zero (the push accumulator) is cleared by a fill kernel on every call;
// calls that overlap on one device race.

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's scratch array, looked up once per
// device with that device current.
tpa_status scratch_address(void **out) {
    int dev = 0;
    TPA_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(TPA_ERR_INVALID_ARG, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(TPA_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return TPA_OK;
}

}  // namespace

extern "C" tpa_status tpa_query_noalloc(tpa_graph_t g, const int32_t *seeds, int64_t k, double c, int S, int T,
                                        float *out, hipStream_t st) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (k < 0) return fail(TPA_ERR_INVALID_ARG, "k must be >= 0");
    if (k == 0) return TPA_OK;
    TPA_TRY(check_query_args(g, c, S, T));
    if (!seeds || !out) return fail(TPA_ERR_INVALID_ARG, "seeds/out is NULL");
    const int kt = choose_kt(g, k);
    const Schedule *s = find_schedule(g, choose_shape(g, kt));
    if (!s)
        return fail(TPA_ERR_INVALID_ARG, "no work schedule for this seed tile yet (building one allocates): "
                                         "call tpa_reserve(g, k) or run one tpa_query of k seeds first");
    // the query workspace, then (seed tiles whose step 2 may be pushed) the
    // pushed-tile buffer
    const size_t wsb = (query_ws_bytes(g, s->n_chunk_items, kt, false) + 255) & ~(size_t)255;
    const size_t tbytes = tile_push_applies(g, kt, false, S) ? tile_push_bytes(g->n, g->m, kt) : 0;
    const size_t need = wsb + tbytes;
    if (need > kScratchBytes)
        return fail(TPA_ERR_INVALID_ARG, "the query needs " + std::to_string(need) +
                                             " bytes of workspace; tpa_query_noalloc holds at most " +
                                             std::to_string(kScratchBytes));
    void *ws = nullptr;
    TPA_TRY(scratch_address(&ws));
    // the push accumulators must be all zero when a query starts
    TPA_TRY(launch_fill_zero(static_cast<float *>(ws), (int64_t)(push_plan_clear_bytes(g->n) / 4), st));
    TileBuf tb;
    if (tbytes) {
        tb.base = static_cast<char *>(ws) + wsb;
        tb.bytes = tbytes;
        tb.kt_cap = kt;
        TPA_TRY(launch_fill_zero(static_cast<float *>(tb.base), (int64_t)(tbytes / 4), st));
    }
    return run_query(g, seeds, nullptr, k, false, c, S, T, out, st, static_cast<float *>(ws), wsb, true,
                     tbytes ? &tb : nullptr);
}
