// Query capture (HIP graphs) and the query autotuner.
//
// A captured query replays the whole launch sequence of tpa_query (every
// seed tile's S-1 CPI steps and the fused combine) with one hipGraphLaunch;
// the seeds / restart / output buffers are fixed at capture and their
// contents may change between replays.  The capture owns its workspace, so
// it stays valid while other queries run on the handle (not concurrently
// with a replay).
//
// The autotuner times the candidate (seed tile, group edge budget) pairs on
// the caller's seeds, keeps only candidates whose outputs agree with the
// single-vector reference path (L1 <= 1e-5 per checked seed), and stores the
// fastest on the handle.

#include <algorithm>
#include <cmath>
#include <vector>

#include "cpi_kernels.h"

struct tpa_query_graph {
    tpa_graph *g = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float *ws = nullptr;
    size_t ws_bytes = 0;
    tpa::TileBuf tbuf;  // its own pushed-tile buffer (seed tiles)
};

namespace tpa {
namespace {

// Per-row L1 distance between two seed-major [rows][n] blocks, one block per
// row with a fixed-order tree reduction.
__global__ void row_l1_kernel(const float *a, const float *b, int64_t n, double *out) {
    __shared__ double red[256];
    const int64_t row = blockIdx.x;
    double s = 0.0;
    for (int64_t v = threadIdx.x; v < n; v += blockDim.x)
        s += fabs((double)a[row * n + v] - (double)b[row * n + v]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[row] = red[0];
}

}  // namespace
}  // namespace tpa

using namespace tpa;

extern "C" tpa_status tpa_query_graph_create(tpa_graph_t g, const int32_t *seeds, const float *q, int64_t k,
                                             int packed, double c, int S, int T, float *out, hipStream_t st,
                                             tpa_query_graph_t *out_graph) {
    if (!out_graph) return fail(TPA_ERR_INVALID_ARG, "out_graph is NULL");
    *out_graph = nullptr;
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (k < 1) return fail(TPA_ERR_INVALID_ARG, "k must be >= 1");
    if ((seeds == nullptr) == (q == nullptr)) return fail(TPA_ERR_INVALID_ARG, "pass exactly one of seeds and q");
    if (!g->preprocessed) return fail(TPA_ERR_NOT_PREPROCESSED, "tpa_preprocess has not run on this graph");
    // schedules and workspace exist before capture (their set-up synchronises)
    const size_t bytes = query_workspace_bytes(g, k, q != nullptr, st);
    if (bytes == 0) return fail(TPA_ERR_HIP, "could not build the work schedule");
    tpa_query_graph *qg = new tpa_query_graph();
    qg->g = g;
    tpa_status rc = dmalloc(reinterpret_cast<void **>(&qg->ws), bytes, st);
    if (rc != TPA_OK) { delete qg; return rc; }
    qg->ws_bytes = bytes;
    rc = clear_push_state(g, qg->ws, st);
    if (rc == TPA_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(TPA_ERR_HIP, "hipStreamSynchronize failed");
    const size_t tbytes = seeds ? tile_buf_bytes(g, choose_kt(g, k), packed != 0, S) : 0;
    if (rc == TPA_OK && tbytes) rc = tile_buf_alloc(&qg->tbuf, tbytes, choose_kt(g, k), st);
    if (rc != TPA_OK) { tile_buf_free(&qg->tbuf); dfree(qg->ws); delete qg; return rc; }
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        tile_buf_free(&qg->tbuf); dfree(qg->ws); delete qg;
        return fail(TPA_ERR_HIP, "hipStreamCreate failed");
    }
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = run_query(g, seeds, q, k, packed != 0, c, S, T, out, cs, qg->ws, qg->ws_bytes, false, &qg->tbuf);
        hipError_t e2 = hipStreamEndCapture(cs, &qg->graph);
        if (rc == TPA_OK && e2 != hipSuccess) rc = fail(TPA_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    } else {
        rc = fail(TPA_ERR_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    if (rc == TPA_OK && hipGraphInstantiate(&qg->exec, qg->graph, nullptr, nullptr, 0) != hipSuccess)
        rc = fail(TPA_ERR_HIP, "hipGraphInstantiate failed");
    (void)hipStreamDestroy(cs);
    if (rc != TPA_OK) {
        if (qg->exec) (void)hipGraphExecDestroy(qg->exec);
        if (qg->graph) (void)hipGraphDestroy(qg->graph);
        tile_buf_free(&qg->tbuf);
        dfree(qg->ws);
        delete qg;
        return rc;
    }
    *out_graph = qg;
    return TPA_OK;
}

extern "C" tpa_status tpa_query_graph_launch(tpa_query_graph_t qg, hipStream_t st) {
    if (!qg || !qg->exec) return fail(TPA_ERR_INVALID_ARG, "query graph is NULL");
    TPA_TRY_HIP(hipGraphLaunch(qg->exec, st));
    return TPA_OK;
}

extern "C" tpa_status tpa_query_graph_destroy(tpa_query_graph_t qg) {
    if (!qg) return TPA_OK;
    (void)hipDeviceSynchronize();
    if (qg->exec) (void)hipGraphExecDestroy(qg->exec);
    if (qg->graph) (void)hipGraphDestroy(qg->graph);
    tile_buf_free(&qg->tbuf);
    dfree(qg->ws);
    delete qg;
    return TPA_OK;
}

extern "C" tpa_status tpa_autotune(tpa_graph_t g, const int32_t *seeds, int64_t k, double c, int S, int T,
                                   float *scratch_out, int *best_tile, int *best_ew, double *best_ms,
                                   hipStream_t st) {
    if (!g || !seeds || !scratch_out || k < 1) return fail(TPA_ERR_INVALID_ARG, "bad argument");
    if (!g->preprocessed) return fail(TPA_ERR_NOT_PREPROCESSED, "tpa_preprocess has not run on this graph");
    const int saved_tile = g->seed_tile, saved_ew = g->edges_per_item;
    const int64_t n = g->n;
    const int64_t nref = std::min<int64_t>(k, 8);
    float *ref = nullptr;
    double *l1 = nullptr;
    TPA_TRY(dalloc(&ref, (size_t)nref * n, st));
    if (dalloc(&l1, nref, st) != TPA_OK) { dfree(ref); return TPA_ERR_OUT_OF_MEMORY; }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    auto cleanup = [&]() {
        dfree(ref); dfree(l1);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    // reference: the single-vector path on the first seeds
    g->seed_tile = 1;
    g->edges_per_item = 0;
    tpa_status rc = run_query(g, seeds, nullptr, nref, false, c, S, T, ref, st, nullptr, 0);
    if (rc != TPA_OK) { g->seed_tile = saved_tile; g->edges_per_item = saved_ew; cleanup(); return rc; }

    std::vector<int> tiles;
    if (k <= 4) tiles.push_back(1);
    for (int t : {8, 16, 32, 64})
        if (t <= 2 * k || t == 8) tiles.push_back(t);
    if (k == 1) tiles = {1};
    const int ews[] = {128, 256, 512, 1024};
    double best = 1e300;
    int bt = 0, be = 0;
    for (int t : tiles) {
        for (int ew : ews) {
            if (t == 1 && ew > 512) continue;  // the single-vector step caps groups at 512 edges
            g->seed_tile = t;
            g->edges_per_item = ew;
            rc = run_query(g, seeds, nullptr, k, false, c, S, T, scratch_out, st, nullptr, 0);  // warm-up
            if (rc != TPA_OK) break;
            double ms = 1e300;
            for (int rep = 0; rep < 2 && rc == TPA_OK; ++rep) {
                (void)hipEventRecord(e0, st);
                rc = run_query(g, seeds, nullptr, k, false, c, S, T, scratch_out, st, nullptr, 0);
                (void)hipEventRecord(e1, st);
                (void)hipEventSynchronize(e1);
                float t_ms = 0.f;
                (void)hipEventElapsedTime(&t_ms, e0, e1);
                ms = std::min(ms, (double)t_ms);
            }
            if (rc != TPA_OK) break;
            row_l1_kernel<<<(unsigned)nref, 256, 0, st>>>(scratch_out, ref, n, l1);
            std::vector<double> h(nref);
            if (hipMemcpyAsync(h.data(), l1, sizeof(double) * nref, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                rc = fail(TPA_ERR_HIP, "autotune parity readback failed");
                break;
            }
            const bool ok = std::all_of(h.begin(), h.end(), [](double d) { return d <= 1e-5; });
            if (ok && ms < best) {
                best = ms;
                bt = t;
                be = ew;
            }
        }
        if (rc != TPA_OK) break;
    }
    cleanup();
    if (rc != TPA_OK || bt == 0) {
        g->seed_tile = saved_tile;
        g->edges_per_item = saved_ew;
        return rc != TPA_OK ? rc : fail(TPA_ERR_HIP, "no autotune candidate passed the parity check");
    }
    g->seed_tile = bt;
    g->edges_per_item = be;
    if (best_tile) *best_tile = bt;
    if (best_ew) *best_ew = be;
    if (best_ms) *best_ms = best;
    return TPA_OK;
}
