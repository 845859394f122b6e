// Reverse-mode derivative of the TPA hot path (an extension of the paper:
// its CPI recursions of Section 2.3 / Algorithms 2-3, differentiated).
//
// For one CPI chain x(i) = (1-c) A~^T x(i-1), i = 1..N, with loss
// L = sum_i beta_i <g, x(i)>, the adjoint lambda(i) = dL/dx(i) obeys
//     lambda(N) = beta_N g,   lambda(i-1) = beta_{i-1} g + (1-c) A~ lambda(i),
// and dL/dA~_uv = (1-c) sum_{i=1..N} x(i-1)[u] lambda(i)[v].  TPA has two
// such chains per loss L = sum_j <grad_out_j, r_TPA_j>:
//   family   (per restart vector q_j): x(0) = c q_j, N = S-1, beta = 1 + scale;
//            dL/dq_j = c lambda(0)
//   stranger (PageRank, once for g = sum_j grad_out_j): x'(0) = c/n_g per
//            block, N = K, beta_i = [i >= T]
// The row-softmax backward then gives dL/dtheta_uv = A~_uv (G_uv - sum_w A~_uw G_uw).
//
// One adjoint step is a pull over the rows of A~ (out-edges): the gather of
// lambda(i)[v] serves both the row sum for lambda(i-1)[u] and the per-edge
// gradient term, fused in one pass.  Work items are the wave items of the
// forward kernels, built over A~'s rows.  The stranger chain's iterates are
// checkpointed every C steps and recomputed per segment (memory (K/C + C)
// vectors instead of K).

#include <algorithm>
#include <cmath>
#include <vector>

#include "cpi_kernels.h"
#include "profile.h"

namespace tpa {
namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kGroupMax = kGroupEdges;  // max edges of a group item (LDS floats per wave)

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct AdjParams {
    const int64_t *rowptr = nullptr;   // A~ (rows = sources u)
    const int32_t *col = nullptr;      // destinations v
    const float *w = nullptr;          // A~ weights in A~ order, or null (1/outdeg)
    const float *inv = nullptr;        // 1/outdeg
    const LongRow *longs = nullptr;
    const float *lam_in = nullptr;     // lambda(i), [n][kt]
    float *lam_out = nullptr;          // lambda(i-1), [n][kt]
    const float *xprev = nullptr;      // x(i-1), [n][kt] (null: no edge gradient)
    float *G = nullptr;                // dL/dA~, [m] in A~ order
    const float *gvec = nullptr;       // kt == 1: g [n]; kt > 1: grad_out tile, seed-major
    int64_t g_stride = 0;              // seed-major row stride (n) for kt > 1
    float beta = 0.f;                  // beta_{i-1}
    float omc = 0.f;                   // 1 - c
    int kt = 1;
    int ncols = 1;
    int64_t n = 0;
    float *partials = nullptr;         // chunk partials [chunk items][kt]
    const float *gT = nullptr;         // kt == 64: grad_out tile node-major [n][64]
    int col_slots = 0;                 // kt == 1: col is the schedule's colg (group items in
                                       // gather order, each entry with its LDS slot); set by adj_step
    const int32_t *lrow = nullptr;     // row of node v in lambda (rank by in-degree; null: v);
                                       // col then holds rows of lambda
    // XCD-sliced schedules (kt == 1): a chunk item's partial slot is its row0
    // and slot_row[slot] its row; set by adj_step from the schedule
    int chunk_slot_in_item = 0;
    const int32_t *slot_row = nullptr;
};

// Row of node u in the lambda vectors.
__device__ __forceinline__ int64_t lam_row(const AdjParams &p, int64_t u) { return p.lrow ? p.lrow[u] : u; }

__device__ __forceinline__ float g_of(const AdjParams &p, int64_t u, int j) {
    if (p.kt == 1) return p.gvec[u];
    return j < p.ncols ? p.gvec[(int64_t)j * p.g_stride + u] : 0.0f;
}

// lambda(i-1)[u][j] = beta g + (1-c) * (explicit weights ? sum : sum / outdeg(u))
__device__ __forceinline__ void adj_epilogue(const AdjParams &p, int64_t u, int j, float sum) {
    const float s = p.w ? sum : sum * p.inv[u];
    p.lam_out[lam_row(p, u) * p.kt + j] = fmaf(p.beta, g_of(p, u, j), p.omc * s);
}

// ------------------------------------------------------------ kt == 1
template <bool WEIGHTED, bool WITHG>
__global__ __launch_bounds__(kThreads) void adj_kernel_1(const Item *__restrict__ items, int64_t n_items,
                                                         AdjParams p) {
    __shared__ float lds_v[kWaves][kGroupMax];
    __shared__ float lds_x[kWaves][kGroupMax];
    // lambda(i)[v] by edge position, for the edge gradient of weighted
    // graphs in gather order (lds_v then holds w * lambda)
    __shared__ float lds_l[WEIGHTED && WITHG ? kWaves : 1][WEIGHTED && WITHG ? kGroupMax : 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + wv;
    if (wid >= n_items) return;
    const Item it = items[wid];
    const int kind = (int)item_kind(it.meta);
    const int nnz = (int)item_nnz(it.meta);
    const int32_t *col = p.col + it.e0;
    if (kind == (int)kItemGroup) {
        constexpr int NS = kGroupMax / 64;
        const int nrows = (int)item_nrows(it.meta);
        const int rel = lane <= nrows ? (int)(p.rowptr[it.row0 + lane] - it.e0) : nnz;
        // In gather order (col_slots) entry e holds the destination to gather
        // and, above it, the edge's position in the item: lambda goes to LDS
        // at that position, so the row sums and the edge gradient (which read
        // LDS by position) are those of the row order, bit for bit.
        const bool slots = p.col_slots != 0;
        int32_t v[NS];
        int pos[NS];
        float gold[NS];  // G of the item's edges (by position), read together with the column ids
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int e = s * 64 + lane;
            const uint32_t raw = e < nnz ? (uint32_t)col[e] : ~0u;
            v[s] = e < nnz ? (int32_t)(slots ? raw & kGroupRowMask : raw) : -1;
            pos[s] = slots ? (int)(raw >> kGroupSlotShift) : e;
            gold[s] = (WITHG && e < nnz) ? p.G[it.e0 + e] : 0.0f;
        }
        const float xr = (WITHG && lane < nrows) ? p.omc * p.xprev[it.row0 + lane] : 0.0f;
        // epilogue operands of row (row0 + lane), loaded ahead
        const float gu = lane < nrows ? p.gvec[it.row0 + lane] : 0.0f;
        const float iu = (!WEIGHTED && lane < nrows) ? p.inv[it.row0 + lane] : 0.0f;
        const int32_t lr = lane < nrows ? (int32_t)lam_row(p, it.row0 + lane) : 0;
        float l[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) l[s] = v[s] >= 0 ? p.lam_in[v[s]] : 0.0f;
        const int rel_next = __shfl(rel, lane + 1 < 64 ? lane + 1 : 63, 64);
        const int len = rel_next - rel;
        float *my = lds_v[wv];
        float *mx = lds_x[wv];
        if (WITHG) {
            // expand (1-c) x(i-1)[row] over the row's edges
            if (lane < nrows && len <= 32)
                for (int k = rel; k < rel_next; ++k) mx[k] = xr;
            uint64_t big = __ballot(lane < nrows && len > 32);
            while (big) {
                const int r = __builtin_ctzll(big);
                big &= big - 1;
                const int b = __builtin_amdgcn_readlane(rel, r), en = __builtin_amdgcn_readlane(rel_next, r);
                const float xv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xr), r));
                for (int k = b + lane; k < en; k += 64) mx[k] = xv;
            }
            wave_sync();
        }
        if (!slots) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int e = s * 64 + lane;
                if (s * 64 < nnz) {
                    if (WITHG && e < nnz) p.G[it.e0 + e] = gold[s] + mx[e] * l[s];
                    my[e] = (WEIGHTED && e < nnz) ? p.w[it.e0 + e] * l[s] : l[s];
                }
            }
        } else {
            float *ml = lds_l[WEIGHTED && WITHG ? wv : 0];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (v[s] >= 0) {
                    my[pos[s]] = WEIGHTED ? p.w[it.e0 + pos[s]] * l[s] : l[s];
                    if (WEIGHTED && WITHG) ml[pos[s]] = l[s];
                }
            }
            wave_sync();
            if (WITHG) {
                const float *lp = WEIGHTED ? ml : my;  // lambda(i)[v] by edge position
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int e = s * 64 + lane;
                    if (e < nnz) p.G[it.e0 + e] = gold[s] + mx[e] * lp[e];
                }
            }
        }
        wave_sync();
        if (lane < nrows && len <= 32) {
            float acc = 0.0f;
            for (int k = rel; k < rel_next; ++k) acc += my[k];
            p.lam_out[lr] = fmaf(p.beta, gu, p.omc * (WEIGHTED ? acc : acc * iu));
        }
        uint64_t big = __ballot(lane < nrows && len > 32);
        while (big) {
            const int r = __builtin_ctzll(big);
            big &= big - 1;
            const int b = __builtin_amdgcn_readlane(rel, r), en = __builtin_amdgcn_readlane(rel_next, r);
            float t = 0.0f;
            for (int k = b + lane; k < en; k += 64) t += my[k];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
            const float gr = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(gu), r));
            const float ir = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(iu), r));
            const int32_t lrr = __builtin_amdgcn_readlane(lr, r);
            if (lane == 0) p.lam_out[lrr] = fmaf(p.beta, gr, p.omc * (WEIGHTED ? t : t * ir));
        }
        return;
    }
    // one row or one chunk of a long row
    const int64_t row = kind == (int)kItemRow     ? (int64_t)it.row0
                        : p.chunk_slot_in_item ? (int64_t)p.slot_row[it.row0]
                                               : (int64_t)p.longs[it.row0].row;
    const float xr = WITHG ? p.omc * p.xprev[row] : 0.0f;
    const bool whole = kind == (int)kItemRow;
    const float gu = whole ? p.gvec[row] : 0.0f;
    const float iu = (whole && !WEIGHTED) ? p.inv[row] : 0.0f;
    constexpr int UNR = 16;
    float s = 0.0f;
    for (int base = 0; base < nnz; base += 64 * UNR) {
        int32_t v[UNR];
        float gold[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const int e = base + k * 64 + lane;
            v[k] = e < nnz ? col[e] : -1;
            gold[k] = (WITHG && e < nnz) ? p.G[it.e0 + e] : 0.0f;
        }
        float l[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) l[k] = v[k] >= 0 ? p.lam_in[v[k]] : 0.0f;
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const int e = base + k * 64 + lane;
            if (v[k] >= 0) {
                if (WITHG) p.G[it.e0 + e] = gold[k] + xr * l[k];
                s += WEIGHTED ? p.w[it.e0 + e] * l[k] : l[k];
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        if (whole)
            p.lam_out[lam_row(p, row)] = fmaf(p.beta, gu, p.omc * (WEIGHTED ? s : s * iu));
        else
            p.partials[p.chunk_slot_in_item ? (int64_t)it.row0 : wid] = s;
    }
}

// ------------------------------------------------------------ kt >= 2
// Lanes (sub, j): 64/KT sub-groups stride over a row's edges, lane j holds
// column j.  The edge gradient term sum_j x_j(i-1)[u] lambda_j(i)[v] is a
// xor-reduction over the KT lanes of a sub-group.
template <int KT, bool WEIGHTED, bool WITHG>
__device__ __forceinline__ float adj_range_kt(const AdjParams &p, int64_t row, int64_t e0, int64_t e1, int sub,
                                              int j) {
    constexpr int SUBS = 64 / KT;
    const float xr = WITHG ? p.omc * p.xprev[row * KT + j] : 0.0f;
    float s = 0.0f;
    // every lane runs the same trip count (the shuffles below need all 64)
    for (int64_t base = e0; base < e1; base += SUBS) {
        const int64_t e = base + sub;
        const bool ok = e < e1;
        const int32_t v = ok ? p.col[e] : 0;
        const float l = ok ? p.lam_in[(int64_t)v * KT + j] : 0.0f;
        if (WITHG) {
            float d = xr * l;
#pragma unroll
            for (int off = 1; off < KT; off <<= 1) d += __shfl_xor(d, off, 64);
            if (ok && j == 0) p.G[e] += d;
        }
        if (ok) s += WEIGHTED ? p.w[e] * l : l;
    }
#pragma unroll
    for (int off = KT; off < 64; off <<= 1) s += __shfl_xor(s, off, 64);
    return s;
}

// One short row by one sub-group of KT lanes (lane j = column j): its edges
// in order, 4 gathers of lambda(i) rows in flight; each edge's gradient term
// is reduced over the sub-group's lanes alone (xor offsets below KT, all in
// the sub-group, which runs the row's trip count as a whole).
constexpr int kShortRowAdjKt = 32;  // rows up to this many edges take one sub-group

template <int KT, bool WEIGHTED, bool WITHG>
__device__ __forceinline__ float adj_row_kt(const AdjParams &p, int64_t row, int64_t e0, int64_t e1, int j) {
    constexpr int UNR = 4;
    const float xr = WITHG ? p.omc * p.xprev[row * KT + j] : 0.0f;
    float s = 0.0f;
    for (int64_t base = e0; base < e1; base += UNR) {
        int32_t v[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) v[k] = base + k < e1 ? p.col[base + k] : -1;
        float l[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) l[k] = v[k] >= 0 ? p.lam_in[(int64_t)v[k] * KT + j] : 0.0f;
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            if (WITHG) {
                float d = xr * l[k];
#pragma unroll
                for (int off = 1; off < KT; off <<= 1) d += __shfl_xor(d, off, 64);
                if (v[k] >= 0 && j == 0) p.G[base + k] += d;
            }
            if (v[k] >= 0) s += WEIGHTED ? p.w[base + k] * l[k] : l[k];
        }
    }
    return s;
}

template <int KT, bool WEIGHTED, bool WITHG>
__global__ __launch_bounds__(kThreads) void adj_kernel_kt(const Item *__restrict__ items, int64_t n_items,
                                                          AdjParams p) {
    constexpr int SUBS = 64 / KT;
    const int lane = threadIdx.x & 63;
    const int j = lane % KT, sub = lane / KT;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (wid >= n_items) return;
    const Item it = items[wid];
    const int kind = (int)item_kind(it.meta);
    const int nnz = (int)item_nnz(it.meta);
    if (kind == (int)kItemGroup) {
        // short rows: SUBS rows at a time, one per sub-group; longer rows:
        // the whole wave, sub-groups striding over the edges.  (A row at a
        // time for the whole wave left most lanes idle on rows of a few edges
        // and serialised the rows' gathers.)
        const int nrows = (int)item_nrows(it.meta);
        const int rel = lane <= nrows ? (int)(p.rowptr[it.row0 + lane] - it.e0) : nnz;
        const int rel_next = __shfl(rel, lane + 1 < 64 ? lane + 1 : 63, 64);
        for (int rb = 0; rb < nrows; rb += SUBS) {
            const int r = min(rb + sub, 63);
            const int b = __shfl(rel, r, 64), en = __shfl(rel_next, r, 64);
            if (rb + sub < nrows && en - b <= kShortRowAdjKt) {
                const float s = adj_row_kt<KT, WEIGHTED, WITHG>(p, it.row0 + r, it.e0 + b, it.e0 + en, j);
                adj_epilogue(p, it.row0 + r, j, s);
            }
        }
        uint64_t big = __ballot(lane < nrows && rel_next - rel > kShortRowAdjKt);
        while (big) {
            const int r = __builtin_ctzll(big);
            big &= big - 1;
            const int b = __builtin_amdgcn_readlane(rel, r), en = __builtin_amdgcn_readlane(rel, r + 1);
            const int64_t row = it.row0 + r;
            const float s = adj_range_kt<KT, WEIGHTED, WITHG>(p, row, it.e0 + b, it.e0 + en, sub, j);
            if (sub == 0) adj_epilogue(p, row, j, s);
        }
        return;
    }
    const int64_t row = kind == (int)kItemRow ? (int64_t)it.row0 : (int64_t)p.longs[it.row0].row;
    const float s = adj_range_kt<KT, WEIGHTED, WITHG>(p, row, it.e0, it.e0 + nnz, sub, j);
    if (sub == 0) {
        if (kind == (int)kItemRow)
            adj_epilogue(p, row, j, s);
        else
            p.partials[wid * KT + j] = s;
    }
}

// ------------------------------------------------------------ kt == 64
// One wave per item, lane j = column j.  The item's edges are walked in
// order, 64 column ids at a time, with 16 gathers of lambda(i) rows (256 B)
// in flight.  The per-edge gradient terms sum_j (1-c) x_j(i-1)[u]
// lambda_j(i)[v] of 16 edges are reduced through a 16 x 64 LDS tile (4
// lanes per edge) and added to G with 16 neighbouring writes.  The row
// operands (x(i-1) row, node-major loss-weight row) are fetched one row
// ahead and 1/outdeg one row per lane, so a row boundary waits on nothing.
constexpr int kAdjU = 16;
constexpr int kAdjTile = 65;

template <bool WEIGHTED, bool WITHG>
__device__ __forceinline__ void adj_item_64(const AdjParams &p, const Item it, int64_t wid, int lane, float *tile) {
    const int kind = (int)item_kind(it.meta);
    const int nnz = (int)item_nnz(it.meta);
    const bool group = kind == (int)kItemGroup;
    const bool chunk = kind == (int)kItemChunk;
    const int nrows = group ? (int)item_nrows(it.meta) : 1;
    const int64_t row0 = chunk ? (int64_t)p.longs[it.row0].row : (int64_t)it.row0;
    const int rel = group ? (lane <= nrows ? (int)(p.rowptr[row0 + lane] - it.e0) : nnz) : (lane == 0 ? 0 : nnz);
    const float inv_l = (!WEIGHTED && lane < nrows) ? p.inv[row0 + lane] : 0.0f;
    const int32_t lr_l = (!chunk && lane < nrows) ? (int32_t)lam_row(p, row0 + lane) : 0;
    int r = 0;
    int rend = __builtin_amdgcn_readlane(rel, 1);
    float xr = WITHG ? p.omc * p.xprev[row0 * 64 + lane] : 0.0f;
    float gc = chunk ? 0.0f : p.gT[row0 * 64 + lane];
    float xr_n = 0.0f, g_n = 0.0f;
    if (nrows > 1) {
        if (WITHG) xr_n = p.omc * p.xprev[(row0 + 1) * 64 + lane];
        g_n = p.gT[(row0 + 1) * 64 + lane];
    }
    float acc = 0.0f;
    auto close_row = [&]() {
        if (chunk) {
            p.partials[wid * 64 + lane] = acc;
        } else {
            const float sc = WEIGHTED ? acc : acc * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(inv_l), r));
            p.lam_out[(int64_t)__builtin_amdgcn_readlane(lr_l, r) * 64 + lane] = fmaf(p.beta, gc, p.omc * sc);
        }
        acc = 0.0f;
        ++r;
        xr = xr_n;
        gc = g_n;
        if (r + 1 < nrows) {
            if (WITHG) xr_n = p.omc * p.xprev[(row0 + r + 1) * 64 + lane];
            g_n = p.gT[(row0 + r + 1) * 64 + lane];
        }
    };
    const int ek = lane >> 2, part = lane & 3;  // tile reduction: 4 lanes per edge
    for (int base = 0; base < nnz; base += 64) {
        const int cnt = min(64, nnz - base);
        const int32_t colv = lane < cnt ? p.col[it.e0 + base + lane] : 0;
        const float wv = (WEIGHTED && lane < cnt) ? p.w[it.e0 + base + lane] : 0.0f;
        for (int t0 = 0; t0 < cnt; t0 += kAdjU) {
            float l[kAdjU];
#pragma unroll
            for (int k = 0; k < kAdjU; ++k) {
                const int32_t v = __builtin_amdgcn_readlane(colv, t0 + k);
                l[k] = p.lam_in[(int64_t)v * 64 + lane];
            }
#pragma unroll
            for (int k = 0; k < kAdjU; ++k) {
                if (t0 + k < cnt) {
                    const int e = base + t0 + k;
                    while (e >= rend) {
                        close_row();
                        rend = __builtin_amdgcn_readlane(rel, r + 1);
                    }
                    const float wk =
                        WEIGHTED ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wv), t0 + k)) : 1.0f;
                    acc += WEIGHTED ? wk * l[k] : l[k];
                    if (WITHG) tile[k * kAdjTile + lane] = xr * l[k];
                }
            }
            if (WITHG) {
                wave_sync();
                float d = 0.0f;
#pragma unroll
                for (int c2 = 0; c2 < 16; ++c2) d += tile[ek * kAdjTile + part * 16 + c2];
                d += __shfl_xor(d, 1, 64);
                d += __shfl_xor(d, 2, 64);
                if (part == 0 && t0 + ek < cnt) p.G[it.e0 + base + t0 + ek] += d;
                wave_sync();
            }
        }
    }
    while (r < nrows) close_row();
}

template <bool WEIGHTED, bool WITHG>
__global__ __launch_bounds__(kThreads) void adj_kernel_64(const Item *__restrict__ items, int64_t n_items,
                                                          AdjParams p) {
    __shared__ float tile[kWaves][kAdjU * kAdjTile];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + wv;
    if (wid >= n_items) return;
    adj_item_64<WEIGHTED, WITHG>(p, items[wid], wid, lane, tile[wv]);
}

__global__ __launch_bounds__(kThreads) void adj_finish_kernel(const LongRow *__restrict__ longs, int64_t n_long,
                                                              AdjParams p) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (wid >= n_long) return;
    const LongRow lr = longs[wid];
    if (p.kt == 1) {
        float t = 0.0f;
        for (int i = lane; i < lr.nchunks; i += 64) t += p.partials[(int64_t)lr.first_item + i];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
        if (lane == 0) adj_epilogue(p, lr.row, 0, t);
    } else {
        for (int j = lane; j < p.kt; j += 64) {
            float t = 0.0f;
            for (int i = 0; i < lr.nchunks; ++i) t += p.partials[((int64_t)lr.first_item + i) * p.kt + j];
            adj_epilogue(p, lr.row, j, t);
        }
    }
}

// g_sum[v] = sum_j grad_out[j][v]
__global__ void gsum_kernel(const float *grad_out, int64_t k, int64_t n, float *gs) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int64_t j = 0; j < k; ++j) s += grad_out[j * n + v];
        gs[v] = s;
    }
}

// lambda(N) tile: lam[v][j] = beta * g(v, j), and, when p.gT is set, the
// node-major copy gT[v][j] = g(v, j).  One block per 64 nodes; for seed
// tiles the seed-major g is transposed through LDS so that both the reads
// (along v) and the writes (along j) are coalesced.
__global__ void lam_init_kernel(AdjParams p, float *lam) {
    __shared__ float tile[64][65];
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    const int kt = p.kt;
    if (kt == 1) {
        for (int i = threadIdx.x; i < 64; i += blockDim.x)
            if (v0 + i < p.n) lam[lam_row(p, v0 + i)] = p.beta * p.gvec[v0 + i];
        return;
    }
    for (int i = threadIdx.x; i < 64 * kt; i += blockDim.x) {
        const int j = i / 64, vv = i % 64;
        tile[vv][j] = (j < p.ncols && v0 + vv < p.n) ? p.gvec[(int64_t)j * p.g_stride + v0 + vv] : 0.0f;
    }
    __syncthreads();
    float *gT = const_cast<float *>(p.gT);
    for (int i = threadIdx.x; i < 64 * kt; i += blockDim.x) {
        const int vv = i / kt, j = i % kt;
        if (v0 + vv < p.n) {
            lam[lam_row(p, v0 + vv) * kt + j] = p.beta * tile[vv][j];
            if (gT) gT[(v0 + vv) * kt + j] = tile[vv][j];
        }
    }
}

// grad_q[col0 + j][v] = c * lambda(0)[v][j], transposed through LDS (one
// block per 64 nodes).
__global__ void gradq_kernel(const float *lam, const int32_t *lrow, int64_t n, int kt, int ncols, float c,
                             int64_t col0, float *gq) {
    __shared__ float tile[64][65];
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    for (int i = threadIdx.x; i < 64 * kt; i += blockDim.x) {
        const int vv = i / kt, j = i % kt;
        tile[vv][j] = v0 + vv < n ? lam[(lrow ? (int64_t)lrow[v0 + vv] : v0 + vv) * kt + j] : 0.0f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * ncols; i += blockDim.x) {
        const int j = i / 64, vv = i % 64;
        if (v0 + vv < n) gq[(col0 + j) * n + v0 + vv] = c * tile[vv][j];
    }
}

// z = x (explicit weights) or x / outdeg (uniform), at row zperm[v] of the
// gather layout when zperm is set
__global__ void scale_kernel(const float *x, const float *inv, int use_inv, int64_t n, const int32_t *zperm,
                             float *z) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        z[zperm ? zperm[v] : v] = use_inv ? x[v] * inv[v] : x[v];
}

// Row softmax backward, in place on G: waves stride over the rows of A~.
__global__ void softmax_bwd_kernel(const int64_t *rowptr, const float *w, const float *inv, int64_t n, float *G) {
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; row < n; row += nwaves) {
        const int64_t b = rowptr[row], e = rowptr[row + 1];
        const float iu = w ? 0.0f : inv[row];
        float s = 0.0f;
        for (int64_t i = b + lane; i < e; i += 64) s += (w ? w[i] : iu) * G[i];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
        for (int64_t i = b + lane; i < e; i += 64) {
            const float a = w ? w[i] : iu;
            G[i] = a * (G[i] - s);
        }
    }
}

inline unsigned grid_1d(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 20));
}
inline unsigned blocks_for(int64_t waves) { return (unsigned)((waves + kWaves - 1) / kWaves); }

template <bool WG>
void launch_adj_kt(const Schedule &s, const AdjParams &p, hipStream_t st) {
    const unsigned grid = blocks_for(s.n_items);
    const Item *it = s.items;
    const int64_t ni = s.n_items;
    const bool w = p.w != nullptr;
#define TPA_ADJ_CASE(KT)                                                                                  \
    if (w) adj_kernel_kt<KT, true, WG><<<grid, kThreads, 0, st>>>(it, ni, p);                             \
    else adj_kernel_kt<KT, false, WG><<<grid, kThreads, 0, st>>>(it, ni, p);
    switch (p.kt) {
        case 1:
            if (w) adj_kernel_1<true, WG><<<grid, kThreads, 0, st>>>(it, ni, p);
            else adj_kernel_1<false, WG><<<grid, kThreads, 0, st>>>(it, ni, p);
            break;
        case 2: TPA_ADJ_CASE(2) break;
        case 4: TPA_ADJ_CASE(4) break;
        case 8: TPA_ADJ_CASE(8) break;
        case 16: TPA_ADJ_CASE(16) break;
        case 32: TPA_ADJ_CASE(32) break;
        case 64:
            if (w) adj_kernel_64<true, WG><<<grid, kThreads, 0, st>>>(it, ni, p);
            else adj_kernel_64<false, WG><<<grid, kThreads, 0, st>>>(it, ni, p);
            break;
        default: break;
    }
#undef TPA_ADJ_CASE
}

tpa_status adj_step(const Schedule &s, const AdjParams &p0, hipStream_t st) {
    // the single-vector step reads the schedule's group-ordered ids in place
    // of A~'s own when it has them
    AdjParams p = p0;
    p.col_slots = 0;
    p.chunk_slot_in_item = s.chunk_slot_in_item ? 1 : 0;
    if (s.chunk_slot_in_item && (p.kt != 1 || p.w || !p.slot_row))
        return fail(TPA_ERR_INVALID_ARG, "an XCD-sliced adjoint schedule takes single-column steps with 1/outdeg weights");
    if (p.kt == 1 && s.colg && p.col == s.colg_src) {
        p.col = s.colg;
        p.col_slots = 1;
    }
    if ((uint64_t)blocks_for(s.n_items) * kThreads > UINT32_MAX)
        return fail(TPA_ERR_INDEX_OVERFLOW, "too many work items for one launch");
    if (s.n_items > 0) {
        int lg = 0;
        while ((1 << lg) < p.kt) ++lg;
        const int slot = profile_begin(16 * lg + 12 + (p.G ? 2 : 0) + (p.w ? 1 : 0), st);
        if (p.G) launch_adj_kt<true>(s, p, st);
        else launch_adj_kt<false>(s, p, st);
        profile_end(slot, st);
    }
    if (s.n_long > 0) adj_finish_kernel<<<blocks_for(s.n_long), kThreads, 0, st>>>(s.longs, s.n_long, p);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

// Work buffers of one tpa_backward call.  The call's i-th buffer reuses
// slot i of the handle's cache when it is large enough, and otherwise
// replaces it, while the cache stays within kAdjCacheBytes; beyond that a
// buffer is allocated for this call only.  Repeated calls of one shape
// (a training loop) then allocate nothing.  Calls on one handle must not
// overlap.
constexpr size_t kAdjCacheBytes = (size_t)8 << 30;

struct Scratch {
    tpa_graph *g;
    size_t next = 0;
    bool keep_sax = false;  // the sliced adjoint sweep is in use
    std::vector<void *> own;  // this call's uncached buffers
    explicit Scratch(tpa_graph *graph) : g(graph) {}
    ~Scratch() {
        for (void *b : own) dfree(b);
    }
    // Device memory, or, when the device is out of it, again after dropping
    // the sliced adjoint sweep (rebuilt at its next use).
    tpa_status alloc(void **p, size_t bytes, hipStream_t st) {
        tpa_status rc = dmalloc(p, bytes, st);
        if (rc == TPA_ERR_OUT_OF_MEMORY && g->sax.col && !keep_sax) {
            (void)hipStreamSynchronize(st);
            g->sax.release();
            rc = dmalloc(p, bytes, st);
        }
        return rc;
    }
    template <class T>
    tpa_status get(T **p, size_t count, hipStream_t st) {
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        auto &cache = g->adj_cache;
        const size_t slot = next++;
        if (slot < cache.size() && cache[slot].second >= bytes) {
            *p = static_cast<T *>(cache[slot].first);
            return TPA_OK;
        }
        size_t held = 0;
        for (size_t i = 0; i < cache.size(); ++i)
            if (i != slot) held += cache[i].second;
        if (held + bytes <= kAdjCacheBytes) {
            if (slot < cache.size()) {
                dfree(cache[slot].first);
                cache[slot] = {nullptr, 0};
            }
            void *b = nullptr;
            TPA_TRY(alloc(&b, bytes, st));
            if (slot < cache.size()) cache[slot] = {b, bytes};
            else cache.push_back({b, bytes});  // slot == cache.size(): slots fill in order
            *p = static_cast<T *>(b);
            return TPA_OK;
        }
        void *b = nullptr;
        TPA_TRY(alloc(&b, bytes, st));
        *p = static_cast<T *>(b);
        own.push_back(*p);
        return TPA_OK;
    }
};

}  // namespace
}  // namespace tpa

using namespace tpa;

extern "C" tpa_status tpa_backward(tpa_graph_t g, const int32_t *seeds, const float *q, int64_t k, int packed,
                                   double c, int S, int T, const float *grad_out, float *grad_logits,
                                   float *grad_q, int checkpoint_every, hipStream_t st) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (!g->preprocessed) return fail(TPA_ERR_NOT_PREPROCESSED, "tpa_preprocess has not run on this graph");
    if (!(c > 0.0 && c < 1.0) || S < 1 || T < S) return fail(TPA_ERR_INVALID_ARG, "need 0 < c < 1, S >= 1, T >= S");
    if (c != g->c || T != g->T) return fail(TPA_ERR_PARAM_MISMATCH, "(c, T) differs from the preprocessed (c, T)");
    if (k < 1) return fail(TPA_ERR_INVALID_ARG, "k must be >= 1");
    if ((seeds == nullptr) == (q == nullptr)) return fail(TPA_ERR_INVALID_ARG, "pass exactly one of seeds and q");
    if (!grad_out) return fail(TPA_ERR_INVALID_ARG, "grad_out is NULL");
    if (!grad_logits && !grad_q) return TPA_OK;
    if (packed && (!seeds || !g->node_block)) return fail(TPA_ERR_INVALID_ARG, "packed needs seeds and a packed graph");
    const int64_t n = g->n, m = g->m, K = g->K;
    // forward recomputation in the gather layout of the query path
    const bool hub = g->gather_layout && g->zperm && (!g->weighted || g->t_wz_valid);
    const float *w_gather = g->weighted ? (hub ? g->t_wz : g->t.w) : nullptr;
    const float omc = (float)(1.0 - c);
    const double pS = std::pow(1.0 - c, (double)S), pT = std::pow(1.0 - c, (double)T);
    const float alpha = (float)((1.0 - pT) / (1.0 - pS));
    Scratch sc(g);

    const Schedule *sf1 = nullptr, *sa1 = nullptr;
    SchedShape adj_shape = choose_shape(g, 1);
    adj_shape.eb = 0;  // the adjoint kernels take wave, group and chunk items
    TPA_TRY(get_schedule(g, choose_shape(g, 1), st, &sf1, false));
    TPA_TRY(get_schedule(g, adj_shape, st, &sa1, true));
    if (hub) TPA_TRY(ensure_group_order(g, sf1, st));
    // the stranger chain is recomputed as preprocessing computed it (in XCD
    // slices on large graphs), so the iterates are bitwise the kept ones
    const Schedule *sx = nullptr;
    const int32_t *colx = nullptr;
    if (hub) TPA_TRY(ensure_sliced_sweep(g, st, &sx, &colx));
    const Schedule *sfs = sx ? sx : sf1;
    // layout 2 on large unpacked graphs: lambda in rank order by in-degree
    // (built before the adjoint's group-ordered ids, which are taken from
    // a_colr then).  A packed graph keeps node order: each block's lambda is
    // a contiguous slice that its own pulls gather from, which a global rank
    // order would scatter (256 packed R-MAT graphs of 14.4M nodes in all:
    // 213 against 231 ms per adjoint).
    const bool lam_rank = g->gather_layout == 2 && g->n >= kLamRankMinN && g->nblocks == 1;
    if (lam_rank) TPA_TRY(ensure_lam_layout(g, st));
    const bool lam_hub = lam_rank && g->a_colr;
    const int32_t *a_col = lam_hub ? g->a_colr : g->a.col;
    const int32_t *lrow = lam_hub ? g->lrank : nullptr;
    TPA_TRY(ensure_group_order(g, sa1, st, true));
    // the stranger chain's adjoint steps in XCD slices on large graphs; its
    // edge gradient is then in the sliced order until the chain ends
    const SlicedAdj *sxa = nullptr;
    if (grad_logits) TPA_TRY(ensure_sliced_adj(g, a_col, st, &sxa));
    sc.keep_sax = sxa != nullptr;
    const Schedule *sas = sxa ? &sxa->s : sa1;
    // (a temporary copy of G, freed before the family chains allocate)
    auto unslice_g = [&]() -> tpa_status {
        if (!sxa) return TPA_OK;
        float *gx = nullptr;
        TPA_TRY(dalloc(&gx, (size_t)m, st));
        hipError_t e = hipMemcpyAsync(gx, grad_logits, sizeof(float) * m, hipMemcpyDeviceToDevice, st);
        tpa_status rc = e == hipSuccess ? launch_unslice(*sxa, gx, grad_logits, st) : TPA_ERR_HIP;
        if (rc == TPA_OK) e = hipStreamSynchronize(st);
        dfree(gx);
        if (rc != TPA_OK || e != hipSuccess)
            return rc != TPA_OK ? rc : fail(TPA_ERR_HIP, std::string("edge gradient order: ") + hipGetErrorString(e));
        sxa = nullptr;  // the sliced sweep may be dropped from here on (see Scratch::alloc)
        sc.keep_sax = false;
        return TPA_OK;
    };

    if (grad_logits && checkpoint_every == 0 && g->xiter_K == K && g->xiter) {
        TPA_TRY_HIP(hipMemsetAsync(grad_logits, 0, sizeof(float) * m, st));
        // ---- stranger chain from the iterates kept by tpa_preprocess ----
        float *gs, *lam0, *lam1, *part_a;
        TPA_TRY(sc.get(&gs, n, st));
        TPA_TRY(sc.get(&lam0, n, st));
        TPA_TRY(sc.get(&lam1, n, st));
        TPA_TRY(sc.get(&part_a, sas->n_chunk_items, st));
        gsum_kernel<<<grid_1d(n), 256, 0, st>>>(grad_out, k, n, gs);
        AdjParams ap;
        ap.rowptr = g->a.rowptr;
        ap.col = sxa ? sxa->col : a_col;
        ap.slot_row = sxa ? sxa->slot_row : nullptr;
        ap.lrow = lrow;
        ap.w = g->weighted ? g->a.w : nullptr;
        ap.inv = g->inv_deg;
        ap.longs = sas->longs;
        ap.G = grad_logits;
        ap.gvec = gs;
        ap.omc = omc;
        ap.kt = 1;
        ap.ncols = 1;
        ap.n = n;
        ap.partials = part_a;
        ap.beta = (K >= T) ? 1.0f : 0.0f;
        lam_init_kernel<<<(unsigned)((n + 63) / 64), 256, 0, st>>>(ap, lam0);
        float *lc = lam0, *ln = lam1;
        for (int64_t i = K; i >= 1; --i) {
            ap.xprev = g->xiter + (size_t)(i - 1) * n;
            ap.lam_in = lc;
            ap.lam_out = ln;
            ap.beta = (i - 1 >= T) ? 1.0f : 0.0f;
            TPA_TRY(adj_step(*sas, ap, st));
            std::swap(lc, ln);
        }
        TPA_TRY(unslice_g());
    } else if (grad_logits) {
        TPA_TRY_HIP(hipMemsetAsync(grad_logits, 0, sizeof(float) * m, st));
        // ---- stranger chain, checkpointed ----
        int64_t C = checkpoint_every;
        if (C == 0) {
            // automatic: keep every iterate (no recomputation) when they take at
            // most a third of the free device memory, else every ceil(sqrt(K))
            size_t free_b = 0, total_b = 0;
            const bool fits = hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
                              (double)(K + 1) * (double)n * sizeof(float) <= (double)free_b / 3.0;
            C = fits ? K : std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt((double)K)));
        }
        if (C < 0 || C > K) C = K;
        const int64_t nck = (K + C - 1) / C;
        float *gs, *ck, *seg, *z0, *z1, *lam0, *lam1, *comp, *part_f, *part_a;
        TPA_TRY(sc.get(&gs, n, st));
        TPA_TRY(sc.get(&ck, (size_t)nck * n, st));
        TPA_TRY(sc.get(&seg, (size_t)C * n, st));
        TPA_TRY(sc.get(&z0, n, st));
        TPA_TRY(sc.get(&z1, n, st));
        TPA_TRY(sc.get(&lam0, n, st));
        TPA_TRY(sc.get(&lam1, n, st));
        TPA_TRY(sc.get(&comp, n, st));
        TPA_TRY(sc.get(&part_f, sfs->n_chunk_items, st));
        TPA_TRY(sc.get(&part_a, sas->n_chunk_items, st));
        gsum_kernel<<<grid_1d(n), 256, 0, st>>>(grad_out, k, n, gs);
        // forward pass: checkpoints x'(0), x'(C), ...
        StepParams fp;
        fp.zperm = hub ? g->zperm : nullptr;
        TPA_TRY(launch_stranger_init(g, (float)c, 1, z0, ck, comp, fp.zperm, st));
        fp.rowptr = g->t.rowptr;
        fp.col = colx ? colx : hub ? g->t_colz : g->t.col;
        fp.w = w_gather;
        fp.inv = g->inv_deg;
        fp.partials = part_f;
        fp.omc = omc;
        fp.c = (float)c;
        fp.kt = 1;
        fp.ncols = 1;
        fp.n = n;
        float *zc = z0, *zn = z1;
        for (int64_t i = 1; i < (nck - 1) * C + 1 && i < K; ++i) {
            fp.zin = zc;
            fp.zout = zn;
            fp.xs_out = (i % C == 0) ? ck + (size_t)(i / C) * n : nullptr;
            TPA_TRY(launch_step(*sfs, kPlain, false, fp, st));
            std::swap(zc, zn);
        }
        // backward over segments
        AdjParams ap;
        ap.rowptr = g->a.rowptr;
        ap.col = sxa ? sxa->col : a_col;
        ap.slot_row = sxa ? sxa->slot_row : nullptr;
        ap.lrow = lrow;
        ap.w = g->weighted ? g->a.w : nullptr;
        ap.inv = g->inv_deg;
        ap.longs = sas->longs;
        ap.G = grad_logits;
        ap.gvec = gs;
        ap.omc = omc;
        ap.kt = 1;
        ap.ncols = 1;
        ap.n = n;
        ap.partials = part_a;
        ap.beta = (K >= T) ? 1.0f : 0.0f;
        lam_init_kernel<<<(unsigned)((n + 63) / 64), 256, 0, st>>>(ap, lam0);
        float *lc = lam0, *ln = lam1;
        for (int64_t sgi = nck - 1; sgi >= 0; --sgi) {
            const int64_t lo = sgi * C, hi = std::min<int64_t>(lo + C, K);
            // recompute x'(lo+1 .. hi-1) into seg[1..]; seg slot 0 is the checkpoint
            float *x_lo = ck + (size_t)sgi * n;
            if (hi - lo > 1) {
                scale_kernel<<<grid_1d(n), 256, 0, st>>>(x_lo, g->inv_deg, g->weighted ? 0 : 1, n, fp.zperm, z0);
                float *a = z0, *b = z1;
                for (int64_t i = lo + 1; i < hi; ++i) {
                    fp.zin = a;
                    fp.zout = b;
                    fp.xs_out = seg + (size_t)(i - lo) * n;
                    TPA_TRY(launch_step(*sfs, kPlain, false, fp, st));
                    std::swap(a, b);
                }
            }
            for (int64_t i = hi; i > lo; --i) {
                ap.xprev = (i - 1 == lo) ? x_lo : seg + (size_t)(i - 1 - lo) * n;
                ap.lam_in = lc;
                ap.lam_out = ln;
                ap.beta = (i - 1 >= T) ? 1.0f : 0.0f;
                TPA_TRY(adj_step(*sas, ap, st));
                std::swap(lc, ln);
            }
        }
        TPA_TRY(unslice_g());
    }

    // ---- family chains per seed tile ----
    const int kt = choose_kt(g, k);
    const Schedule *sfk = nullptr, *sak = nullptr;
    SchedShape adj_shape_k = choose_shape(g, kt);
    adj_shape_k.eb = 0;
    TPA_TRY(get_schedule(g, choose_shape(g, kt), st, &sfk, false));
    TPA_TRY(get_schedule(g, adj_shape_k, st, &sak, true));
    const int nit = std::max(S - 1, 1);  // stored iterates x(0..S-2)
    float *xf, *z0, *z1, *lam0, *lam1, *part_f, *part_a, *gT = nullptr;
    TPA_TRY(sc.get(&xf, (size_t)nit * n * kt, st));
    if (kt == 64) TPA_TRY(sc.get(&gT, (size_t)n * kt, st));
    TPA_TRY(sc.get(&z0, (size_t)n * kt, st));
    TPA_TRY(sc.get(&z1, (size_t)n * kt, st));
    TPA_TRY(sc.get(&lam0, (size_t)n * kt, st));
    TPA_TRY(sc.get(&lam1, (size_t)n * kt, st));
    TPA_TRY(sc.get(&part_f, (size_t)sfk->n_chunk_items * kt, st));
    TPA_TRY(sc.get(&part_a, (size_t)sak->n_chunk_items * kt, st));
    StepParams fp;
    fp.rowptr = g->t.rowptr;
    fp.zperm = hub ? g->zperm : nullptr;
    fp.w = g->weighted ? g->t.w : nullptr;
    fp.inv = g->inv_deg;
    fp.partials = part_f;
    fp.omc = omc;
    fp.c = (float)c;
    fp.kt = kt;
    fp.n = n;
    fp.node_block = packed ? g->node_block : nullptr;
    fp.seed_stride = packed ? (int)k : 0;
    AdjParams ap;
    ap.rowptr = g->a.rowptr;
    ap.col = a_col;
    ap.lrow = lrow;
    ap.w = g->weighted ? g->a.w : nullptr;
    ap.inv = g->inv_deg;
    ap.longs = sak->longs;
    ap.G = grad_logits;
    ap.g_stride = n;
    ap.gT = gT;
    ap.omc = omc;
    ap.kt = kt;
    ap.n = n;
    ap.partials = part_a;
    for (int64_t base = 0; base < k; base += kt) {
        const int ncols = (int)std::min<int64_t>(kt, k - base);
        fp.seeds = seeds ? seeds + base : nullptr;
        fp.qdense = q ? q + base * n : nullptr;
        fp.ncols = ncols;
        // x(0) and the scaled vector for step 1
        if (q) {
            TPA_TRY(launch_dense_init(fp, z0, xf, st));
        } else {
            TPA_TRY(launch_onehot_init(fp, xf, st));
        }
        float *zc = z0, *zn = z1;
        for (int i = 1; i <= S - 2; ++i) {
            fp.zin = zc;
            fp.zout = zn;
            fp.xs_out = xf + (size_t)i * n * kt;
            const bool first = i == 1 && !q;  // first steps read node ids and A~^T's own weight order
            fp.col = first ? g->t.col : (hub ? g->t_colz : g->t.col);
            fp.w = first ? (g->weighted ? g->t.w : nullptr) : w_gather;
            TPA_TRY(launch_step(*sfk, kPlain, i == 1 && !q, fp, st));
            std::swap(zc, zn);
        }
        ap.gvec = grad_out + base * n;
        ap.ncols = ncols;
        ap.beta = alpha;
        lam_init_kernel<<<(unsigned)((n + 63) / 64), 256, 0, st>>>(ap, lam0);
        float *lc = lam0, *ln = lam1;
        for (int i = S - 1; i >= 1; --i) {
            ap.xprev = grad_logits ? xf + (size_t)(i - 1) * n * kt : nullptr;
            ap.G = grad_logits;
            ap.lam_in = lc;
            ap.lam_out = ln;
            ap.beta = alpha;
            TPA_TRY(adj_step(*sak, ap, st));
            std::swap(lc, ln);
        }
        if (grad_q)
            gradq_kernel<<<(unsigned)((n + 63) / 64), 256, 0, st>>>(lc, lrow, n, kt, ncols, (float)c, base, grad_q);
    }
    if (grad_logits) {
        const unsigned sgrid = (unsigned)std::min<int64_t>((n * 64 + 255) / 256, 1 << 20);
        softmax_bwd_kernel<<<sgrid, 256, 0, st>>>(g->a.rowptr, g->weighted ? g->a.w : nullptr, g->inv_deg, n,
                                                  grad_logits);
    }
    TPA_TRY_HIP(hipGetLastError());
    TPA_TRY_HIP(hipStreamSynchronize(st));  // scratch buffers are freed on return
    return TPA_OK;
}
