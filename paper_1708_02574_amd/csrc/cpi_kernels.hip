// CPI step kernels for gfx950.
//
// One CPI step (Section 2.3, Algorithm 1) is x(i) = (1-c) A~^T x(i-1): a
// pull over the rows of A~^T, i.e. an irregular gather with about 2 flops
// per 8 bytes.  It is bound by HBM (and by the gather's cache behaviour),
// not by arithmetic, so there is no matrix-core work here; what matters is
// coalesced index streams, enough loads in flight, and balance across
// power-law rows.
//
// Work decomposition (built once per graph, see get_schedule): one wave
// (64 lanes) per work item; four independent waves per 256-thread block.
//   * short-row group (<= 64 rows, < 2*EW edges): the item's edges are read
//     64 at a time, one per lane (coalesced index loads); each lane finds its
//     row by a binary search over the row starts held across the wave, a
//     segmented wave scan adds up each row's part of the strip, and the lane
//     owning the row picks its total -- no LDS, no atomics;
//   * whole row (EW..EL edges): one wave, lanes stride over the edges;
//   * chunk of a long row (> EL edges): as above into a partial slot; a
//     finish pass adds a row's chunk sums in chunk order.
// All sums are in a fixed order, so results are bitwise reproducible.
//
// Seed tiles (kt > 1 columns, node-major [n][kt] vectors): lanes are split
// into 64/kt sub-groups of kt lanes; lane (sub, j) adds column j over every
// (64/kt)-th edge of a row, so each gathered row segment of kt floats is one
// contiguous access; sub-groups are then combined by xor shuffles.

#include <cmath>

#include "cpi_kernels.h"

namespace tpa {
namespace {

constexpr int kWaves = 4;          // waves (items) per block
constexpr int kThreads = 64 * kWaves;

__device__ __forceinline__ int32_t seed_of(const StepParams &p, int64_t v, int j) {
    if (j >= p.ncols) return -1;
    const int64_t b = p.node_block ? (int64_t)p.node_block[v] * p.seed_stride : 0;
    return p.seeds[b + j];
}

// Epilogue for row v, column j, with pulled sum `sum`.
template <int MODE>
__device__ __forceinline__ void epilogue(const StepParams &p, int64_t v, int j, float sum) {
    if (MODE == kFamily) {
        if (j >= p.ncols) return;
        const int32_t seed = seed_of(p, v, j);
        const float y = fmaf(p.omc, sum, (v == (int64_t)seed) ? p.c : 0.0f);
        if (p.last) {
            const float o = (seed == -2) ? __int_as_float(0x7fc00000) : fmaf(p.alpha, y, p.str[v]);
            p.out[(p.out_col0 + j) * p.n + v] = o;
        } else {
            p.zout[v * p.kt + j] = p.w ? y : y * p.inv[v];
        }
    } else {
        const float x = p.omc * sum;
        p.zout[v] = p.w ? x : x * p.inv[v];
        if (p.accumulate) {
            // Kahan-compensated r~_stranger += x
            const float a = p.acc[v];
            const float yk = x - p.comp[v];
            const float t = a + yk;
            p.comp[v] = (t - a) - yk;
            p.acc[v] = t;
        }
    }
}

// Value contributed by edge e (source u) to column j of a row whose seed is
// `seed` (only used on the first family step, where x(0) = c e_seed).
template <bool FIRST>
__device__ __forceinline__ float edge_value(const StepParams &p, int64_t e, int32_t u, int j,
                                            int32_t seed) {
    if (FIRST) {
        if (u != seed) return 0.0f;
        return p.c * (p.w ? p.w[e] : p.inv[u]);
    }
    const float z = p.zin[(int64_t)u * p.kt + j];
    return p.w ? p.w[e] * z : z;
}

// ------------------------------------------------------------ kt == 1
template <int MODE, bool FIRST>
__device__ void short_group_1(const StepParams &p, const Item it, int lane) {
    constexpr int UNR = 4;
    const int r0 = it.row0, nrows = it.row1 - it.row0;
    const int64_t e0 = p.rowptr[r0];
    const int nnz = (int)(p.rowptr[it.row1] - e0);
    const int lr = lane < nrows ? lane : nrows;
    const int rel_start = (int)(p.rowptr[r0 + lr] - e0);
    const int rel_end = lane < nrows ? (int)(p.rowptr[r0 + lane + 1] - e0) : rel_start;
    const bool packed = p.node_block != nullptr;
    int32_t seed_uniform = -1;
    if (MODE == kFamily && FIRST && !packed) seed_uniform = p.seeds[0];
    float acc = 0.0f;
    for (int base = 0; base < nnz; base += 64 * UNR) {
        int32_t u[UNR];
#pragma unroll
        for (int s = 0; s < UNR; ++s) {
            const int e = base + s * 64 + lane;
            u[s] = (e < nnz) ? p.col[e0 + e] : -1;
        }
        float val[UNR];
        if (!FIRST) {
#pragma unroll
            for (int s = 0; s < UNR; ++s) {
                const int e = base + s * 64 + lane;
                val[s] = (u[s] >= 0) ? edge_value<false>(p, e0 + e, u[s], 0, -1) : 0.0f;
            }
        }
#pragma unroll
        for (int s = 0; s < UNR; ++s) {
            const int sb = base + s * 64;
            if (sb >= nnz) break;
            const int e = sb + lane;
            // row of edge e: largest row j with start_j <= e
            int lo = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const int mid = lo + step;
                const int sm = __shfl(rel_start, mid, 64);
                if (mid < nrows && sm <= e) lo = mid;
            }
            float v;
            if (FIRST) {
                int32_t seed = seed_uniform;
                if (packed) seed = seed_of(p, r0 + lo, 0);
                v = (u[s] >= 0) ? edge_value<true>(p, e0 + e, u[s], 0, seed) : 0.0f;
            } else {
                v = val[s];
            }
            // segmented inclusive scan over the strip (rows are contiguous)
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const float t = __shfl_up(v, d, 64);
                const int rr = __shfl_up(lo, d, 64);
                if (lane >= d && rr == lo) v += t;
            }
            // the lane owning a row picks the scan value at its last edge in the strip
            const int send = min(sb + 64, nnz);
            const bool hit = lane < nrows && rel_end > rel_start && rel_start < send && rel_end > sb;
            const int tail = min(rel_end, send) - 1 - sb;
            const float got = __shfl(v, hit ? tail : 0, 64);
            if (hit) acc += got;
        }
    }
    if (lane < nrows) epilogue<MODE>(p, r0 + lane, 0, acc);
}

template <int MODE, bool FIRST>
__device__ void single_row_1(const StepParams &p, const Item it, int lane, int el) {
    constexpr int UNR = 8;
    const int64_t row = it.row0;
    int64_t e0 = p.rowptr[row], e1 = p.rowptr[row + 1];
    if (it.chunk >= 0) {
        e0 += (int64_t)it.chunk * el;
        e1 = min(e1, e0 + (int64_t)el);
    }
    int32_t seed = -1;
    if (MODE == kFamily && FIRST) seed = seed_of(p, row, 0);
    float s = 0.0f;
    for (int64_t base = e0; base < e1; base += 64 * UNR) {
        int32_t u[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const int64_t e = base + k * 64 + lane;
            u[k] = (e < e1) ? p.col[e] : -1;
        }
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const int64_t e = base + k * 64 + lane;
            if (u[k] >= 0) s += edge_value<FIRST>(p, e, u[k], 0, seed);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        if (it.chunk >= 0)
            p.partials[it.slot] = s;
        else
            epilogue<MODE>(p, row, 0, s);
    }
}

template <int MODE, bool FIRST>
__global__ __launch_bounds__(kThreads) void step_kernel_1(const Item *items, int64_t n_items, int el,
                                                          StepParams p) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (wid >= n_items) return;
    const Item it = items[wid];
    if (it.chunk == -1)
        short_group_1<MODE, FIRST>(p, it, lane);
    else
        single_row_1<MODE, FIRST>(p, it, lane, el);
}

// ------------------------------------------------------------ kt > 1
template <int KT, int MODE, bool FIRST>
__device__ __forceinline__ float row_range_sum(const StepParams &p, int64_t e0, int64_t e1, int sub,
                                               int j, int32_t seed) {
    constexpr int SUBS = 64 / KT;
    constexpr int UNR = 4;
    float s = 0.0f;
    for (int64_t base = e0 + sub; base < e1; base += SUBS * UNR) {
        int32_t u[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const int64_t e = base + k * SUBS;
            u[k] = (e < e1) ? p.col[e] : -1;
        }
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const int64_t e = base + k * SUBS;
            if (u[k] >= 0) s += edge_value<FIRST>(p, e, u[k], j, seed);
        }
    }
#pragma unroll
    for (int off = KT; off < 64; off <<= 1) s += __shfl_xor(s, off, 64);
    return s;
}

template <int KT, int MODE, bool FIRST>
__global__ __launch_bounds__(kThreads) void step_kernel_kt(const Item *items, int64_t n_items, int el,
                                                           StepParams p) {
    const int lane = threadIdx.x & 63;
    const int j = lane % KT, sub = lane / KT;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (wid >= n_items) return;
    const Item it = items[wid];
    const bool packed = p.node_block != nullptr;
    int32_t seed = -1;
    if (MODE == kFamily && !packed) seed = j < p.ncols ? p.seeds[j] : -1;
    if (it.chunk == -1) {
        for (int64_t r = it.row0; r < it.row1; ++r) {
            if (MODE == kFamily && packed) seed = seed_of(p, r, j);
            const float s = row_range_sum<KT, MODE, FIRST>(p, p.rowptr[r], p.rowptr[r + 1], sub, j, seed);
            if (sub == 0) epilogue<MODE>(p, r, j, s);
        }
    } else {
        const int64_t row = it.row0;
        int64_t e0 = p.rowptr[row], e1 = p.rowptr[row + 1];
        if (it.chunk >= 0) {
            e0 += (int64_t)it.chunk * el;
            e1 = min(e1, e0 + (int64_t)el);
        }
        if (MODE == kFamily && packed) seed = seed_of(p, row, j);
        const float s = row_range_sum<KT, MODE, FIRST>(p, e0, e1, sub, j, seed);
        if (sub == 0) {
            if (it.chunk >= 0)
                p.partials[(int64_t)it.slot * KT + j] = s;
            else
                epilogue<MODE>(p, row, j, s);
        }
    }
}

// Finish pass: add the chunk sums of each long row in chunk order.
template <int MODE>
__global__ __launch_bounds__(kThreads) void finish_kernel(const LongRow *longs, int64_t n_long, StepParams p) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (wid >= n_long) return;
    const LongRow lr = longs[wid];
    const int kt = p.kt;
    if (kt == 1) {
        float s = 0.0f;
        for (int i = lane; i < lr.nchunks; i += 64) s += p.partials[(int64_t)lr.slot0 + i];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) epilogue<MODE>(p, lr.row, 0, s);
    } else {
        for (int j = lane; j < kt; j += 64) {
            float s = 0.0f;
            for (int i = 0; i < lr.nchunks; ++i) s += p.partials[((int64_t)lr.slot0 + i) * kt + j];
            epilogue<MODE>(p, lr.row, j, s);
        }
    }
}

__global__ void stranger_init_kernel(int64_t n, float c, const float *restart_pr, float inv_n,
                                     const float *inv, const float *w_present, int include_x0,
                                     float *zout, float *acc, float *comp) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const float x0 = c * (restart_pr ? restart_pr[v] : inv_n);
        zout[v] = w_present ? x0 : x0 * inv[v];
        acc[v] = include_x0 ? x0 : 0.0f;
        comp[v] = 0.0f;
    }
}

__global__ void combine_only_kernel(StepParams p) {
    const int64_t total = p.n * (int64_t)p.ncols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(i / p.n);
        const int64_t v = i - (int64_t)j * p.n;
        const int32_t seed = seed_of(p, v, j);
        const float y = (v == (int64_t)seed) ? p.c : 0.0f;
        p.out[(p.out_col0 + j) * p.n + v] =
            (seed == -2) ? __int_as_float(0x7fc00000) : fmaf(p.alpha, y, p.str[v]);
    }
}

__global__ void check_seeds_kernel(const int32_t *seeds, int64_t k, int per_block, int64_t n,
                                   const int32_t *node_block, int32_t *dst, int32_t *err) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = seeds[i];
        bool ok = s >= 0 && (int64_t)s < n;
        if (ok && node_block) ok = (int64_t)node_block[s] == i / per_block;
        dst[i] = ok ? s : -2;
        if (!ok) *err = 1;
    }
}

inline unsigned blocks_for(int64_t waves) { return (unsigned)((waves + kWaves - 1) / kWaves); }

inline unsigned grid_1d(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 20));
}

template <int MODE, bool FIRST>
void launch_kt(const Schedule &s, const StepParams &p, hipStream_t st) {
    const unsigned grid = blocks_for(s.n_items);
    switch (p.kt) {
        case 1: step_kernel_1<MODE, FIRST><<<grid, kThreads, 0, st>>>(s.items, s.n_items, s.el, p); break;
        case 2: step_kernel_kt<2, MODE, FIRST><<<grid, kThreads, 0, st>>>(s.items, s.n_items, s.el, p); break;
        case 4: step_kernel_kt<4, MODE, FIRST><<<grid, kThreads, 0, st>>>(s.items, s.n_items, s.el, p); break;
        case 8: step_kernel_kt<8, MODE, FIRST><<<grid, kThreads, 0, st>>>(s.items, s.n_items, s.el, p); break;
        case 16: step_kernel_kt<16, MODE, FIRST><<<grid, kThreads, 0, st>>>(s.items, s.n_items, s.el, p); break;
        case 32: step_kernel_kt<32, MODE, FIRST><<<grid, kThreads, 0, st>>>(s.items, s.n_items, s.el, p); break;
        case 64: step_kernel_kt<64, MODE, FIRST><<<grid, kThreads, 0, st>>>(s.items, s.n_items, s.el, p); break;
        default: break;
    }
}

}  // namespace

tpa_status launch_step(const Schedule &s, int mode, bool first, const StepParams &p, hipStream_t st) {
    if (p.kt != 1 && p.kt != 2 && p.kt != 4 && p.kt != 8 && p.kt != 16 && p.kt != 32 && p.kt != 64)
        return fail(TPA_ERR_INVALID_ARG, "seed tile must be 1, 2, 4, 8, 16, 32 or 64");
    if (mode == kStranger && p.kt != 1) return fail(TPA_ERR_INVALID_ARG, "stranger step is single-column");
    if (s.n_items > 0) {
        if (mode == kFamily) {
            if (first) launch_kt<kFamily, true>(s, p, st);
            else launch_kt<kFamily, false>(s, p, st);
        } else {
            launch_kt<kStranger, false>(s, p, st);
        }
    }
    if (s.n_long > 0) {
        if (mode == kFamily)
            finish_kernel<kFamily><<<blocks_for(s.n_long), kThreads, 0, st>>>(s.longs, s.n_long, p);
        else
            finish_kernel<kStranger><<<blocks_for(s.n_long), kThreads, 0, st>>>(s.longs, s.n_long, p);
    }
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_stranger_init(const tpa_graph *g, float c, int include_x0, float *zout, float *acc,
                                float *comp, hipStream_t st) {
    stranger_init_kernel<<<grid_1d(g->n), 256, 0, st>>>(g->n, c, g->restart_pr, (float)(1.0 / (double)g->n),
                                                         g->inv_deg, g->t.w, include_x0, zout, acc, comp);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_combine_only(const StepParams &p, hipStream_t st) {
    combine_only_kernel<<<grid_1d(p.n * (int64_t)p.ncols), 256, 0, st>>>(p);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_check_seeds(const int32_t *seeds, int64_t k, int per_block, const tpa_graph *g,
                              int32_t *dst, hipStream_t st) {
    check_seeds_kernel<<<grid_1d(k), 256, 0, st>>>(seeds, k, per_block > 0 ? per_block : 1, g->n,
                                                   per_block > 0 ? g->node_block : nullptr, dst, g->dev_err);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

}  // namespace tpa
