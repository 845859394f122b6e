// CPI step kernels for gfx950.
//
// One CPI step (Section 2.3, Algorithm 1) is x(i) = (1-c) A~^T x(i-1): a
// pull over the rows of A~^T, an irregular gather with about 2 flops per
// 8 bytes.  It is bound by memory (HBM and the gather's cache behaviour),
// not arithmetic, so there is no matrix-core work here; what matters is
// coalesced index streams, many loads in flight per wave, and balance
// across power-law rows.
//
// Work decomposition (built once per graph, get_schedule): one wave (64
// lanes) per work item, four independent waves per 256-thread block.
//
// Single vector (kt == 1):
//   * group item (<= 63 rows, <= EW edges): the item's edges are read one
//     per lane, 64 at a time, all strips issued before the first use
//     (coalesced index loads, then the gathers); the products go to the
//     wave's LDS slice; lane r then adds up row r's slice when the row has
//     <= 32 edges, and the whole wave adds up each longer row;
//   * row item: lanes stride over one row's edges, then a xor butterfly;
//   * chunk item (rows longer than EL): as a row item into a partial slot;
//     a finish pass (second launch, only when such rows exist) adds each
//     long row's partials in chunk order and applies the epilogue.
// Seed tile of 64 (kt == 64, one column per lane): the wave walks its
//   item's edges in order with wave-uniform control; column ids are loaded
//   64 at a time and broadcast with readlane, and 32 row gathers of 256 B
//   (one per edge, contiguous across the lanes) are in flight at once.
// Seed tiles of 2..32 (generic): lanes (sub, j) form 64/kt sub-groups of kt
//   lanes (lane j = column j).  Each sub-group sums one short row of a group
//   item, edges in order with 4 gathers in flight; rows longer than 32
//   edges, and row or chunk items, are summed by the whole wave, sub-groups
//   striding over the edges, and xor shuffles combine.
// Every sum is taken in a fixed order: results are bitwise reproducible.

#include <cmath>

#include "cpi_kernels.h"
#include "profile.h"

namespace tpa {
namespace {

constexpr int kWaves = 4;          // waves (items) per block
constexpr int kThreads = 64 * kWaves;
constexpr int kGroupMax = kGroupEdges;  // max edges of a group item (LDS floats per wave)

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float qnan() { return __int_as_float(0x7fc00000); }

// Seed of column j for the block of node v (plain graphs: one block).
__device__ __forceinline__ int32_t seed_of(const StepParams &p, int64_t v, int j) {
    if (j >= p.ncols) return -1;
    const int64_t b = p.node_block ? (int64_t)p.node_block[v] * p.seed_stride : 0;
    return p.seeds[b + j];
}

__device__ __forceinline__ bool seed_valid(const StepParams &p, int64_t v, int32_t s) {
    if (s < 0 || (int64_t)s >= p.n) return false;
    return p.node_block ? p.node_block[s] == p.node_block[v] : true;
}

// Per-row operands of the epilogue, loadable ahead of the sum:
//   family   a = r~_stranger[v] (last step) or 1/outdeg(v)
//   stranger a = 1/outdeg(v), b = r~_stranger[v], c = Kahan compensation
struct EpiPre {
    float a = 0.f, b = 0.f, c = 0.f;
    int32_t zi = 0;  // row of v in zout
};

// Row of node v in the work vectors.
__device__ __forceinline__ int64_t zrow(const StepParams &p, int64_t v) { return p.zperm ? p.zperm[v] : v; }

// Frontier skip in force for this launch (see StepParams::bits).
__device__ __forceinline__ bool frontier_on(const StepParams &p) { return p.bits && (!p.bits_on || *p.bits_on); }

// Row u of the gathered vector may be non-zero.
__device__ __forceinline__ bool row_live(const StepParams &p, int32_t u) {
    return (p.bits[(uint32_t)u >> 5] >> ((uint32_t)u & 31u)) & 1u;
}

template <int MODE>
__device__ __forceinline__ EpiPre epi_load(const StepParams &p, int64_t v) {
    EpiPre q;
    if (!(MODE == kFamily && p.last)) q.zi = (int32_t)zrow(p, v);
    if (MODE == kFamily) {
        if (p.last) q.a = p.str[v];
        else if (!p.w) q.a = p.inv[v];
    } else if (MODE == kPlain) {
        if (!p.w) q.a = p.inv[v];
    } else {
        if (!p.w) q.a = p.inv[v];
        if (p.accumulate) {
            q.b = p.acc[v];
            q.c = p.comp[v];
        }
    }
    return q;
}

__device__ __forceinline__ EpiPre epi_readlane(const EpiPre &q, int r) {
    EpiPre o;
    o.a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.a), r));
    o.b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.b), r));
    o.c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q.c), r));
    o.zi = __builtin_amdgcn_readlane(q.zi, r);
    return o;
}

// Column j's seed when the caller loaded it ahead (plain seed lists), or
// kSeedLookup to read it per row (packed graphs, dense restarts).
constexpr int32_t kSeedLookup = INT32_MIN;

__device__ __forceinline__ int32_t seed_ahead(const StepParams &p, int j) {
    if (p.node_block || p.qdense) return kSeedLookup;
    return j < p.ncols ? p.seeds[j] : -1;
}

// Epilogue for row v, column j, with pulled sum `sum` and operands q.
template <int MODE>
__device__ __forceinline__ void epi_store(const StepParams &p, int64_t v, int j, float sum, const EpiPre &q,
                                          int32_t seed_pre = kSeedLookup) {
    if (MODE == kFamily) {
        if (j >= p.ncols) return;
        int32_t seed = -1;
        float restart;
        if (p.qdense) {
            restart = p.qT[v * p.kt + j];
        } else {
            seed = seed_pre != kSeedLookup ? seed_pre : seed_of(p, v, j);
            restart = (v == (int64_t)seed) ? p.c : 0.0f;
        }
        const float y = fmaf(p.omc, sum, restart);
        if (p.last) {
            float o;
            if (p.qdense || seed_valid(p, v, seed)) {
                o = fmaf(p.alpha, y, q.a);
            } else {
                o = qnan();
                *p.err = 1;
            }
            p.out[(p.out_col0 + j) * p.n + v] = o;
        } else {
            p.zout[(int64_t)q.zi * p.kt + j] = p.w ? y : y * q.a;
        }
    } else if (MODE == kPlain) {
        const float x = p.omc * sum;
        if (p.xs_out) p.xs_out[v * p.kt + j] = x;
        if (p.tacc && p.iter >= p.s_iter && p.iter <= p.klast[j]) {
            // Kahan-compensated window sum of column j
            const int64_t i = v * p.kt + j;
            const float b = p.tacc[i], yk = x - p.tcomp[i];
            const float t = b + yk;
            p.tcomp[i] = (t - b) - yk;
            p.tacc[i] = t;
        }
        p.zout[(int64_t)q.zi * p.kt + j] = p.w ? x : x * q.a;
    } else {
        const float x = p.omc * sum;
        p.zout[q.zi] = p.w ? x : x * q.a;
        if (p.xs_out) p.xs_out[v] = x;
        if (p.accumulate) {
            // Kahan-compensated r~_stranger += x
            const float yk = x - q.c;
            const float t = q.b + yk;
            p.comp[v] = (t - q.b) - yk;
            p.acc[v] = t;
        }
    }
}

template <int MODE>
__device__ __forceinline__ void epilogue(const StepParams &p, int64_t v, int j, float sum) {
    epi_store<MODE>(p, v, j, sum, epi_load<MODE>(p, v));
}

// Contribution of edge e = (u -> row) to column j.  On the first family
// step x(0) = c e_seed, so only the seed's own out-edges contribute and no
// vector is gathered (the source is in the row's block, so its seed is
// looked up through u).  Uniform weights: the gathered vector is already
// scaled by 1/outdeg; explicit weights: multiply by w[e].
template <bool FIRST, bool WEIGHTED, int KT>
__device__ __forceinline__ float edge_value(const StepParams &p, int64_t e, int32_t u, int j) {
    if (FIRST) {
        if (u != seed_of(p, u, j)) return 0.0f;
        return p.c * (WEIGHTED ? p.w[e] : p.inv[u]);
    }
    const float z = p.zin[(int64_t)u * KT + j];
    return WEIGHTED ? p.w[e] * z : z;
}

// Finish pass over long rows: add each row's chunk partials in chunk order
// and apply the epilogue (a separate launch after the step kernel, so no
// cross-workgroup synchronisation is needed inside the step).
template <int MODE>
__device__ __forceinline__ void finish_row(const StepParams &p, const LongRow &lr, int lane) {
    const int kt = p.kt;
    if (kt == 1) {
        float t = 0.0f;
        for (int i = lane; i < lr.nchunks; i += 64) t += p.partials[(int64_t)lr.first_item + i];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
        if (lane == 0) epilogue<MODE>(p, lr.row, 0, t);
    } else {
        // column j's partials in chunk order, 16 loads in flight per round
        constexpr int R = 16;
        for (int j = lane; j < kt; j += 64) {
            const float *pj = p.partials + (int64_t)lr.first_item * kt + j;
            float t = 0.0f;
            int i = 0;
            for (; i + R <= lr.nchunks; i += R) {
                float v[R];
#pragma unroll
                for (int k = 0; k < R; ++k) v[k] = pj[(int64_t)(i + k) * kt];
#pragma unroll
                for (int k = 0; k < R; ++k) t += v[k];
            }
            for (; i < lr.nchunks; ++i) t += pj[(int64_t)i * kt];
            epilogue<MODE>(p, lr.row, j, t);
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(kThreads) void finish_kernel(const LongRow *__restrict__ longs, int64_t n_long,
                                                          StepParams p) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (wid >= n_long || (p.skip_on && *p.skip_on)) return;
    finish_row<MODE>(p, longs[wid], lane);
}

// Gather row r of the pushed second step: acc[r] holds the row's gathered
// value (y2 scaled by 1/outdeg for uniform weights) in 2^62 fixed point, the
// restart term included; it is cleared for the next query.  Returns whether
// the row is non-zero.
__device__ __forceinline__ bool push_convert_row(const StepParams &p, const PushPlan &pp, int64_t r) {
    const unsigned long long a = pp.acc[r];
    p.zout[r] = (float)((double)a * 0x1p-62);
    if (a) pp.acc[r] = 0ull;
    return a != 0ull;
}

// Rows [base, base + 256) of acc (2^62 fixed point) into the gathered
// vector p.zout, acc cleared, and the span's eight words of the frontier
// bitmap (rows past n left clear).  One wave: lane i converts rows 4i..4i+3
// (two 16-byte loads, one 16-byte store where aligned), and lanes 0..7 write
// word w from the 4 row bits of lanes 8w..8w+7.
__device__ __forceinline__ void convert_span(const StepParams &p, const PushPlan &pp, int64_t base, int lane,
                                             bool vec) {
    const int64_t r0 = base + 4 * lane;
    uint32_t live4 = 0u;  // bit k: row r0 + k is non-zero
    if (vec && r0 + 3 < p.n) {
        ulonglong2 *a = reinterpret_cast<ulonglong2 *>(pp.acc + r0);
        const ulonglong2 lo = a[0], hi = a[1];
        *reinterpret_cast<float4 *>(p.zout + r0) =
            make_float4((float)((double)lo.x * 0x1p-62), (float)((double)lo.y * 0x1p-62),
                        (float)((double)hi.x * 0x1p-62), (float)((double)hi.y * 0x1p-62));
        if (lo.x | lo.y) a[0] = make_ulonglong2(0ull, 0ull);
        if (hi.x | hi.y) a[1] = make_ulonglong2(0ull, 0ull);
        live4 = (lo.x != 0ull ? 1u : 0u) | (lo.y != 0ull ? 2u : 0u) | (hi.x != 0ull ? 4u : 0u) |
                (hi.y != 0ull ? 8u : 0u);
    } else {
        for (int k = 0; k < 4; ++k)
            if (r0 + k < p.n && push_convert_row(p, pp, r0 + k)) live4 |= 1u << k;
    }
    uint64_t b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) b[k] = __ballot((live4 >> k) & 1u);
    if (lane < 8) {
        uint32_t word = 0u;
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) word |= (uint32_t)((b[k] >> (8 * lane + j)) & 1ull) << (4 * j + k);
        const int64_t w = (base >> 5) + lane;
        if (w < pp.nwords) pp.bits[w] = word;
    }
}

// ------------------------------------------------------------ kt == 1
template <int MODE, bool FIRST, bool WEIGHTED>
__device__ __forceinline__ void item_1(const StepParams &p, const Item it, int64_t wid, int lane, float *my) {
    const int kind = (int)item_kind(it.meta);
    const int nnz = (int)item_nnz(it.meta);
    const int32_t *col = p.col + it.e0;
    const int32_t seed_pre = MODE == kFamily ? seed_ahead(p, 0) : kSeedLookup;
    if (kind == (int)kItemGroup) {
        constexpr int NS = kGroupMax / 64;
        const int nrows = (int)item_nrows(it.meta);
        const int rel = lane <= nrows ? (int)(p.rowptr[it.row0 + lane] - it.e0) : nnz;
        // all index loads, the epilogue operands, then all gathers, then LDS.
        // In gather order (col_slots) entry e holds the row to gather and,
        // above it, the edge's position in the item, where its product goes:
        // the LDS slice is then in row order as before, so are the sums.
        const bool slots = p.col_slots != 0;
        uint32_t raw[NS];  // kNoEdge past the item's end
        constexpr uint32_t kNoEdge = ~0u;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int e = s * 64 + lane;
            raw[s] = e < nnz ? (uint32_t)col[e] : kNoEdge;
        }
        EpiPre q;
        if (lane < nrows) q = epi_load<MODE>(p, it.row0 + lane);
        int32_t u[NS];
        int pos[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            u[s] = raw[s] == kNoEdge ? -1 : (int32_t)(slots ? raw[s] & kGroupRowMask : raw[s]);
            pos[s] = slots ? (int)(raw[s] >> kGroupSlotShift) : s * 64 + lane;
        }
        if (!FIRST && frontier_on(p)) {
#pragma unroll
            for (int s = 0; s < NS; ++s)
                if (u[s] >= 0 && !row_live(p, u[s])) u[s] = -1;  // a zero row: its term is 0
        }
        float v[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s)
            v[s] = u[s] >= 0 ? edge_value<FIRST, WEIGHTED, 1>(p, it.e0 + pos[s], u[s], 0) : 0.0f;
        wave_sync();  // the previous item's LDS reads are done
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (raw[s] != kNoEdge) my[pos[s]] = v[s];
        const int rel_next = __shfl(rel, lane + 1 < 64 ? lane + 1 : 63, 64);
        wave_sync();
        // rows of <= 32 edges: lane r adds row r's slice; longer rows: the
        // whole wave strides over the slice, then a xor butterfly
        const int len = rel_next - rel;
        if (lane < nrows && len <= 32) {
            float acc = 0.0f;
            for (int k = rel; k < rel_next; ++k) acc += my[k];
            epi_store<MODE>(p, it.row0 + lane, 0, acc, q, seed_pre);
        }
        uint64_t big = __ballot(lane < nrows && len > 32);
        while (big) {
            const int r = __builtin_ctzll(big);
            big &= big - 1;
            const int b = __builtin_amdgcn_readlane(rel, r), en = __builtin_amdgcn_readlane(rel_next, r);
            const EpiPre qr = epi_readlane(q, r);
            float t = 0.0f;
            for (int k = b + lane; k < en; k += 64) t += my[k];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
            if (lane == 0) epi_store<MODE>(p, it.row0 + r, 0, t, qr, seed_pre);
        }
        return;
    }
    // one row, or one chunk of a long row
    constexpr int UNR = 16;
    EpiPre q;
    if (kind == (int)kItemRow && lane == 0) q = epi_load<MODE>(p, it.row0);
    const bool sparse = !FIRST && frontier_on(p);
    float s = 0.0f;
    for (int base = 0; base < nnz; base += 64 * UNR) {
        int32_t u[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const int e = base + k * 64 + lane;
            u[k] = e < nnz ? col[e] : -1;
        }
        if (sparse) {
#pragma unroll
            for (int k = 0; k < UNR; ++k)
                if (u[k] >= 0 && !row_live(p, u[k])) u[k] = -1;
        }
        float v[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k)
            v[k] = u[k] >= 0 ? edge_value<FIRST, WEIGHTED, 1>(p, it.e0 + base + k * 64 + lane, u[k], 0) : 0.0f;
#pragma unroll
        for (int k = 0; k < UNR; ++k) s += v[k];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        if (kind == (int)kItemRow)
            epi_store<MODE>(p, it.row0, 0, s, q, seed_pre);
        else
            p.partials[p.chunk_slot_in_item ? (int64_t)it.row0 : wid] = s;
    }
}

// A block item: the block's 4 waves each add a quarter of one row (64-edge
// aligned), then wave 0 adds the quarter sums in wave order.
template <int MODE, bool FIRST, bool WEIGHTED>
__device__ __forceinline__ void block_row_1(const StepParams &p, const Item it, int lane, int wv,
                                            float (*lds)[kGroupMax]) {
    const int nnz = (int)item_nnz(it.meta);
    const int qlen = (((nnz + kWaves - 1) / kWaves) + 63) & ~63;
    const int qb = wv * qlen, qe = min(nnz, qb + qlen);
    EpiPre q;
    if (wv == 0 && lane == 0) q = epi_load<MODE>(p, it.row0);
    const int32_t *col = p.col + it.e0;
    constexpr int UNR = 16;
    const bool sparse = !FIRST && frontier_on(p);
    float s = 0.0f;
    for (int base = qb; base < qe; base += 64 * UNR) {
        int32_t u[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
            const int e = base + k * 64 + lane;
            u[k] = e < qe ? col[e] : -1;
        }
        if (sparse) {
#pragma unroll
            for (int k = 0; k < UNR; ++k)
                if (u[k] >= 0 && !row_live(p, u[k])) u[k] = -1;
        }
        float v[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k)
            v[k] = u[k] >= 0 ? edge_value<FIRST, WEIGHTED, 1>(p, it.e0 + base + k * 64 + lane, u[k], 0) : 0.0f;
#pragma unroll
        for (int k = 0; k < UNR; ++k) s += v[k];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) lds[wv][0] = s;
    __syncthreads();
    if (wv == 0 && lane == 0) {
        float t = lds[0][0];
        for (int w = 1; w < kWaves; ++w) t += lds[w][0];
        epi_store<MODE>(p, it.row0, 0, t, q);
    }
}

// One wave per work item (the hardware dispatcher balances the waves); the
// 4 slots of a block item are taken by the 4 waves of one block.
template <int MODE, bool FIRST, bool WEIGHTED>
__global__ __launch_bounds__(kThreads) void step_kernel_1(const Item *__restrict__ items, int64_t n_items,
                                                          StepParams p) {
    __shared__ float lds[kWaves][kGroupMax];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + wv;
    if (wid >= n_items || (p.skip_on && *p.skip_on)) return;
    const Item it = items[wid];
    if (item_kind(it.meta) == kItemBlock) {
        block_row_1<MODE, FIRST, WEIGHTED>(p, it, lane, wv, lds);
        return;
    }
    item_1<MODE, FIRST, WEIGHTED>(p, it, wid, lane, lds[wv]);
}

// ------------------------------------------------------------ XCD-sliced, kt == 1
// Group-kind items of an XCD-sliced schedule (kt == 1, 1/outdeg weights,
// never a first step): BAND, slice x's runs of up to 63 medium rows into
// consecutive partial slots (from xrel's first entry); otherwise consecutive rows whose offsets come from
// rowptr_x, summed only for the short rows (medium and long rows have no
// edges in that section and take their epilogue in the finish pass).  The
// products go through the wave's LDS slice as in a group item.
template <int MODE, bool BAND>
__device__ __forceinline__ void item_1x(const StepParams &p, const Item it, int lane, float *my) {
    constexpr int NS = kGroupMax / 64;
    const int nrows = (int)item_nrows(it.meta);
    const int nnz = (int)item_nnz(it.meta);
    const int32_t *col = p.col + it.e0;
    const int32_t seed_pre = MODE == kFamily ? seed_ahead(p, 0) : kSeedLookup;
    int rel;
    bool own = false;  // the lane's row takes its epilogue here
    int64_t slot0 = 0;
    if (BAND) {
        const int32_t *tab = p.xrel + it.row0;
        slot0 = tab[0];
        rel = lane <= nrows ? tab[1 + lane] : nnz;
    } else {
        const int64_t rx = lane <= nrows ? p.rowptr_x[it.row0 + lane] : 0;
        rel = lane <= nrows ? (int)((rx & kRowxMask) - it.e0) : nnz;
        own = lane < nrows && !((rx >> kRowxForeignBit) & 1);
    }
    int32_t u[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int e = s * 64 + lane;
        u[s] = e < nnz ? col[e] : -1;
    }
    EpiPre q;
    if (!BAND && own) q = epi_load<MODE>(p, it.row0 + lane);
    if (frontier_on(p)) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (u[s] >= 0 && !row_live(p, u[s])) u[s] = -1;  // a zero row: its term is 0
    }
    float v[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) v[s] = u[s] >= 0 ? edge_value<false, false, 1>(p, 0, u[s], 0) : 0.0f;
    wave_sync();  // the previous item's LDS reads are done
#pragma unroll
    for (int s = 0; s < NS; ++s)
        if (s * 64 + lane < nnz) my[s * 64 + lane] = v[s];
    const int rel_next = __shfl(rel, lane + 1 < 64 ? lane + 1 : 63, 64);
    wave_sync();
    const int len = rel_next - rel;
    if (lane < nrows && len <= 32) {
        float acc = 0.0f;
        for (int k = rel; k < rel_next; ++k) acc += my[k];
        if (BAND) p.partials[slot0 + lane] = acc;
        else if (own) epi_store<MODE>(p, it.row0 + lane, 0, acc, q, seed_pre);
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
        if (BAND) {
            if (lane == 0) p.partials[slot0 + r] = t;
        } else {
            const EpiPre qr = epi_readlane(q, r);  // a row with edges here is the item's own
            if (lane == 0) epi_store<MODE>(p, it.row0 + r, 0, t, qr, seed_pre);
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(kThreads) void step_kernel_1x(const Item *__restrict__ items, int64_t n_items,
                                                           StepParams p) {
    __shared__ float lds[kWaves][kGroupMax];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + wv;
    if (wid >= n_items || (p.skip_on && *p.skip_on)) return;
    const Item it = items[wid];
    if (item_kind(it.meta) == kItemChunk)
        item_1<MODE, false, false>(p, it, wid, lane, lds[wv]);
    else if (it.meta & kItemBandBit)
        item_1x<MODE, true>(p, it, lane, lds[wv]);
    else
        item_1x<MODE, false>(p, it, lane, lds[wv]);
}

// Finish of the medium rows of an XCD-sliced schedule, one thread per row:
// its 8 slice sums (slice x of medium row i in slot x * n_rows + i, added
// pairwise in a fixed order), then the epilogue.
template <int MODE>
__global__ __launch_bounds__(kThreads) void finish8_kernel(const LongRow *__restrict__ rows, int64_t n_rows,
                                                           StepParams p) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n_rows || (p.skip_on && *p.skip_on)) return;
    const int32_t row = rows[i].row;
    float v[kSliceCount];
#pragma unroll
    for (int x = 0; x < kSliceCount; ++x) v[x] = p.partials[(int64_t)x * n_rows + i];
    const float t = ((v[0] + v[4]) + (v[2] + v[6])) + ((v[1] + v[5]) + (v[3] + v[7]));
    epilogue<MODE>(p, row, 0, t);
}

// Finish of the long rows of an XCD-sliced schedule: 8 lanes per row stride
// over its chunk sums (slice, then chunk order; a fixed xor order).
template <int MODE>
__global__ __launch_bounds__(kThreads) void finish_long8_kernel(const LongRow *__restrict__ longs, int64_t n_long,
                                                                StepParams p) {
    const int lane = threadIdx.x & 63;
    const int64_t i = ((int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6)) * 8 + (lane >> 3);
    if (p.skip_on && *p.skip_on) return;
    const bool ok = i < n_long;
    LongRow lr = {0, 0, 0, 0};
    if (ok) lr = longs[i];
    float t = 0.0f;
    for (int k = lane & 7; k < lr.nchunks; k += 8) t += p.partials[(int64_t)lr.first_item + k];
    t += __shfl_xor(t, 4, 64);
    t += __shfl_xor(t, 2, 64);
    t += __shfl_xor(t, 1, 64);
    if (ok && (lane & 7) == 0) epilogue<MODE>(p, lr.row, 0, t);
}

// The second family step of a single seed, gated by the push plan's flag:
// when the step was pushed, the launch converts the fixed-point sums of
// every gather row; otherwise it pulls the step over A~^T.  Blocks stride
// over 4-item slots (one slot each at the launch's grid); block items fill
// whole slots, so all 4 waves of a block meet the same barriers.

template <bool WEIGHTED>
__global__ __launch_bounds__(kThreads) void gated_step_kernel_1(const Item *__restrict__ items, int64_t n_items,
                                                                StepParams p, PushPlan pp) {
    __shared__ float lds[kWaves][kGroupMax];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (*pp.flag) {
        // pushed: convert every gather row, coalesced, no work items
        const bool vec = (reinterpret_cast<uintptr_t>(p.zout) & 15) == 0;
        const int64_t first = ((int64_t)blockIdx.x * kWaves + wv) * 256;
        const int64_t step = (int64_t)gridDim.x * kWaves * 256;
        for (int64_t base = first; base < p.n; base += step)  // wave-uniform trip count
            convert_span(p, pp, base, lane, vec);
        return;
    }
    const int64_t slots = (n_items + kWaves - 1) / kWaves;
    for (int64_t b = blockIdx.x; b < slots; b += gridDim.x) {
        const int64_t wid = b * kWaves + wv;
        if (wid >= n_items) continue;  // only in the last slot, which holds no block item
        const Item it = items[wid];
        const int kind = (int)item_kind(it.meta);
        if (kind == (int)kItemBlock) {
            block_row_1<kFamily, false, WEIGHTED>(p, it, lane, wv, lds);
            __syncthreads();  // wave 0 has read the quarter sums before the slot is reused
        } else {
            item_1<kFamily, false, WEIGHTED>(p, it, wid, lane, lds[wv]);
        }
    }
}

__global__ __launch_bounds__(kThreads) void gated_finish_kernel(const LongRow *__restrict__ longs, int64_t n_long,
                                                                StepParams p, PushPlan pp) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (wid >= n_long) return;
    if (*pp.flag) return;  // the step launch converted every row
    finish_row<kFamily>(p, longs[wid], lane);
}

// ------------------------------------------------------------ kt == 64
// Value of one edge for lane j; u and (for explicit weights) w are uniform.
template <bool FIRST, bool WEIGHTED>
__device__ __forceinline__ float walk_value(const StepParams &p, int32_t u, float w, int j,
                                            int32_t seed_plain, float cinv_plain) {
    if (FIRST) {
        int32_t seed = seed_plain;
        if (p.node_block) seed = (j < p.ncols) ? p.seeds[(int64_t)p.node_block[u] * p.seed_stride + j] : -1;
        if (u != seed) return 0.0f;
        return WEIGHTED ? p.c * w : (p.node_block ? p.c * p.inv[u] : cinv_plain);
    }
    const float z = p.zin[(int64_t)u * 64 + j];
    return WEIGHTED ? w * z : z;
}

// Final output of the last family step for row v, column j (the fused
// combine of Algorithm 3), with r~_stranger[v] in q.a; NaN (and the sticky
// flag) for an invalid seed.
__device__ __forceinline__ float family_out_value(const StepParams &p, int64_t v, int j, float sum, const EpiPre &q,
                                                  int32_t seed_pre) {
    int32_t seed = -1;
    float restart;
    if (p.qdense) {
        restart = p.qT[v * p.kt + j];
    } else {
        seed = seed_pre != kSeedLookup ? seed_pre : seed_of(p, v, j);
        restart = (v == (int64_t)seed) ? p.c : 0.0f;
    }
    const float y = fmaf(p.omc, sum, restart);
    if (p.qdense || seed_valid(p, v, seed)) return fmaf(p.alpha, y, q.a);
    *p.err = 1;
    return qnan();
}

// The last step of a 64-column tile stages 16 rows x 64 columns in LDS
// (row stride 65) and writes each seed column's run of rows with one
// coalesced store, instead of 64 scattered 4-byte stores per row.
constexpr int kStageRows = 16;
constexpr int kStageStride = 65;

__device__ __forceinline__ void stage_write(const StepParams &p, const float *buf, int64_t row_base, int cnt,
                                            int lane) {
    wave_sync();
    for (int j = 0; j < p.ncols; ++j)
        if (lane < cnt) p.out[(p.out_col0 + j) * p.n + row_base + lane] = buf[lane * kStageStride + j];
    wave_sync();
}

// SPARSE: the launch's frontier skip is on (a gather per live row only); the
// dense walk is compiled without the per-edge test.  The item's fields are
// wave-uniform and kept in scalar registers, so its loop bounds and row
// boundaries cost scalar compares only.
// One batch of U row gathers of a 64-edge strip (column ids colv; lane j
// takes column j of each edge's row).  SPARSE zeroes, and does not load,
// the rows the frontier bitmap marks dead.
template <bool FIRST, bool WEIGHTED, bool SPARSE, int U>
__device__ __forceinline__ void gather_batch(const StepParams &p, int32_t colv, float wv, uint64_t live, int t0,
                                             int lane, int32_t seed_plain, float cinv_plain, float (&v)[U]) {
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const float w = WEIGHTED ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wv), t0 + k)) : 0.0f;
        const int32_t u = __builtin_amdgcn_readlane(colv, t0 + k);
        v[k] = (!SPARSE || ((live >> (t0 + k)) & 1ull)) ? walk_value<FIRST, WEIGHTED>(p, u, w, lane, seed_plain, cinv_plain)
                                                        : 0.0f;
    }
}

template <int MODE, bool FIRST, bool WEIGHTED, bool SPARSE>
__device__ __forceinline__ void item_64(const StepParams &p, const Item it0, int64_t wid, int lane, float *buf) {
    Item it;
    it.e0 = ((int64_t)__builtin_amdgcn_readfirstlane((int32_t)(it0.e0 >> 32)) << 32) |
            (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)it0.e0);
    it.row0 = __builtin_amdgcn_readfirstlane(it0.row0);
    it.meta = __builtin_amdgcn_readfirstlane(it0.meta);
    const int kind = (int)item_kind(it.meta);
    const int nnz = (int)item_nnz(it.meta);
    int32_t seed_plain = -1;
    float cinv_plain = 0.0f;
    if (FIRST && !p.node_block && lane < p.ncols) {
        seed_plain = p.seeds[lane];
        if (!WEIGHTED && seed_plain >= 0 && (int64_t)seed_plain < p.n) cinv_plain = p.c * p.inv[seed_plain];
    }
    constexpr int U = 32;  // row gathers in flight per wave
    constexpr bool sparse = SPARSE && !FIRST;
    // the epilogue's per-row operands are loaded ahead, one row per lane, and
    // each lane's seed once: no memory round trip at a row boundary
    const int32_t seed_pre = MODE == kFamily ? seed_ahead(p, lane) : kSeedLookup;
    if (kind == (int)kItemGroup) {
        const bool staged = MODE == kFamily && p.last;
        const int nrows = (int)item_nrows(it.meta);
        const int rel = lane <= nrows ? (int)(p.rowptr[it.row0 + lane] - it.e0) : nnz;
        EpiPre q;
        if (lane < nrows) q = epi_load<MODE>(p, it.row0 + lane);
        int r = 0;
        int rend = __builtin_amdgcn_readlane(rel, 1);
        float acc = 0.0f;
        for (int base = 0; base < nnz; base += 64) {
            const int cnt = min(64, nnz - base);
            const int32_t colv = lane < cnt ? p.col[it.e0 + base + lane] : 0;
            const float wv = (WEIGHTED && lane < cnt) ? p.w[it.e0 + base + lane] : 0.0f;
            const uint64_t live = sparse ? __ballot(lane < cnt && row_live(p, colv)) : ~0ull;
            // one copy of the row-closing code per edge of a batch (unrolling
            // the strip's two batches as well doubled the kernel's code and
            // slowed it)
            for (int t0 = 0; t0 < cnt; t0 += U) {
                float v[U];
                gather_batch<FIRST, WEIGHTED, sparse, U>(p, colv, wv, live, t0, lane, seed_plain, cinv_plain, v);
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    if (t0 + k < cnt) {
                        // close every row that ends before this edge, then add its value
                        const int e = base + t0 + k;
                        while (e >= rend) {
                            const EpiPre qr = epi_readlane(q, r);
                            if (staged) {
                                buf[(r % kStageRows) * kStageStride + lane] =
                                    lane < p.ncols ? family_out_value(p, it.row0 + r, lane, acc, qr, seed_pre) : 0.0f;
                                if (r % kStageRows == kStageRows - 1)
                                    stage_write(p, buf, it.row0 + r - (kStageRows - 1), kStageRows, lane);
                            } else {
                                epi_store<MODE>(p, it.row0 + r, lane, acc, qr, seed_pre);
                            }
                            acc = 0.0f;
                            ++r;
                            rend = __builtin_amdgcn_readlane(rel, r + 1);
                        }
                        acc += v[k];
                    }
                }
            }
        }
        for (; r < nrows; ++r) {
            const EpiPre qr = epi_readlane(q, r);
            if (staged) {
                buf[(r % kStageRows) * kStageStride + lane] =
                    lane < p.ncols ? family_out_value(p, it.row0 + r, lane, acc, qr, seed_pre) : 0.0f;
                if (r % kStageRows == kStageRows - 1)
                    stage_write(p, buf, it.row0 + r - (kStageRows - 1), kStageRows, lane);
            } else {
                epi_store<MODE>(p, it.row0 + r, lane, acc, qr, seed_pre);
            }
            acc = 0.0f;
        }
        if (staged && nrows % kStageRows)
            stage_write(p, buf, it.row0 + nrows - nrows % kStageRows, nrows % kStageRows, lane);
        return;
    }
    // one row (or a chunk of one): U edges in flight, sequential per lane
    EpiPre q1;
    if (kind == (int)kItemRow) q1 = epi_load<MODE>(p, it.row0);
    float s = 0.0f;
    for (int base = 0; base < nnz; base += 64) {
        const int cnt = min(64, nnz - base);
        const int32_t colv = lane < cnt ? p.col[it.e0 + base + lane] : 0;
        const float wv = (WEIGHTED && lane < cnt) ? p.w[it.e0 + base + lane] : 0.0f;
        const uint64_t live = sparse ? __ballot(lane < cnt && row_live(p, colv)) : ~0ull;
        for (int t0 = 0; t0 < cnt; t0 += U) {
            float v[U];
            gather_batch<FIRST, WEIGHTED, sparse, U>(p, colv, wv, live, t0, lane, seed_plain, cinv_plain, v);
#pragma unroll
            for (int k = 0; k < U; ++k)
                if (t0 + k < cnt) s += v[k];
        }
    }
    if (kind == (int)kItemRow)
        epi_store<MODE>(p, it.row0, lane, s, q1, seed_pre);
    else
        p.partials[wid * 64 + lane] = s;
}

// 7 resident blocks per CU (at most 72 VGPRs): the walk is bound by the
// latency of its gather batches, and a seventh wave per SIMD beats the
// registers it costs (24.0 against 25.1 ms for 1024 seeds on rmat20).
// WALK: 0 = the frontier skip decided per launch on the device (bits_on),
// 1 = sparse (skip on), 2 = dense.  The host picks it, so that each variant
// gets its own registers: one kernel holding both walks spilled, and the
// dense walk without the per-edge frontier test is 12 % faster (64-seed tile
// on 2^20 nodes: 511 to 450 us per step).
template <int MODE, bool FIRST, bool WEIGHTED, int WALK>
__global__ __launch_bounds__(kThreads, 7) void step_kernel_64(const Item *__restrict__ items, int64_t n_items,
                                                           StepParams p) {
    __shared__ float stage[kWaves][kStageRows * kStageStride];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + wv;
    if (wid >= n_items || (p.skip_on && *p.skip_on)) return;
    if (WALK == 0) {
        if (!FIRST && frontier_on(p)) item_64<MODE, FIRST, WEIGHTED, true>(p, items[wid], wid, lane, stage[wv]);
        else item_64<MODE, FIRST, WEIGHTED, false>(p, items[wid], wid, lane, stage[wv]);
    } else {
        item_64<MODE, FIRST, WEIGHTED, WALK == 1>(p, items[wid], wid, lane, stage[wv]);
    }
}

// ------------------------------------------------------------ kt = 2..32
template <int KT, bool FIRST, bool WEIGHTED>
__device__ __forceinline__ float range_sum_kt(const StepParams &p, int64_t e0, int64_t e1, int sub, int j) {
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
        float v[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k)
            v[k] = u[k] >= 0 ? edge_value<FIRST, WEIGHTED, KT>(p, base + k * SUBS, u[k], j) : 0.0f;
#pragma unroll
        for (int k = 0; k < UNR; ++k) s += v[k];
    }
#pragma unroll
    for (int off = KT; off < 64; off <<= 1) s += __shfl_xor(s, off, 64);
    return s;
}

// One row summed by one sub-group of KT lanes (lane j = column j), its
// edges in order with 4 gathers in flight.
template <int KT, bool FIRST, bool WEIGHTED>
__device__ __forceinline__ float row_sum_kt(const StepParams &p, int64_t e0, int64_t e1, int j) {
    constexpr int UNR = 4;
    float s = 0.0f;
    for (int64_t base = e0; base < e1; base += UNR) {
        int32_t u[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) u[k] = base + k < e1 ? p.col[base + k] : -1;
        float v[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) v[k] = u[k] >= 0 ? edge_value<FIRST, WEIGHTED, KT>(p, base + k, u[k], j) : 0.0f;
#pragma unroll
        for (int k = 0; k < UNR; ++k) s += v[k];
    }
    return s;
}

__device__ __forceinline__ EpiPre epi_shfl(const EpiPre &q, int r) {
    EpiPre o;
    o.a = __shfl(q.a, r, 64);
    o.b = __shfl(q.b, r, 64);
    o.c = __shfl(q.c, r, 64);
    o.zi = __shfl(q.zi, r, 64);
    return o;
}

constexpr int kShortRowKt = 32;  // rows up to this many edges take one sub-group

// STAGED (the last family step): a group item's outputs are kept in the
// wave's LDS slice, [row][KT] with row stride KT + 1, and written column by
// column, each column's run of the item's rows with one coalesced store,
// instead of KT scattered 4-byte stores per row (seed-major output).
template <int KT, int MODE, bool FIRST, bool WEIGHTED, bool STAGED = false>
__device__ __forceinline__ void item_kt(const StepParams &p, const Item it, int64_t wid, int lane,
                                        float *buf = nullptr) {
    constexpr int SUBS = 64 / KT;
    const int j = lane % KT, sub = lane / KT;
    const int kind = (int)item_kind(it.meta);
    const int nnz = (int)item_nnz(it.meta);
    const int32_t seed_pre = MODE == kFamily ? seed_ahead(p, j) : kSeedLookup;
    if (kind == (int)kItemGroup) {
        // row offsets and epilogue operands loaded ahead, one row per lane
        const int nrows = (int)item_nrows(it.meta);
        const int rel = lane <= nrows ? (int)(p.rowptr[it.row0 + lane] - it.e0) : nnz;
        const int rel_next = __shfl(rel, lane + 1 < 64 ? lane + 1 : 63, 64);
        EpiPre q;
        if (lane < nrows) q = epi_load<MODE>(p, it.row0 + lane);
        // short rows: SUBS rows at a time, one per sub-group
        for (int rb = 0; rb < nrows; rb += SUBS) {
            const int r = min(rb + sub, 63);
            const int b = __shfl(rel, r, 64), en = __shfl(rel_next, r, 64);
            const bool mine = rb + sub < nrows && en - b <= kShortRowKt;
            const EpiPre qr = epi_shfl(q, r);
            if (mine) {
                const float s = row_sum_kt<KT, FIRST, WEIGHTED>(p, it.e0 + b, it.e0 + en, j);
                if (STAGED) {
                    if (j < p.ncols) buf[r * (KT + 1) + j] = family_out_value(p, it.row0 + r, j, s, qr, seed_pre);
                } else {
                    epi_store<MODE>(p, it.row0 + r, j, s, qr, seed_pre);
                }
            }
        }
        // longer rows: the whole wave, sub-groups striding over the edges
        uint64_t big = __ballot(lane < nrows && rel_next - rel > kShortRowKt);
        while (big) {
            const int r = __builtin_ctzll(big);
            big &= big - 1;
            const int b = __builtin_amdgcn_readlane(rel, r), en = __builtin_amdgcn_readlane(rel, r + 1);
            const EpiPre qr = epi_readlane(q, r);
            const float s = range_sum_kt<KT, FIRST, WEIGHTED>(p, it.e0 + b, it.e0 + en, sub, j);
            if (sub == 0) {
                if (STAGED) {
                    if (j < p.ncols) buf[r * (KT + 1) + j] = family_out_value(p, it.row0 + r, j, s, qr, seed_pre);
                } else {
                    epi_store<MODE>(p, it.row0 + r, j, s, qr, seed_pre);
                }
            }
        }
        if (STAGED) {
            wave_sync();
            for (int jj = 0; jj < p.ncols; ++jj)
                if (lane < nrows) p.out[(p.out_col0 + jj) * p.n + it.row0 + lane] = buf[lane * (KT + 1) + jj];
            wave_sync();  // the slice is reused by the wave's next item
        }
        return;
    }
    EpiPre q1;
    if (kind == (int)kItemRow) q1 = epi_load<MODE>(p, it.row0);
    const float s = range_sum_kt<KT, FIRST, WEIGHTED>(p, it.e0, it.e0 + nnz, sub, j);
    if (sub == 0) {
        if (kind == (int)kItemRow)
            epi_store<MODE>(p, it.row0, j, s, q1, seed_pre);
        else
            p.partials[wid * KT + j] = s;
    }
}

template <int KT, int MODE, bool FIRST, bool WEIGHTED>
__global__ __launch_bounds__(kThreads) void step_kernel_kt(const Item *__restrict__ items, int64_t n_items,
                                                           StepParams p) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (wid >= n_items || (p.skip_on && *p.skip_on)) return;
    item_kt<KT, MODE, FIRST, WEIGHTED>(p, items[wid], wid, lane);
}

// The last family step of a tile of KT columns, its outputs staged per item
// (a group item holds at most 63 rows).
template <int KT, bool FIRST, bool WEIGHTED>
__global__ __launch_bounds__(kThreads) void last_step_kernel_kt(const Item *__restrict__ items, int64_t n_items,
                                                                StepParams p) {
    __shared__ float stage[kWaves][64 * (KT + 1)];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wid = (int64_t)blockIdx.x * kWaves + wv;
    if (wid >= n_items || (p.skip_on && *p.skip_on)) return;
    item_kt<KT, kFamily, FIRST, WEIGHTED, true>(p, items[wid], wid, lane, stage[wv]);
}

__global__ void stranger_init_kernel(int64_t n, float c, const float *restart_pr, float inv_n,
                                     const float *inv, const float *w_present, int include_x0,
                                     float *zout, float *acc, float *comp, const int32_t *zperm) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const float x0 = c * (restart_pr ? restart_pr[v] : inv_n);
        zout[zperm ? zperm[v] : v] = w_present ? x0 : x0 * inv[v];
        acc[v] = include_x0 ? x0 : 0.0f;
        comp[v] = 0.0f;
    }
}

__global__ void dense_init_kernel(StepParams p, float *z0, float *x0) {
    const int64_t total = p.n * (int64_t)p.kt;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = i / p.kt;
        const int j = (int)(i - v * p.kt);
        const float x = p.qT ? p.qT[i] : (j < p.ncols ? p.c * p.qdense[(int64_t)j * p.n + v] : 0.0f);
        z0[zrow(p, v) * p.kt + j] = p.w ? x : x * p.inv[v];
        if (x0) x0[i] = x;
    }
}

// Tile transpose of the dense restarts: a block takes 64 nodes, reads each
// column's run of 64 entries (coalesced) into LDS and writes the 64 x kt
// node-major block (coalesced).
constexpr int kTransNodes = 64;

__global__ __launch_bounds__(256) void dense_transpose_kernel(StepParams p, float *qT) {
    __shared__ float tile[64][kTransNodes + 1];
    const int64_t v0 = (int64_t)blockIdx.x * kTransNodes;
    const int t = threadIdx.x & 63, r = threadIdx.x >> 6;
    for (int j = r; j < p.kt; j += 4) {
        const int64_t v = v0 + t;
        tile[j][t] = (j < p.ncols && v < p.n) ? p.c * p.qdense[(int64_t)j * p.n + v] : 0.0f;
    }
    __syncthreads();
    const int64_t nv = min((int64_t)kTransNodes, p.n - v0);
    for (int i = threadIdx.x; i < nv * p.kt; i += blockDim.x) {
        const int vl = i / p.kt, j = i - vl * p.kt;
        qT[(v0 + vl) * p.kt + j] = tile[j][vl];
    }
}

__global__ void onehot_init_kernel(StepParams p, float *x0) {
    const int64_t total = p.n * (int64_t)p.kt;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = i / p.kt;
        const int j = (int)(i - v * p.kt);
        x0[i] = (v == (int64_t)seed_of(p, v, j)) ? p.c : 0.0f;
    }
}

__global__ void fill_zero_kernel(float *z, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        z[i] = 0.0f;
}

// Seed of pushed slot w = (block, column), or -1 when the slot holds no
// valid seed of its block.
__device__ __forceinline__ int32_t push_slot_seed(const StepParams &p, int64_t w, int &j) {
    const int64_t b = w / p.ncols;
    j = (int)(w - b * p.ncols);
    const int32_t s = p.seeds[b * (p.node_block ? p.seed_stride : 0) + j];
    if (s < 0 || (int64_t)s >= p.n) return -1;
    if (p.node_block && p.node_block[s] != b) return -1;
    return s;
}

// Claim gather row zr of y1 in the frontier bitmap; the first claimant
// zeroes the row's kt entries.
__device__ __forceinline__ void claim_row(const StepParams &p, uint32_t *bits, int64_t zr) {
    const uint32_t bit = 1u << (zr & 31);
    if (atomicOr(&bits[zr >> 5], bit) & bit) return;
    float *row = p.zout + zr * p.kt;
    if ((p.kt & 3) == 0) {
        for (int j = 0; j < p.kt; j += 4) *reinterpret_cast<float4 *>(row + j) = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
        for (int j = 0; j < p.kt; ++j) row[j] = 0.0f;
    }
}

// Rows of y1 for seed tiles with the frontier skip on: every seed row and
// out-neighbour row is marked in bits (cleared before) and zeroed once, so
// the push that follows writes into zeroed rows and no unmarked row of
// zout is ever read (the pull after it skips them).  One wave per slot.
__global__ void push_first_rows_kernel(StepParams p, const int64_t *a_rowptr, const int32_t *a_col, int64_t nslots,
                                       uint32_t *bits) {
    if (p.skip_on && *p.skip_on) return;
    const int lane = threadIdx.x & 63;
    const int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    if (w >= nslots) return;
    int j = 0;
    const int32_t s = push_slot_seed(p, w, j);
    if (s < 0) return;
    const int64_t e0 = a_rowptr[s], e1 = a_rowptr[s + 1];
    for (int64_t e = e0 + lane; e < e1; e += 64) claim_row(p, bits, zrow(p, a_col[e]));
    if (lane == 0) claim_row(p, bits, zrow(p, s));
}

// First family step from one-hot seeds, pushed over each seed's out-edges:
// y1 = c e_s + (1-c) c A~^T e_s is non-zero only at s and its out-neighbors
// (one wave per (block, column) seed; the rest of zout was zero-filled, or,
// with the frontier skip, the rows written here were zeroed).
__global__ void push_first_kernel(StepParams p, const int64_t *a_rowptr, const int32_t *a_col, const float *a_w,
                                  int64_t nslots) {
    if (p.skip_on && *p.skip_on) return;
    const int lane = threadIdx.x & 63;
    const int64_t w = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    if (w >= nslots) return;
    int j = 0;
    const int32_t s = push_slot_seed(p, w, j);
    if (s < 0) return;
    const int64_t e0 = a_rowptr[s], e1 = a_rowptr[s + 1];
    const float cw = p.c * p.omc;
    bool self = false;
    for (int64_t e = e0 + lane; e < e1; e += 64) {
        const int32_t v = a_col[e];
        const float wt = a_w ? a_w[e] : p.inv[s];
        const float y = fmaf(cw, wt, v == s ? p.c : 0.0f);
        const int64_t zr = zrow(p, v);
        p.zout[zr * p.kt + j] = a_w ? y : y * p.inv[v];
        self |= (v == s);
    }
    if (!__any(self) && lane == 0) {
        const int64_t zr = zrow(p, s);
        p.zout[zr * p.kt + j] = a_w ? p.c : p.c * p.inv[s];
    }
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ long long wave_scan_incl(long long x, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const long long y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

constexpr int kPlanMax = 2048;  // frontier nodes a block plans in LDS; larger frontiers pull step 2

__device__ __forceinline__ unsigned long long to_fixed62(float x) { return __double2ull_rn((double)x * 0x1p62); }

// The first two family steps of one seed (kt == 1, unpacked), in one launch.
// Every block plans step 2 itself, in LDS: F = out(s) + {s} (s appended
// when it has no self-loop), y1 on F as gathered values (x(1) lives on the
// seed's out-edges), the first A~ edge of each node of F (est) and the
// exclusive prefix sums of their out-degrees (offs), W = offs[|F|] edges
// in all.  When |F| <= kPlanMax and W <= wmax, step 2 is pushed: thread t
// takes edge slots t, t + T, ... (T threads), finds its node f by binary
// search over offs, so its edge is est[f] + t - offs[f], and adds the
// edge's term, in gathered form, to acc[zrow(v)] in 2^62 fixed point; no
// atomic result is waited for.  Every term is in [0, 1] and they add up to
// at most the mass of y2, below 1, so the sum cannot overflow.  Block 0
// records the decision (flag, ctrl = {W, |F|}) and adds the restart term
// c e_s.  Otherwise y1 is written densely to p.zout (the launch takes the
// first step's parameters, so that is the vector the pulled step 2 reads;
// zero for an invalid seed).
__global__ __launch_bounds__(256) void push_steps12_kernel(StepParams p, const int64_t *a_rowptr,
                                                           const int32_t *a_col, const float *a_w, PushPlan pp) {
    __shared__ long long soffs[kPlanMax + 1];
    __shared__ long long sest[kPlanMax];
    __shared__ float sy[kPlanMax];
    __shared__ long long swave[4];
    __shared__ int sself;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int32_t s = p.seeds[0];
    const bool valid = s >= 0 && (int64_t)s < p.n;
    const int64_t e0 = valid ? a_rowptr[s] : 0, e1 = valid ? a_rowptr[s + 1] : 0;
    const int64_t d = e1 - e0;
    const bool fits = valid && d < kPlanMax;  // |F| <= d + 1 <= kPlanMax
    const float cw = p.c * p.omc;
    long long run = 0;
    int nf = 0;
    if (fits) {
        if (tid == 0) sself = 0;
        __syncthreads();
        for (int base = 0; base < (int)d; base += 256) {  // block-uniform trip count
            const int f = base + tid;
            long long deg = 0;
            if (f < d) {
                const int32_t v = a_col[e0 + f];
                const float wt = a_w ? a_w[e0 + f] : p.inv[s];
                const float y = fmaf(cw, wt, v == s ? p.c : 0.0f);
                sy[f] = a_w ? y : y * p.inv[v];
                if (v == s) sself = 1;
                const int64_t rb = a_rowptr[v];
                deg = a_rowptr[v + 1] - rb;
                sest[f] = rb;
            }
            const long long incl = wave_scan_incl(deg, lane);
            if (lane == 63) swave[wv] = incl;
            __syncthreads();
            long long before = run;
            for (int w = 0; w < wv; ++w) before += swave[w];
            if (f < d) soffs[f] = before + incl - deg;
            run += swave[0] + swave[1] + swave[2] + swave[3];
            __syncthreads();  // swave is rewritten next round
        }
        nf = (int)d;
        if (!sself) {
            if (tid == 0) {
                sy[nf] = a_w ? p.c : p.c * p.inv[s];
                sest[nf] = e0;
                soffs[nf] = run;
            }
            run += d;
            ++nf;
        }
        if (tid == 0) soffs[nf] = run;
        __syncthreads();
    }
    const long long W = run;
    const bool push = fits && W <= pp.wmax;
    if (blockIdx.x == 0 && tid == 0) {
        pp.ctrl[0] = W;
        pp.ctrl[1] = nf;
        pp.ctrl[2] = 0;  // the third step's frontier list starts empty
        pp.ctrl[3] = 0;
        *pp.flag3 = 0;
        *pp.flag4 = 0;
        *pp.flag = push ? 1 : 0;
        // the restart term of y2 (other blocks may already be adding to the row)
        if (push) atomicAdd(&pp.acc[zrow(p, s)], to_fixed62(a_w ? p.c : p.c * p.inv[s]));
    }
    if (!push) {
        // step 2 will be pulled: y1 densely, as the gathered vector that the
        // step reads (the first step's output)
        float *y1 = p.zout;
        for (int64_t v = blockIdx.x * (int64_t)blockDim.x + tid; v < p.n; v += (int64_t)gridDim.x * blockDim.x) {
            float val = 0.0f;
            if (valid) {
                int64_t lo = e0, hi = e1;  // first edge with a_col >= v
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (a_col[mid] < v) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < e1 && a_col[lo] == v) {
                    const float y = fmaf(cw, a_w ? a_w[lo] : p.inv[s], v == (int64_t)s ? p.c : 0.0f);
                    val = a_w ? y : y * p.inv[v];
                } else if (v == (int64_t)s) {
                    val = a_w ? p.c : p.c * p.inv[s];
                }
            }
            y1[zrow(p, v)] = val;
        }
        return;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + tid; t < W; t += stride) {
        int lo = 0, hi = nf;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (soffs[mid] <= t) lo = mid;
            else hi = mid;
        }
        const int64_t e = sest[lo] + (t - soffs[lo]);
        const float zu = sy[lo];
        const int32_t v = a_col[e];
        // (1-c) x1 term of row v, as its gathered value (times 1/outdeg(v)
        // for uniform weights)
        const float term = a_w ? p.omc * (zu * a_w[e]) : (p.omc * zu) * p.inv[v];
        atomicAdd(&pp.acc[zrow(p, v)], to_fixed62(term));
    }
}

// ------------------------------------------------------------ pushed third step
// Whether step 3 of the current single-seed query is pushed: step 2 was,
// and its support's out-edges and pieces are within the limits.  The
// counters are final once the list launch has ended.
__device__ __forceinline__ bool third_pushed(const PushPlan &pp) {
    return pp.wmax3 > 0 && *pp.flag && pp.ctrl[2] <= pp.wmax3 && pp.ctrl[3] <= pp.qmax3;
}

// The frontier list of y2: every row set in bits (written by the step-2
// conversion) gives its node u (through zinv, the node at each gather row)
// and ceil(outdeg(u) / kTilePiece) pieces.  Threads take rows (row r of
// round i at r = (i * gridDim.x + block) * 256 + thread), so the live rows'
// lookups run in parallel; each block walks its rows twice, first counting
// its pieces and out-edges (one block scan, one atomic per counter for the
// whole block: counters that every wave bumped serialised the list), then
// writing the pieces from its reserved base.  The list order is arbitrary;
// the fixed-point sums do not depend on it.
__device__ __forceinline__ bool list_row(const PushPlan &pp, const int32_t *zinv, const int64_t *a_rowptr, int64_t zr,
                                         int64_t n, int64_t &u, int64_t &deg) {
    if (zr >= n || !((pp.bits[zr >> 5] >> (zr & 31)) & 1u)) return false;
    u = zinv ? (int64_t)zinv[zr] : zr;
    deg = a_rowptr[u + 1] - a_rowptr[u];
    return true;
}

__global__ __launch_bounds__(256) void frontier_list_kernel(StepParams p, PushPlan pp, const int64_t *a_rowptr,
                                                            const int32_t *zinv) {
    __shared__ long long swq[4], sww[4];
    __shared__ long long sbase;
    __shared__ int sover;
    if (!*pp.flag || pp.wmax3 <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t r0 = (int64_t)blockIdx.x * 256 + tid;
    // past the limit the step is pulled: nothing to list (one read for the
    // whole block, so that every wave meets the barriers below)
    if (tid == 0) sover = __hip_atomic_load(&pp.ctrl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > pp.wmax3;
    __syncthreads();
    if (sover) return;
    long long tq = 0, tw = 0;  // this thread's pieces and out-edges
    constexpr int R = 8;       // rows whose bitmap words are read together
    for (int64_t zb = r0; zb < p.n; zb += R * stride) {
        bool live[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int64_t zr = zb + i * stride;
            live[i] = zr < p.n && ((pp.bits[zr >> 5] >> (zr & 31)) & 1u);
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            int64_t u = 0, deg = 0;
            if (live[i] && list_row(pp, zinv, a_rowptr, zb + i * stride, p.n, u, deg)) {
                tq += (deg + kTilePiece - 1) / kTilePiece;
                tw += deg;
            }
        }
    }
    const long long iq = wave_scan_incl(tq, lane);
    const long long iw = wave_scan_incl(tw, lane);
    if (lane == 63) {
        swq[wv] = iq;
        sww[wv] = iw;
    }
    __syncthreads();
    long long before = 0, bq = 0, bw = 0;
    for (int w = 0; w < 4; ++w) {
        if (w < wv) before += swq[w];
        bq += swq[w];
        bw += sww[w];
    }
    if (tid == 0) {
        sbase = bq ? (long long)atomicAdd(reinterpret_cast<unsigned long long *>(&pp.ctrl[3]), (unsigned long long)bq) : 0;
        const long long wsum =
            bw ? (long long)atomicAdd(reinterpret_cast<unsigned long long *>(&pp.ctrl[2]), (unsigned long long)bw) + bw : 0;
        sover = wsum > pp.wmax3;  // already past the limit: the pieces will not be pushed
    }
    __syncthreads();
    if (bq == 0 || sover) return;
    long long q = sbase + before + iq - tq;  // this thread's first piece
    if (tq == 0) return;
    for (int64_t zb = r0; zb < p.n; zb += R * stride) {  // the same rows in the same order
#pragma unroll
        for (int i = 0; i < R; ++i) {
            int64_t u = 0, deg = 0;
            if (list_row(pp, zinv, a_rowptr, zb + i * stride, p.n, u, deg))
                for (int64_t off = 0; off < deg; off += kTilePiece, ++q)
                    if (q < pp.qmax3) pp.pieces3[q] = (long long)(u << 32) | off;
        }
    }
}

// The pushed third step: waves stride over the pieces; each lane adds its
// edge's (1-c) term of y2 (gathered from p.zin) to acc at the destination's
// gather row in 2^62 fixed point; one thread adds the restart term c e_s.
// The terms of y3 add up to at most its mass, below 1.
__global__ __launch_bounds__(256) void push_third_kernel(StepParams p, PushPlan pp, const int64_t *a_rowptr,
                                                         const int32_t *a_col, const float *a_w) {
    if (!third_pushed(pp)) return;
    const int lane = threadIdx.x & 63;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int32_t s = p.seeds[0];
        atomicAdd(&pp.acc[zrow(p, s)], to_fixed62(a_w ? p.c : p.c * p.inv[s]));
        *pp.flag3 = 1;
        *pp.flag4 = pp.ctrl[2] <= p.n / 16 ? 1 : 0;
    }
    const int64_t nq = pp.ctrl[3];
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; q < nq; q += nwaves) {
        const long long pc = pp.pieces3[q];
        const int64_t u = pc >> 32;
        const int64_t e0 = a_rowptr[u] + (pc & 0xffffffffll);
        const int64_t e1 = min(e0 + (int64_t)kTilePiece, a_rowptr[u + 1]);
        const float zu = p.zin[zrow(p, u)];
        for (int64_t e = e0 + lane; e < e1; e += 64) {
            const int32_t v = a_col[e];
            const float term = a_w ? p.omc * (zu * a_w[e]) : (p.omc * zu) * p.inv[v];
            atomicAdd(&pp.acc[zrow(p, v)], to_fixed62(term));
        }
    }
}

// y3 from acc as the next gathered vector, every row (acc cleared), and the
// rows of its support in the frontier bitmap.  Nothing unless step 3 was
// pushed (flag3 is cleared by the next query's first launch).
__global__ __launch_bounds__(256) void convert_third_kernel(StepParams p, PushPlan pp) {
    if (!*pp.flag3) return;
    // y3's support into the frontier bitmap as well, for step 4's skip
    const int lane = threadIdx.x & 63;
    const bool vec = (reinterpret_cast<uintptr_t>(p.zout) & 15) == 0;
    const int64_t first = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 256;
    const int64_t step = (((int64_t)gridDim.x * blockDim.x) >> 6) * 256;
    for (int64_t base = first; base < p.n; base += step)  // wave-uniform trip count
        convert_span(p, pp, base, lane, vec);
}

// ------------------------------------------------------------ pushed tiles
// Plan of a seed tile's pushed second step (one block of 1024 threads).
// Column j holds d_j + 1 entries when its seed row has no self-loop (the
// out-neighbours in edge order, then the seed itself), d_j otherwise; an
// invalid seed or a column past ncols holds none.  Entry i gets its node's
// y1 in gathered form, as the first step's push writes it, and its A~
// edges; its edges are cut into pieces of kTilePiece, whose indices come
// from a block scan.  Block-uniform loops throughout (the scans need every
// wave at each barrier).
__global__ __launch_bounds__(1024) void tile_plan_kernel(StepParams p, const int64_t *a_rowptr, const int32_t *a_col,
                                                         const float *a_w, TilePush tp) {
    __shared__ long long cstart[65];  // first entry of column j
    __shared__ long long swq[16], sww[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (wv == 0) {
        long long cnt = 0;
        if (lane < p.ncols) {
            const int32_t s = p.seeds[lane];
            if (s >= 0 && (int64_t)s < p.n) {
                const int64_t e0 = a_rowptr[s], e1 = a_rowptr[s + 1];
                int64_t lo = e0, hi = e1;  // first edge with a_col >= s (rows are sorted)
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (a_col[mid] < s) lo = mid + 1;
                    else hi = mid;
                }
                cnt = (e1 - e0) + ((lo < e1 && a_col[lo] == s) ? 0 : 1);
            }
        }
        const long long incl = wave_scan_incl(cnt, lane);
        cstart[lane + 1] = incl;
        if (lane == 0) cstart[0] = 0;
    }
    __syncthreads();
    const long long P = cstart[64];
    const float cw = p.c * p.omc;
    long long runq = 0, runw = 0;
    const bool fits = P > 0 && P <= kTilePlanMax;
    if (fits) {
        for (long long base = 0; base < P; base += 1024) {  // block-uniform trip count
            const long long i = base + tid;
            long long deg = 0, npc = 0;
            if (i < P) {
                int lo = 0, hi = 64;  // column: the last j with cstart[j] <= i
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (cstart[mid] <= i) lo = mid;
                    else hi = mid;
                }
                const int j = lo;
                const int32_t s = p.seeds[j];
                const int64_t e0 = a_rowptr[s], d = a_rowptr[s + 1] - e0;
                const long long l = i - cstart[j];
                int32_t f = s;
                float y = p.c;
                if (l < d) {
                    f = a_col[e0 + l];
                    y = fmaf(cw, a_w ? a_w[e0 + l] : p.inv[s], f == s ? p.c : 0.0f);
                }
                const int64_t f0 = a_rowptr[f], f1 = a_rowptr[f + 1];
                tp.ent_e0[i] = f0;
                tp.ent_e1[i] = f1;
                tp.ent_y[i] = a_w ? y : y * p.inv[f];
                tp.ent_col[i] = j;
                deg = f1 - f0;
                npc = (deg + kTilePiece - 1) / kTilePiece;
            }
            const long long iq = wave_scan_incl(npc, lane);
            const long long iw = wave_scan_incl(deg, lane);
            if (lane == 63) {
                swq[wv] = iq;
                sww[wv] = iw;
            }
            __syncthreads();
            long long q0 = runq + iq - npc;
            for (int w = 0; w < wv; ++w) q0 += swq[w];
            for (long long k = 0; k < npc; ++k)
                if (q0 + k < tp.qmax) tp.pieces[q0 + k] = (long long)(i << 32) | (k * kTilePiece);
            for (int w = 0; w < 16; ++w) {
                runq += swq[w];
                runw += sww[w];
            }
            __syncthreads();  // swq, sww are rewritten next round
        }
    }
    const bool push = fits && runw <= tp.wmax && runq <= tp.qmax;
    if (tid == 0) {
        tp.ctrl[0] = runw;
        tp.ctrl[1] = push ? runq : 0;
        tp.ctrl[2] = P;
        *tp.flag = push ? 1 : 0;
    }
    // the restart terms c e_s of y2, and their rows (the push adds to them
    // in a later launch)
    if (push && tid < p.ncols) {
        const int32_t s = p.seeds[tid];
        if (s >= 0 && (int64_t)s < p.n) {
            const int64_t zr = zrow(p, s);
            atomicAdd(&tp.acc[zr * p.kt + tid], to_fixed62(a_w ? p.c : p.c * p.inv[s]));
            tp.mark[zr] = 1;
        }
    }
}

// The pushed second step of a seed tile: waves stride over the plan's
// pieces; lanes take a piece's edges in order and add each edge's term of
// column j to acc in 2^62 fixed point (no atomic result awaited), marking
// its row with a byte store (an atomic OR into a bitmap word, which the
// rows of 32 hub-ranked nodes share, serialises: it tripled the launch).
// Every term lies in [0, 1] and column j's terms add up to at most the mass
// of its y2, below 1, so no sum overflows.
__global__ __launch_bounds__(256) void tile_push_kernel(StepParams p, const int32_t *a_col, const float *a_w,
                                                        TilePush tp) {
    if (!*tp.flag) return;
    const int lane = threadIdx.x & 63;
    const int64_t nq = tp.ctrl[1];
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; q < nq; q += nwaves) {
        const long long pc = tp.pieces[q];
        const int i = (int)(pc >> 32);
        const int64_t e0 = tp.ent_e0[i] + (pc & 0xffffffffll);
        const int64_t e1 = min(e0 + (int64_t)kTilePiece, tp.ent_e1[i]);
        const int j = tp.ent_col[i];
        const float zu = tp.ent_y[i];
        for (int64_t e = e0 + lane; e < e1; e += 64) {
            const int32_t v = a_col[e];
            const float term = a_w ? p.omc * (zu * a_w[e]) : (p.omc * zu) * p.inv[v];
            const int64_t zr = zrow(p, v);
            atomicAdd(&tp.acc[zr * p.kt + j], to_fixed62(term));
            tp.mark[zr] = 1;
        }
    }
}

// y2 of a pushed tile as the next gathered vector: rows the push reached
// are converted from acc (which is cleared), the others are zero.  Four
// entries per thread: one row's (kt >= 4, 16-byte accesses), else one at a
// time.
__global__ __launch_bounds__(256) void tile_convert_kernel(StepParams p, TilePush tp) {
    if (!*tp.flag) return;
    const int kt = p.kt;
    const int64_t total = p.n * (int64_t)kt;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
    for (int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i0 < total; i0 += stride) {
        if (kt >= 4) {
            const int64_t zr = i0 / kt;
            const bool live = tp.mark[zr] != 0;
            float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
            if (live) {
                ulonglong2 *a = reinterpret_cast<ulonglong2 *>(tp.acc + i0);
                const ulonglong2 lo = a[0], hi = a[1];
                z = make_float4((float)((double)lo.x * 0x1p-62), (float)((double)lo.y * 0x1p-62),
                                (float)((double)hi.x * 0x1p-62), (float)((double)hi.y * 0x1p-62));
                if (lo.x | lo.y) a[0] = make_ulonglong2(0ull, 0ull);
                if (hi.x | hi.y) a[1] = make_ulonglong2(0ull, 0ull);
            }
            *reinterpret_cast<float4 *>(p.zout + i0) = z;
        } else {
            for (int k = 0; k < 4 && i0 + k < total; ++k) {
                const int64_t i = i0 + k, zr = i / kt;
                float z = 0.0f;
                if (tp.mark[zr]) {
                    const unsigned long long a = tp.acc[i];
                    z = (float)((double)a * 0x1p-62);
                    if (a) tp.acc[i] = 0ull;
                }
                p.zout[i] = z;
            }
        }
    }
}

__global__ void fill_zero_gated_kernel(float *z, int64_t n, const int32_t *skip_on) {
    if (skip_on && *skip_on) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        z[i] = 0.0f;
}

__global__ void combine_only_kernel(StepParams p) {
    const int64_t total = p.n * (int64_t)p.ncols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(i / p.n);
        const int64_t v = i - (int64_t)j * p.n;
        int32_t seed = -1;
        float y;
        if (p.qdense) {
            y = p.c * p.qdense[(int64_t)j * p.n + v];
        } else {
            seed = seed_of(p, v, j);
            y = (v == (int64_t)seed) ? p.c : 0.0f;
        }
        float o;
        if (p.qdense || seed_valid(p, v, seed)) {
            o = fmaf(p.alpha, y, p.str[v]);
        } else {
            o = qnan();
            *p.err = 1;
        }
        p.out[(p.out_col0 + j) * p.n + v] = o;
    }
}

inline unsigned blocks_for(int64_t waves) { return (unsigned)((waves + kWaves - 1) / kWaves); }

inline unsigned grid_1d(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 20));
}

// tiles of 2..16 columns: the last family step stages its outputs (a
// 32-column stage takes 34 KB of LDS per block, and the occupancy it costs
// made that step slower than the unstaged one)
#define KT_LAUNCH(K)                                                                                   \
    do {                                                                                               \
        if (MODE == kFamily && p.last && (K) <= 16)                                                    \
            last_step_kernel_kt<K, FIRST, WEIGHTED><<<grid, kThreads, 0, st>>>(it, ni, p);             \
        else                                                                                           \
            step_kernel_kt<K, MODE, FIRST, WEIGHTED><<<grid, kThreads, 0, st>>>(it, ni, p);            \
    } while (0)

template <int MODE, bool FIRST, bool WEIGHTED>
void launch_kt(const Schedule &s, const StepParams &p, hipStream_t st) {
    const unsigned grid = blocks_for(s.n_items);
    const Item *it = s.items;
    const int64_t ni = s.n_items;
    switch (p.kt) {
        case 1:
            if constexpr (!FIRST && !WEIGHTED) {
                if (s.chunk_slot_in_item) {
                    step_kernel_1x<MODE><<<grid, kThreads, 0, st>>>(it, ni, p);
                    break;
                }
            }
            step_kernel_1<MODE, FIRST, WEIGHTED><<<grid, kThreads, 0, st>>>(it, ni, p);
            break;
        case 2: KT_LAUNCH(2); break;
        case 4: KT_LAUNCH(4); break;
        case 8: KT_LAUNCH(8); break;
        case 16: KT_LAUNCH(16); break;
        case 32: KT_LAUNCH(32); break;
        case 64: {
            const int walk = FIRST ? 2 : p.bits ? (p.bits_on ? 0 : 1) : 2;
            if (walk == 0) step_kernel_64<MODE, FIRST, WEIGHTED, 0><<<grid, kThreads, 0, st>>>(it, ni, p);
            else if (walk == 1) step_kernel_64<MODE, FIRST, WEIGHTED, 1><<<grid, kThreads, 0, st>>>(it, ni, p);
            else step_kernel_64<MODE, FIRST, WEIGHTED, 2><<<grid, kThreads, 0, st>>>(it, ni, p);
            break;
        }
        default: break;
    }
}

template <int MODE, bool FIRST>
void launch_w(const Schedule &s, const StepParams &p, hipStream_t st) {
    if (p.w) launch_kt<MODE, FIRST, true>(s, p, st);
    else launch_kt<MODE, FIRST, false>(s, p, st);
}

}  // namespace

namespace {

// The single-vector kernels read a schedule's group-ordered column ids in
// place of the hub-first ones they were built from, and take the chunk
// slots of an XCD-sliced schedule from its items.
StepParams with_group_order(const Schedule &s, const StepParams &p) {
    StepParams q = p;
    q.col_slots = 0;
    q.chunk_slot_in_item = s.chunk_slot_in_item ? 1 : 0;
    q.rowptr_x = s.rowptr_x;
    q.xrel = s.xrel;
    if (q.kt == 1 && s.colg && q.col == s.colg_src) {
        q.col = s.colg;
        q.col_slots = 1;
    }
    return q;
}

}  // namespace

tpa_status launch_step(const Schedule &s, int mode, bool first, const StepParams &p0, hipStream_t st) {
    const StepParams p = with_group_order(s, p0);
    if (p.kt != 1 && p.kt != 2 && p.kt != 4 && p.kt != 8 && p.kt != 16 && p.kt != 32 && p.kt != 64)
        return fail(TPA_ERR_INVALID_ARG, "seed tile must be 1, 2, 4, 8, 16, 32 or 64");
    if (mode == kStranger && p.kt != 1) return fail(TPA_ERR_INVALID_ARG, "stranger step is single-column");
    if (s.chunk_slot_in_item && (p.kt != 1 || first || p.w))
        return fail(TPA_ERR_INVALID_ARG, "an XCD-sliced schedule takes single-column pulls with 1/outdeg weights");
    if (p.kt == 1 && s.ew > kGroupMax) return fail(TPA_ERR_INVALID_ARG, "group items exceed the LDS slice");
    if (p.kt != 1 && s.eb > s.el) return fail(TPA_ERR_INVALID_ARG, "block items need a single-column step");
    if ((uint64_t)blocks_for(s.n_items) * kThreads > UINT32_MAX)
        return fail(TPA_ERR_INDEX_OVERFLOW, "too many work items for one launch");
    if (s.n_items > 0) {
        int lg = 0;
        while ((1 << lg) < p.kt) ++lg;
        // the last family step of a single seed and of tiles of 16 and 64 has its own code
        const bool last_code = mode == kFamily && p.last && (p.kt == 1 || p.kt == 16 || p.kt == 64);
        // and a pull launched under a device-side gate (empty when the device
        // pushed that step) has one shared code, so that the others time
        // only steps that ran
        const int code = p.skip_on ? 118 + (p.w ? 1 : 0)
                         : last_code ? 112 + 2 * (p.kt == 1 ? 0 : p.kt == 16 ? 1 : 2) + (p.w ? 1 : 0)
                                     : 16 * lg + 4 * mode + 2 * (first ? 1 : 0) + (p.w ? 1 : 0);
        const int slot = profile_begin(code, st);
        if (mode == kFamily) {
            if (first) launch_w<kFamily, true>(s, p, st);
            else launch_w<kFamily, false>(s, p, st);
        } else if (mode == kPlain) {
            if (first) launch_w<kPlain, true>(s, p, st);
            else launch_w<kPlain, false>(s, p, st);
        } else {
            launch_w<kStranger, false>(s, p, st);
        }
        profile_end(slot, st);
    }
    if (s.n_long > 0 && s.chunk_slot_in_item) {
        const int slot = profile_begin(127, st);
        const unsigned grid = blocks_for((s.n_long + 7) / 8);
        if (mode == kFamily)
            finish_long8_kernel<kFamily><<<grid, kThreads, 0, st>>>(s.longs, s.n_long, p);
        else if (mode == kPlain)
            finish_long8_kernel<kPlain><<<grid, kThreads, 0, st>>>(s.longs, s.n_long, p);
        else
            finish_long8_kernel<kStranger><<<grid, kThreads, 0, st>>>(s.longs, s.n_long, p);
        profile_end(slot, st);
    } else if (s.n_long > 0) {
        const int slot = profile_begin(127, st);
        if (mode == kFamily)
            finish_kernel<kFamily><<<blocks_for(s.n_long), kThreads, 0, st>>>(s.longs, s.n_long, p);
        else if (mode == kPlain)
            finish_kernel<kPlain><<<blocks_for(s.n_long), kThreads, 0, st>>>(s.longs, s.n_long, p);
        else
            finish_kernel<kStranger><<<blocks_for(s.n_long), kThreads, 0, st>>>(s.longs, s.n_long, p);
        profile_end(slot, st);
    }
    if (s.n_long8 > 0) {
        const int slot = profile_begin(127, st);
        const unsigned grid = (unsigned)((s.n_long8 + kThreads - 1) / kThreads);
        if (mode == kFamily)
            finish8_kernel<kFamily><<<grid, kThreads, 0, st>>>(s.longs8, s.n_long8, p);
        else if (mode == kPlain)
            finish8_kernel<kPlain><<<grid, kThreads, 0, st>>>(s.longs8, s.n_long8, p);
        else
            finish8_kernel<kStranger><<<grid, kThreads, 0, st>>>(s.longs8, s.n_long8, p);
        profile_end(slot, st);
    }
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_stranger_init(const tpa_graph *g, float c, int include_x0, float *zout, float *acc,
                                float *comp, const int32_t *zperm, hipStream_t st) {
    stranger_init_kernel<<<grid_1d(g->n), 256, 0, st>>>(g->n, c, g->restart_pr, (float)(1.0 / (double)g->n),
                                                         g->inv_deg, g->t.w, include_x0, zout, acc, comp, zperm);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_dense_init(const StepParams &p, float *z0, float *x0, hipStream_t st) {
    dense_init_kernel<<<grid_1d(p.n * (int64_t)p.kt), 256, 0, st>>>(p, z0, x0);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_dense_transpose(const StepParams &p, float *qT, hipStream_t st) {
    if (!p.qdense || !qT || p.kt < 1 || p.kt > 64) return fail(TPA_ERR_INVALID_ARG, "dense transpose needs q and kt <= 64");
    const int64_t blocks = (p.n + kTransNodes - 1) / kTransNodes;
    if (blocks > UINT32_MAX) return fail(TPA_ERR_INDEX_OVERFLOW, "too many nodes for one launch");
    if (blocks > 0) dense_transpose_kernel<<<(unsigned)blocks, 256, 0, st>>>(p, qT);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

// One block per 64 nodes: read the tile block (coalesced), write each
// column's run of 64 entries (coalesced).
__global__ __launch_bounds__(256) void tile_to_rows_kernel(const float *tile, int kt, int ncols, int64_t n,
                                                           const int32_t *seeds, float *out, int64_t col0,
                                                           int32_t *err) {
    __shared__ float blk[64][64 + 1];
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    const int64_t nv = min((int64_t)64, n - v0);
    for (int i = threadIdx.x; i < nv * kt; i += blockDim.x) {
        const int vl = i / kt, j = i - vl * kt;
        blk[j][vl] = tile[(v0 + vl) * kt + j];
    }
    __syncthreads();
    const int t = threadIdx.x & 63, r = threadIdx.x >> 6;
    for (int j = r; j < ncols; j += 4) {
        bool ok = true;
        if (seeds) {
            const int32_t sd = seeds[j];
            ok = sd >= 0 && (int64_t)sd < n;
        }
        if (t < nv) out[(col0 + j) * n + v0 + t] = ok ? blk[j][t] : qnan();
        if (!ok && t == 0 && blockIdx.x == 0) *err = 1;
    }
}

tpa_status launch_tile_to_rows(const float *tile, int kt, int ncols, int64_t n, const int32_t *seeds, float *out,
                               int64_t col0, int32_t *err, hipStream_t st) {
    if (kt < 1 || kt > 64 || ncols < 0 || ncols > kt) return fail(TPA_ERR_INVALID_ARG, "bad tile shape");
    const int64_t blocks = (n + 63) / 64;
    if (blocks > UINT32_MAX) return fail(TPA_ERR_INDEX_OVERFLOW, "too many nodes for one launch");
    if (blocks > 0 && ncols > 0)
        tile_to_rows_kernel<<<(unsigned)blocks, 256, 0, st>>>(tile, kt, ncols, n, seeds, out, col0, err);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_fill_zero(float *z, int64_t n, hipStream_t st) {
    if (n > 0) fill_zero_kernel<<<grid_1d(n), 256, 0, st>>>(z, n);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_onehot_init(const StepParams &p, float *x0, hipStream_t st) {
    onehot_init_kernel<<<grid_1d(p.n * (int64_t)p.kt), 256, 0, st>>>(p, x0);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_push_first(const StepParams &p, const tpa_graph *g, int64_t nblocks, uint32_t *bits,
                             int64_t nwords, hipStream_t st) {
    const int64_t nslots = nblocks * p.ncols;
    const unsigned slot_grid = (unsigned)((nslots * 64 + 255) / 256);
    if (bits) {
        fill_zero_gated_kernel<<<grid_1d(nwords), 256, 0, st>>>(reinterpret_cast<float *>(bits), nwords, p.skip_on);
        push_first_rows_kernel<<<slot_grid, 256, 0, st>>>(p, g->a.rowptr, g->a.col, nslots, bits);
    } else {
        fill_zero_gated_kernel<<<grid_1d(p.n * (int64_t)p.kt), 256, 0, st>>>(p.zout, p.n * (int64_t)p.kt,
                                                                             p.skip_on);
    }
    push_first_kernel<<<slot_grid, 256, 0, st>>>(p, g->a.rowptr, g->a.col, g->weighted ? g->a.w : nullptr, nslots);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

namespace {
size_t bits_bytes(int64_t n) { return (((size_t)(n + 31) / 32) * 4 + 255) & ~(size_t)255; }
}  // namespace

// Pieces of the pushed third step: one or more per node of y2's support
// (at most 2^22 nodes counted), and one per kTilePiece of m/20 edges.
int64_t third_qmax(int64_t n, int64_t m) {
    return std::min<int64_t>(n, int64_t(1) << 22) + m / 20 / kTilePiece + 2;
}

size_t push_plan_clear_bytes(int64_t n) {
    const size_t a = ((size_t)n * 8 + 255) & ~(size_t)255;
    return a + 256 + bits_bytes(n);
}

size_t push_plan_bytes(int64_t n, int64_t m, bool third) {
    return push_plan_clear_bytes(n) + (third ? (((size_t)third_qmax(n, m) * 8 + 255) & ~(size_t)255) : 0);
}

PushPlan push_plan_at(void *base, int64_t n, int64_t m, int64_t wmax, int64_t wmax3) {
    char *b = static_cast<char *>(base);
    const size_t a = ((size_t)n * 8 + 255) & ~(size_t)255;
    PushPlan pp;
    pp.acc = reinterpret_cast<unsigned long long *>(b);
    pp.ctrl = reinterpret_cast<int64_t *>(b + a);
    pp.flag = reinterpret_cast<int32_t *>(b + a + 64);
    pp.flag3 = reinterpret_cast<int32_t *>(b + a + 68);
    pp.flag4 = reinterpret_cast<int32_t *>(b + a + 72);
    pp.bits = reinterpret_cast<uint32_t *>(b + a + 256);
    pp.nwords = (n + 31) / 32;
    pp.wmax = wmax;
    pp.pieces3 = reinterpret_cast<int64_t *>(b + push_plan_clear_bytes(n));
    pp.qmax3 = wmax3 > 0 ? third_qmax(n, m) : 0;
    pp.wmax3 = wmax3;
    return pp;
}

namespace {
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
// pieces: one or more per plan entry, up to 4m frontier edges in all
int64_t tile_qmax(int64_t m) { return 4 * (m / kTilePiece + 1) + kTilePlanMax; }
}  // namespace

size_t tile_push_bytes(int64_t n, int64_t m, int kt) {
    const size_t P = kTilePlanMax;
    return align256((size_t)n * kt * 8) + align256((size_t)n) + 256 + align256(P * 8) * 2 + align256(P * 4) * 2 +
           align256((size_t)tile_qmax(m) * 8);
}

TilePush tile_push_at(void *base, int64_t n, int64_t m, int kt, int64_t wmax) {
    char *b = static_cast<char *>(base);
    const size_t P = kTilePlanMax;
    TilePush tp;
    tp.acc = reinterpret_cast<unsigned long long *>(b);
    b += align256((size_t)n * kt * 8);
    tp.mark = reinterpret_cast<uint8_t *>(b);
    b += align256((size_t)n);
    tp.ctrl = reinterpret_cast<int64_t *>(b);
    tp.flag = reinterpret_cast<int32_t *>(b + 64);
    b += 256;
    tp.ent_e0 = reinterpret_cast<int64_t *>(b);
    b += align256(P * 8);
    tp.ent_e1 = reinterpret_cast<int64_t *>(b);
    b += align256(P * 8);
    tp.ent_y = reinterpret_cast<float *>(b);
    b += align256(P * 4);
    tp.ent_col = reinterpret_cast<int32_t *>(b);
    b += align256(P * 4);
    tp.pieces = reinterpret_cast<int64_t *>(b);
    tp.qmax = tile_qmax(m);
    tp.wmax = wmax;
    return tp;
}

tpa_status launch_tile_plan(const StepParams &p, const tpa_graph *g, const TilePush &tp, hipStream_t st) {
    if (p.kt < 2 || p.node_block || !p.seeds || p.ncols > 64) return fail(TPA_ERR_INVALID_ARG, "tile push needs seed lists");
    const int slot = profile_begin(122, st);
    const int64_t mwords = (p.n + 3) / 4;  // mark as 4-byte words (its bytes are 256-aligned)
    fill_zero_kernel<<<grid_1d(mwords), 256, 0, st>>>(reinterpret_cast<float *>(tp.mark), mwords);
    tile_plan_kernel<<<1, 1024, 0, st>>>(p, g->a.rowptr, g->a.col, g->weighted ? g->a.w : nullptr, tp);
    profile_end(slot, st);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_tile_push(const StepParams &p, const tpa_graph *g, const TilePush &tp, hipStream_t st) {
    // waves stride over the pieces: about 4 pieces per wave at the bound
    const int64_t blocks = std::min<int64_t>(std::max<int64_t>(1, (tp.wmax / kTilePiece + kTilePlanMax) / 16), 2048);
    const int slot = profile_begin(123, st);
    tile_push_kernel<<<(unsigned)blocks, 256, 0, st>>>(p, g->a.col, g->weighted ? g->a.w : nullptr, tp);
    profile_end(slot, st);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_tile_convert(const StepParams &p, const TilePush &tp, hipStream_t st) {
    const int64_t total = p.n * (int64_t)p.kt;
    const int slot = profile_begin(125, st);
    tile_convert_kernel<<<grid_1d((total + 3) / 4), 256, 0, st>>>(p, tp);
    profile_end(slot, st);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_push_steps12(const StepParams &p, const tpa_graph *g, const PushPlan &pp, hipStream_t st) {
    if (p.kt != 1 || p.node_block || !p.seeds) return fail(TPA_ERR_INVALID_ARG, "push plan needs a single unpacked seed");
    // grid-stride over the W edge slots: about 16 slots per thread up to the bound
    const int64_t blocks = std::min<int64_t>(std::max<int64_t>(1, (pp.wmax + 16 * 256 - 1) / (16 * 256)), 4096);
    const int slot = profile_begin(124, st);
    push_steps12_kernel<<<(unsigned)blocks, 256, 0, st>>>(p, g->a.rowptr, g->a.col, g->weighted ? g->a.w : nullptr,
                                                          pp);
    profile_end(slot, st);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_gated_step(const Schedule &s, const StepParams &p0, const PushPlan &pp, hipStream_t st) {
    const StepParams p = with_group_order(s, p0);
    if (p.kt != 1 || p.node_block || !p.seeds || p.last)
        return fail(TPA_ERR_INVALID_ARG, "a gated step is a single-seed non-last family step");
    if (s.ew > kGroupMax) return fail(TPA_ERR_INVALID_ARG, "group items exceed the LDS slice");
    if ((uint64_t)blocks_for(s.n_items) * kThreads > UINT32_MAX)
        return fail(TPA_ERR_INDEX_OVERFLOW, "too many work items for one launch");
    if (s.n_items > 0) {
        const int slot = profile_begin(120 + (p.w ? 1 : 0), st);
        const unsigned grid = blocks_for(s.n_items);  // one slot per block: the pushed case converts in parallel
        if (p.w) gated_step_kernel_1<true><<<grid, kThreads, 0, st>>>(s.items, s.n_items, p, pp);
        else gated_step_kernel_1<false><<<grid, kThreads, 0, st>>>(s.items, s.n_items, p, pp);
        profile_end(slot, st);
    }
    if (s.n_long > 0) gated_finish_kernel<<<blocks_for(s.n_long), kThreads, 0, st>>>(s.longs, s.n_long, p, pp);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_push_third(const StepParams &p, const tpa_graph *g, const PushPlan &pp, hipStream_t st) {
    if (p.kt != 1 || p.node_block || !p.seeds || p.last)
        return fail(TPA_ERR_INVALID_ARG, "a pushed third step is a single-seed non-last family step");
    const int slot = profile_begin(126, st);
    const int64_t lblocks = std::max<int64_t>(1, std::min<int64_t>((p.n + 255) / 256, 1024));
    frontier_list_kernel<<<(unsigned)lblocks, 256, 0, st>>>(p, pp, g->a.rowptr, g->zperm && p.zperm ? g->zinv : nullptr);
    // waves stride over the pieces
    const int64_t blocks = std::min<int64_t>(std::max<int64_t>(1, pp.qmax3 / 16), 1024);
    push_third_kernel<<<(unsigned)blocks, 256, 0, st>>>(p, pp, g->a.rowptr, g->a.col, g->weighted ? g->a.w : nullptr);
    profile_end(slot, st);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_convert_third(const StepParams &p, const PushPlan &pp, hipStream_t st) {
    // a wave per 256-row span, at most 2048 blocks striding
    convert_third_kernel<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>((p.n + 1023) / 1024, 2048)), 256, 0, st>>>(p, pp);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status launch_combine_only(const StepParams &p, hipStream_t st) {
    combine_only_kernel<<<grid_1d(p.n * (int64_t)p.ncols), 256, 0, st>>>(p);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

}  // namespace tpa
