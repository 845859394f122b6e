// Exact RWR by CPI and the accuracy harness's device operations.
//
//   tpa_cpi    Algorithm 1 for one restart vector and any iteration window
//              [s_iter, t_iter]; s_iter = 0, t_iter = unbounded is exact RWR
//              up to the truncation eps (Theorem 1), and the windows
//              [0, S-1], [S, T-1], [T, unbounded] give the exact family,
//              neighbor and stranger parts that TPA approximates (Section 3,
//              Table 3's comparison).
//   tpa_topk   the k largest entries of each row, ties by smaller index (the
//              top-k lists whose recall the paper reports, Section 4).
//   tpa_row_l1 L1 distance per row, sum_v |a*x[v] - y[v]|, in FP64.

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "cpi_kernels.h"
#include "tpa_internal.h"

namespace tpa {
namespace {

// x(0) = c q (one-hot seed or dense q) as the gathered vector, r = x(0) when
// the window starts at 0, compensation zero.
__global__ void cpi_init_kernel(int64_t n, float c, int32_t seed, const float *q, const float *inv, int weighted,
                                int include_x0, const int32_t *zperm, float *zout, float *acc, float *comp) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const float x0 = q ? c * q[v] : (v == (int64_t)seed ? c : 0.0f);
        zout[zperm ? zperm[v] : v] = weighted ? x0 : x0 * inv[v];
        acc[v] = include_x0 ? x0 : 0.0f;
        comp[v] = 0.0f;
    }
}

// sum_v |q[v]| in FP64 for row blockIdx.x of q [rows][n], one block per
// row, fixed order.
__global__ void l1_norm_kernel(const float *q, int64_t n, double *out) {
    __shared__ double red[256];
    const float *qr = q + (int64_t)blockIdx.x * n;
    double s = 0.0;
    for (int64_t v = threadIdx.x; v < n; v += blockDim.x) s += fabs((double)qr[v]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Per-row L1 distance in two fixed-order passes: block (row, b) of a
// [rows x kL1Parts] grid reduces part b of the row into part[row][b]; then
// one thread per row adds its parts in order.  Deterministic for a given n.
constexpr int kL1Parts = 64;

__global__ void row_l1_parts_kernel(const float *x, const float *y, int64_t n, double a, double *part) {
    __shared__ double red[256];
    const int64_t row = blockIdx.y;
    const int64_t per = (n + kL1Parts - 1) / kL1Parts;
    const int64_t b0 = (int64_t)blockIdx.x * per, b1 = min(n, b0 + per);
    double s = 0.0;
    for (int64_t v = b0 + threadIdx.x; v < b1; v += blockDim.x)
        s += fabs(a * (double)x[row * n + v] - (double)y[row * n + v]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[row * kL1Parts + blockIdx.x] = red[0];
}

__global__ void row_l1_sum_kernel(const double *part, int64_t rows, double *out) {
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (row >= rows) return;
    double s = 0.0;
    for (int b = 0; b < kL1Parts; ++b) s += part[row * kL1Parts + b];
    out[row] = s;
}

// ------------------------------------------------------------------ top-k
// Order-preserving key of a float (larger value, larger key); -0 and +0 are
// one value; NaN maps to 0, below every number.
__device__ __forceinline__ uint32_t order_key(float f) {
    if (f != f) return 0u;
    const uint32_t b = f == 0.0f ? 0u : __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

constexpr int kTopkMax = 1024;

// hist[bin] += 1 for every active lane.  Lanes of a wave that share a bin
// (common in the top digits, where most values share an exponent) are
// counted with one atomic; after four shared bins the rest add one by one.
__device__ __forceinline__ void hist_add(uint32_t *hist, uint32_t bin, bool active) {
    const int lane = threadIdx.x & 63;
    uint64_t pending = __ballot(active);
    for (int it = 0; it < 4 && pending; ++it) {
        const int leader = __builtin_ctzll(pending);
        const uint32_t b = __builtin_amdgcn_readlane(bin, leader);
        const uint64_t same = __ballot(active && bin == b) & pending;
        if (lane == leader) atomicAdd(&hist[b], (uint32_t)__popcll(same));
        pending &= ~same;
    }
    if ((pending >> lane) & 1ull) atomicAdd(&hist[bin], 1u);
}

// One stage of the top-k selection.  Every input row is cut into segments
// of `seg` entries (seg >= k) and one block takes one segment.  Entry i of
// row r has key order_key(vals[r*len + i]) and index i on the first stage,
// keys/idx[r*len + i] on later ones.  A block writes its segment's
// min(k, segment length) best entries, sorted by (key descending, index
// ascending), at position segment*k of its output row (row length
// out_len), or, on the last stage (one segment per row), the final k
// indices and their values from the original rows.
struct TopkStage {
    const float *vals = nullptr;
    const uint32_t *keys = nullptr;
    const int32_t *idx = nullptr;
    int64_t len = 0;
    int64_t seg = 0;
    int64_t nseg = 0;
    int k = 0;
    uint32_t *out_keys = nullptr;
    int32_t *out_idx = nullptr;
    int64_t out_len = 0;
    const float *orig = nullptr;  // original rows [rows][n]
    int64_t n = 0;
    int32_t *idx_out = nullptr;
    float *val_out = nullptr;
};

__device__ __forceinline__ uint32_t stage_key(const TopkStage &t, int64_t at) {
    return t.vals ? order_key(t.vals[at]) : t.keys[at];
}

// Per block: a most-significant-digit-first radix select (four 8-bit digits)
// finds the key K of the segment's kk-th best entry; the entries above K are
// taken, then those equal to K in position order until kk are chosen (on
// every stage, equal keys sit in index order: segments cover increasing
// index ranges and each candidate list is sorted); a bitonic sort orders
// the kk pairs.
template <int NT>
__global__ __launch_bounds__(NT) void topk_stage_kernel(TopkStage t) {
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_prefix, s_need, s_count;
    __shared__ uint32_t skey[kTopkMax];
    __shared__ int32_t sidx[kTopkMax];
    __shared__ uint32_t scan[NT / 64];
    const int tid = threadIdx.x;
    const int64_t r = (int64_t)blockIdx.x / t.nseg, sg = (int64_t)blockIdx.x - r * t.nseg;
    const int64_t b0 = sg * t.seg;
    const int64_t m = min(t.len - b0, t.seg);  // entries of this segment
    const int kk = (int)min<int64_t>(t.k, m);
    const int64_t at0 = r * t.len + b0;        // first entry of the segment
    if (tid == 0) {
        s_prefix = 0u;
        s_need = (uint32_t)kk;
    }
    constexpr int UL = 8;  // loads in flight per thread
    for (int d = 0; d < 4; ++d) {
        const int shift = 24 - 8 * d;
        const uint32_t mask_hi = d == 0 ? 0u : (0xffffffffu << (shift + 8));
        for (int i = tid; i < 256; i += blockDim.x) hist[i] = 0u;
        __syncthreads();
        const uint32_t prefix = s_prefix;
        for (int64_t base = 0; base < m; base += (int64_t)blockDim.x * UL) {  // same trip count in every lane
            uint32_t key[UL];
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int64_t v = base + (int64_t)u * blockDim.x + tid;
                key[u] = v < m ? stage_key(t, at0 + v) : 0u;
            }
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int64_t v = base + (int64_t)u * blockDim.x + tid;
                hist_add(hist, (key[u] >> shift) & 255u, v < m && (key[u] & mask_hi) == prefix);
            }
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t need = s_need, acc = 0u;
            int b = 255;
            for (; b > 0; --b) {
                if (acc + hist[b] >= need) break;
                acc += hist[b];
            }
            s_prefix = prefix | ((uint32_t)b << shift);
            s_need = need - acc;
        }
        __syncthreads();
    }
    const uint32_t K = s_prefix;
    const uint32_t take_eq = s_need;  // entries equal to K to take, first positions first
    if (tid == 0) s_count = 0u;
    __syncthreads();
    // entries above K (fewer than kk of them), in any order
    for (int64_t base = 0; base < m; base += (int64_t)blockDim.x * UL) {
        uint32_t key[UL];
#pragma unroll
        for (int u = 0; u < UL; ++u) {
            const int64_t v = base + (int64_t)u * blockDim.x + tid;
            key[u] = v < m ? stage_key(t, at0 + v) : 0u;
        }
#pragma unroll
        for (int u = 0; u < UL; ++u) {
            const int64_t v = base + (int64_t)u * blockDim.x + tid;
            if (v < m && key[u] > K) {
                const uint32_t pos = atomicAdd(&s_count, 1u);
                skey[pos] = key[u];
                sidx[pos] = t.vals ? (int32_t)(b0 + v) : t.idx[at0 + v];
            }
        }
    }
    __syncthreads();
    const uint32_t above = s_count;
    // entries equal to K, the take_eq at the first positions: wave w owns the
    // contiguous part [w*part, (w+1)*part) and walks it 64 entries at a time
    // (coalesced); a scan of the per-wave counts gives each part its first
    // rank, and ballots rank the entries inside a chunk
    {
        const int wv = tid >> 6, lane = tid & 63;
        const int nw = (int)blockDim.x >> 6;
        const int64_t part = ((m + nw - 1) / nw + 63) & ~(int64_t)63;
        const int64_t s0 = (int64_t)wv * part, s1 = min(m, s0 + part);
        uint32_t cnt = 0u;
        for (int64_t v0 = s0; v0 < s1; v0 += 64) {
            const int64_t v = v0 + lane;
            cnt += (uint32_t)__popcll(__ballot(v < s1 && stage_key(t, at0 + v) == K));
        }
        if (lane == 0) scan[wv] = cnt;
        __syncthreads();
        uint32_t rank = 0u;
        for (int w = 0; w < wv; ++w) rank += scan[w];
        for (int64_t v0 = s0; v0 < s1 && rank < take_eq; v0 += 64) {
            const int64_t v = v0 + lane;
            const bool eq = v < s1 && stage_key(t, at0 + v) == K;
            const uint64_t mk = __ballot(eq);
            const uint32_t rk = rank + (uint32_t)__popcll(mk & ((1ull << lane) - 1ull));
            if (eq && rk < take_eq) {
                skey[above + rk] = K;
                sidx[above + rk] = t.vals ? (int32_t)(b0 + v) : t.idx[at0 + v];
            }
            rank += (uint32_t)__popcll(mk);
        }
    }
    __syncthreads();
    // bitonic sort of the kk pairs (padded to a power of two)
    int p2 = 1;
    while (p2 < kk) p2 <<= 1;
    for (int i = tid; i < p2; i += blockDim.x)
        if (i >= kk) {
            skey[i] = 0u;
            sidx[i] = INT32_MAX;
        }
    __syncthreads();
    for (int size = 2; size <= p2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < p2; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    // "before": larger key, then smaller index
                    const bool desc = (i & size) == 0;
                    const uint32_t ki = skey[i], kj = skey[j];
                    const int32_t ii = sidx[i], ij = sidx[j];
                    const bool j_first = kj > ki || (kj == ki && ij < ii);
                    if (j_first == desc) {
                        skey[i] = kj;
                        skey[j] = ki;
                        sidx[i] = ij;
                        sidx[j] = ii;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (t.idx_out) {
        for (int i = tid; i < kk; i += blockDim.x) {
            const int32_t v = sidx[i];
            t.idx_out[r * t.k + i] = v;
            t.val_out[r * t.k + i] = t.orig[r * t.n + v];
        }
    } else {
        const int64_t o = r * t.out_len + sg * t.k;
        for (int i = tid; i < kk; i += blockDim.x) {
            t.out_keys[o + i] = skey[i];
            t.out_idx[o + i] = sidx[i];
        }
    }
}

}  // namespace
}  // namespace tpa

using namespace tpa;

extern "C" tpa_status tpa_cpi(tpa_graph_t g, int32_t seed, const float *q, double c, int s_iter, int t_iter,
                              double eps, float *out, hipStream_t st) {
    if (!g || !out) return fail(TPA_ERR_INVALID_ARG, "NULL argument");
    if ((seed >= 0) == (q != nullptr)) return fail(TPA_ERR_INVALID_ARG, "pass exactly one of seed >= 0 and q");
    if (seed >= g->n) return fail(TPA_ERR_INVALID_ARG, "seed out of range");
    if (!(c > 0.0 && c < 1.0)) return fail(TPA_ERR_INVALID_ARG, "c must lie in (0, 1)");
    if (s_iter < 0 || t_iter < -1 || (t_iter >= 0 && t_iter < s_iter))
        return fail(TPA_ERR_INVALID_ARG, "need 0 <= s_iter <= t_iter, or t_iter = -1");
    if (!(eps >= 0.0) || (eps == 0.0 && t_iter < 0))
        return fail(TPA_ERR_INVALID_ARG, "eps must be >= 0, and > 0 without a last iteration");
    const int64_t n = g->n;
    // last iteration: Algorithm 1's L1 break at c (1-c)^i ||q||_1 < eps
    // (Lemma 2; exact for q >= 0), capped by t_iter
    int64_t K = t_iter >= 0 ? t_iter : INT64_MAX;
    if (eps > 0.0) {
        double qn = 1.0;
        if (q) {
            double *d = nullptr;
            TPA_TRY(dalloc(&d, 1, st));
            l1_norm_kernel<<<1, 256, 0, st>>>(q, n, d);
            hipError_t e = hipMemcpyAsync(&qn, d, sizeof(double), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            dfree(d);
            TPA_TRY_HIP(e);
        }
        if (qn > 0.0) K = std::min<int64_t>(K, stranger_last_iteration(c, eps / qn));
        else K = 0;
    }
    const Schedule *s = nullptr;
    TPA_TRY(get_schedule(g, choose_shape(g, 1), st, &s));
    if (g->gather_layout) {
        TPA_TRY(ensure_zlayout(g, st));
        TPA_TRY(ensure_wz(g, st));
    }
    const bool hub = g->gather_layout && g->zperm && (!g->weighted || g->t_wz_valid);
    if (hub) TPA_TRY(ensure_group_order(g, s, st));
    float *tmp = nullptr;
    TPA_TRY(dalloc(&tmp, 3 * (size_t)n + (size_t)std::max<int64_t>(s->n_chunk_items, 1), st));
    float *z0 = tmp, *z1 = tmp + n, *comp = tmp + 2 * n, *part = tmp + 3 * n;
    cpi_init_kernel<<<std::min<int64_t>((n + 255) / 256, 1 << 20), 256, 0, st>>>(
        n, (float)c, seed, q, g->inv_deg, g->weighted ? 1 : 0, s_iter == 0 ? 1 : 0, hub ? g->zperm : nullptr, z0,
        out, comp);
    tpa_status rc = TPA_OK;
    if (hipGetLastError() != hipSuccess) rc = fail(TPA_ERR_HIP, "cpi init launch failed");
    StepParams p;
    p.rowptr = g->t.rowptr;
    p.col = hub ? g->t_colz : g->t.col;
    p.zperm = hub ? g->zperm : nullptr;
    p.w = g->weighted ? (hub ? g->t_wz : g->t.w) : nullptr;
    p.inv = g->inv_deg;
    p.partials = part;
    p.omc = (float)(1.0 - c);
    p.c = (float)c;
    p.kt = 1;
    p.n = n;
    p.acc = out;
    p.comp = comp;
    for (int64_t i = 1; rc == TPA_OK && i <= K; ++i) {
        p.zin = (i & 1) ? z0 : z1;
        p.zout = (i & 1) ? z1 : z0;
        p.accumulate = i >= s_iter;
        rc = launch_step(*s, kStranger, false, p, st);
    }
    const hipError_t e = hipStreamSynchronize(st);
    dfree(tmp);
    TPA_TRY(rc);
    TPA_TRY_HIP(e);
    return TPA_OK;
}

extern "C" tpa_status tpa_cpi_batch(tpa_graph_t g, const int32_t *seeds, const float *q, int64_t k, double c,
                                    int s_iter, int t_iter, double eps, float *out, hipStream_t st) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (k < 0) return fail(TPA_ERR_INVALID_ARG, "k must be >= 0");
    if (!(c > 0.0 && c < 1.0)) return fail(TPA_ERR_INVALID_ARG, "c must lie in (0, 1)");
    if (s_iter < 0 || t_iter < -1 || (t_iter >= 0 && t_iter < s_iter))
        return fail(TPA_ERR_INVALID_ARG, "need 0 <= s_iter <= t_iter, or t_iter = -1");
    if (!(eps >= 0.0) || (eps == 0.0 && t_iter < 0))
        return fail(TPA_ERR_INVALID_ARG, "eps must be >= 0, and > 0 without a last iteration");
    if (k == 0) return TPA_OK;
    if ((seeds == nullptr) == (q == nullptr)) return fail(TPA_ERR_INVALID_ARG, "pass exactly one of seeds and q");
    if (!out) return fail(TPA_ERR_INVALID_ARG, "out is NULL");
    const int64_t n = g->n;
    // per restart j: Algorithm 1's last iteration min(t_iter, first i with
    // c (1-c)^i ||q_j||_1 < eps), as in tpa_cpi
    std::vector<double> qn((size_t)k, 1.0);
    if (q && eps > 0.0) {
        double *d = nullptr;
        TPA_TRY(dalloc(&d, (size_t)k, st));
        hipError_t e = hipSuccess;
        for (int64_t r0 = 0; r0 < k && e == hipSuccess; r0 += 65535) {
            const int64_t rr = std::min<int64_t>(65535, k - r0);
            l1_norm_kernel<<<(unsigned)rr, 256, 0, st>>>(q + r0 * n, n, d + r0);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(qn.data(), d, sizeof(double) * k, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        dfree(d);
        TPA_TRY_HIP(e);
    }
    std::vector<int32_t> klast((size_t)k);
    for (int64_t j = 0; j < k; ++j) {
        int64_t K = t_iter >= 0 ? t_iter : INT64_MAX;
        if (eps > 0.0) K = qn[j] > 0.0 ? std::min<int64_t>(K, stranger_last_iteration(c, eps / qn[j])) : 0;
        klast[j] = (int32_t)std::min<int64_t>(K, INT32_MAX);
    }
    const int kt = choose_kt(g, k);
    const Schedule *s = nullptr;
    TPA_TRY(get_schedule(g, choose_shape(g, kt), st, &s));
    if (g->gather_layout) {
        TPA_TRY(ensure_zlayout(g, st));
        TPA_TRY(ensure_wz(g, st));
    }
    const bool hub = g->gather_layout && g->zperm && (!g->weighted || g->t_wz_valid);
    if (hub && kt == 1) TPA_TRY(ensure_group_order(g, s, st));
    const size_t tile = (size_t)n * kt;
    float *buf = nullptr;
    const size_t nbuf = 4 * tile + (q ? tile : 0) + (size_t)std::max<int64_t>(s->n_chunk_items, 1) * kt;
    TPA_TRY(dalloc(&buf, nbuf, st));
    int32_t *kd = nullptr;
    if (dalloc(&kd, 64, st) != TPA_OK) {
        dfree(buf);
        return TPA_ERR_OUT_OF_MEMORY;
    }
    float *z0 = buf, *z1 = buf + tile, *acc = buf + 2 * tile, *comp = buf + 3 * tile;
    float *qT = q ? buf + 4 * tile : nullptr;
    float *part = buf + 4 * tile + (q ? tile : 0);
    StepParams p;
    p.rowptr = g->t.rowptr;
    p.zperm = hub ? g->zperm : nullptr;
    p.inv = g->inv_deg;
    p.partials = part;
    p.omc = (float)(1.0 - c);
    p.c = (float)c;
    p.kt = kt;
    p.n = n;
    p.tacc = acc;
    p.tcomp = comp;
    p.klast = kd;
    p.s_iter = s_iter;
    const int32_t *col_gather = hub ? g->t_colz : g->t.col;
    const float *w_gather = g->weighted ? (hub ? g->t_wz : g->t.w) : nullptr;
    tpa_status rc = TPA_OK;
    int32_t kh[64];
    for (int64_t base = 0; rc == TPA_OK && base < k; base += kt) {
        const int ncols = (int)std::min<int64_t>(kt, k - base);
        int64_t K = 0;
        for (int j = 0; j < kt; ++j) {
            kh[j] = j < ncols ? klast[base + j] : -1;
            K = std::max<int64_t>(K, kh[j]);
        }
        if (hipMemcpyAsync(kd, kh, sizeof(int32_t) * kt, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {  // kh is reused by the next tile
            rc = fail(TPA_ERR_HIP, "klast upload failed");
            break;
        }
        p.seeds = seeds ? seeds + base : nullptr;
        p.qdense = q ? q + base * n : nullptr;
        p.ncols = ncols;
        p.qT = nullptr;
        // x(0) into the window sum when s_iter = 0; for dense restarts also
        // the vector step 1 reads (one-hot first steps gather nothing)
        if (q) {
            rc = launch_dense_transpose(p, qT, st);
            p.qT = qT;
            if (rc == TPA_OK) rc = launch_dense_init(p, z0, s_iter == 0 ? acc : nullptr, st);
        } else if (s_iter == 0) {
            rc = launch_onehot_init(p, acc, st);
        }
        if (rc == TPA_OK && s_iter != 0) rc = launch_fill_zero(acc, (int64_t)tile, st);
        if (rc == TPA_OK) rc = launch_fill_zero(comp, (int64_t)tile, st);
        p.qT = nullptr;  // plain steps add no restart
        for (int64_t i = 1; rc == TPA_OK && i <= K; ++i) {
            p.zin = (i & 1) ? z0 : z1;
            p.zout = (i & 1) ? z1 : z0;
            p.iter = (int)i;
            const bool first = i == 1 && !q;  // one-hot restarts: x(1) needs no gather
            p.col = first ? g->t.col : col_gather;
            p.w = first ? (g->weighted ? g->t.w : nullptr) : w_gather;
            rc = launch_step(*s, kPlain, first, p, st);
        }
        if (rc == TPA_OK) rc = launch_tile_to_rows(acc, kt, ncols, n, p.seeds, out, base, g->dev_err, st);
    }
    const hipError_t e = hipStreamSynchronize(st);
    dfree(buf);
    dfree(kd);
    TPA_TRY(rc);
    TPA_TRY_HIP(e);
    return TPA_OK;
}

extern "C" tpa_status tpa_topk(const float *vals, int64_t rows, int64_t n, int k, int32_t *idx_out,
                               float *val_out, hipStream_t st) {
    if (rows < 0 || n < 1 || k < 1 || k > kTopkMax || k > n)
        return fail(TPA_ERR_INVALID_ARG, "need rows >= 0, n >= 1 and 1 <= k <= min(n, 1024)");
    if (rows == 0) return TPA_OK;
    if (!vals || !idx_out || !val_out) return fail(TPA_ERR_INVALID_ARG, "NULL argument");
    if (n > INT32_MAX) return fail(TPA_ERR_INDEX_OVERFLOW, "rows longer than 2^31 - 1");
    // stages: segments of seg >= 16 k entries, each keeping its k best, so
    // every stage shrinks the rows at least 16-fold; the last stage has one
    // segment per row
    const int64_t seg = std::max<int64_t>(4096, 16 * (int64_t)k);
    std::vector<int64_t> lens{n};
    while (lens.back() > seg) {
        const int64_t len = lens.back(), nseg = (len + seg - 1) / seg;
        lens.push_back((nseg - 1) * k + std::min<int64_t>(k, len - (nseg - 1) * seg));
    }
    for (size_t i = 0; i < lens.size(); ++i) {
        const int64_t nseg = (lens[i] + seg - 1) / seg;
        if (rows > INT32_MAX / nseg) return fail(TPA_ERR_INDEX_OVERFLOW, "too many rows for one launch");
    }
    // candidate lists of the intermediate stages (keys, then indices), in
    // one allocation
    std::vector<uint32_t *> bufs(lens.size() > 1 ? lens.size() - 1 : 0, nullptr);
    uint32_t *work = nullptr;
    tpa_status rc = TPA_OK;
    if (!bufs.empty()) {
        size_t total = 0;
        for (size_t i = 1; i < lens.size(); ++i) total += 2 * (size_t)rows * (size_t)lens[i];
        rc = dalloc(&work, total, st);
        size_t off = 0;
        for (size_t i = 1; rc == TPA_OK && i < lens.size(); ++i) {
            bufs[i - 1] = work + off;
            off += 2 * (size_t)rows * (size_t)lens[i];
        }
    }
    for (size_t i = 0; i < lens.size() && rc == TPA_OK; ++i) {
        TopkStage t;
        if (i == 0) {
            t.vals = vals;
        } else {
            t.keys = bufs[i - 1];
            t.idx = reinterpret_cast<const int32_t *>(bufs[i - 1] + (size_t)rows * lens[i]);
        }
        t.len = lens[i];
        t.seg = seg;
        t.nseg = (lens[i] + seg - 1) / seg;
        t.k = k;
        if (i + 1 < lens.size()) {
            t.out_keys = bufs[i];
            t.out_idx = reinterpret_cast<int32_t *>(bufs[i] + (size_t)rows * lens[i + 1]);
            t.out_len = lens[i + 1];
        } else {
            t.orig = vals;
            t.n = n;
            t.idx_out = idx_out;
            t.val_out = val_out;
        }
        // wide blocks when there are few segments, narrow ones when many
        // fill the device
        const unsigned grid = (unsigned)(rows * t.nseg);
        if (grid >= 512) topk_stage_kernel<256><<<grid, 256, 0, st>>>(t);
        else topk_stage_kernel<1024><<<grid, 1024, 0, st>>>(t);
        if (hipGetLastError() != hipSuccess) rc = fail(TPA_ERR_HIP, "top-k launch failed");
    }
    if (work) {
        const hipError_t e = hipStreamSynchronize(st);
        dfree(work);
        TPA_TRY(rc);
        TPA_TRY_HIP(e);
    }
    return rc;
}

extern "C" tpa_status tpa_row_l1(const float *x, const float *y, int64_t rows, int64_t n, double a, double *out,
                                 hipStream_t st) {
    if (rows < 0 || n < 0) return fail(TPA_ERR_INVALID_ARG, "negative size");
    if (rows == 0) return TPA_OK;
    if (!x || !y || !out) return fail(TPA_ERR_INVALID_ARG, "NULL argument");
    if (rows > 65535) return fail(TPA_ERR_INDEX_OVERFLOW, "at most 65535 rows per call");
    double *part = nullptr;
    TPA_TRY(dalloc(&part, (size_t)rows * kL1Parts, st));
    row_l1_parts_kernel<<<dim3(kL1Parts, (unsigned)rows), 256, 0, st>>>(x, y, n, a, part);
    row_l1_sum_kernel<<<(unsigned)((rows + 255) / 256), 256, 0, st>>>(part, rows, out);
    const hipError_t e = hipGetLastError();
    // the buffer is freed after the kernels that use it have run
    const hipError_t e2 = hipStreamSynchronize(st);
    dfree(part);
    TPA_TRY_HIP(e);
    TPA_TRY_HIP(e2);
    return TPA_OK;
}
