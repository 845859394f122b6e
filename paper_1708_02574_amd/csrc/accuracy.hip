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

// sum_v |q[v]| in FP64, one block, fixed order.
__global__ void l1_norm_kernel(const float *q, int64_t n, double *out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t v = threadIdx.x; v < n; v += blockDim.x) s += fabs((double)q[v]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
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

constexpr int kTopkThreads = 1024;
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

// One block per row.  A most-significant-digit-first radix select (four 8-bit
// digits) finds the key K of the k-th largest entry; the entries above K are
// taken, then those equal to K in index order until k are chosen; a bitonic
// sort orders the k pairs by (key descending, index ascending).
__global__ __launch_bounds__(kTopkThreads) void topk_kernel(const float *vals, int64_t n, int k, int32_t *idx_out,
                                                            float *val_out) {
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_prefix, s_need, s_count;
    __shared__ uint32_t skey[kTopkMax];
    __shared__ int32_t sidx[kTopkMax];
    __shared__ uint32_t scan[kTopkThreads];
    const int tid = threadIdx.x;
    const float *row = vals + (int64_t)blockIdx.x * n;
    if (tid == 0) {
        s_prefix = 0u;
        s_need = (uint32_t)k;
    }
    // radix select: after digit d, s_prefix holds the top d digits of K and
    // s_need the number of entries still to take among those with that prefix
    for (int d = 0; d < 4; ++d) {
        const int shift = 24 - 8 * d;
        const uint32_t mask_hi = d == 0 ? 0u : (0xffffffffu << (shift + 8));
        for (int i = tid; i < 256; i += blockDim.x) hist[i] = 0u;
        __syncthreads();
        const uint32_t prefix = s_prefix;
        constexpr int UL = 8;  // loads in flight per thread
        for (int64_t base = 0; base < n; base += (int64_t)blockDim.x * UL) {  // same trip count in every lane
            uint32_t key[UL];
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int64_t v = base + (int64_t)u * blockDim.x + tid;
                key[u] = v < n ? order_key(row[v]) : 0u;
            }
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int64_t v = base + (int64_t)u * blockDim.x + tid;
                hist_add(hist, (key[u] >> shift) & 255u, v < n && (key[u] & mask_hi) == prefix);
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
    const uint32_t take_eq = s_need;  // entries equal to K to take, lowest indices first
    if (tid == 0) s_count = 0u;
    __syncthreads();
    // entries above K (fewer than k of them), in any order
    {
        constexpr int UL = 8;
        for (int64_t base = 0; base < n; base += (int64_t)blockDim.x * UL) {
            uint32_t key[UL];
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int64_t v = base + (int64_t)u * blockDim.x + tid;
                key[u] = v < n ? order_key(row[v]) : 0u;
            }
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int64_t v = base + (int64_t)u * blockDim.x + tid;
                if (v < n && key[u] > K) {
                    const uint32_t pos = atomicAdd(&s_count, 1u);
                    skey[pos] = key[u];
                    sidx[pos] = (int32_t)v;
                }
            }
        }
    }
    __syncthreads();
    const uint32_t above = s_count;
    // entries equal to K, the take_eq with the lowest indices: wave w owns the
    // contiguous segment [w*seg, (w+1)*seg) and walks it 64 entries at a
    // time (coalesced); a scan of the per-wave counts gives each segment its
    // first rank, and ballots rank the entries inside a chunk
    {
        const int wv = tid >> 6, lane = tid & 63;
        const int nw = (int)blockDim.x >> 6;
        const int64_t seg = ((n + nw - 1) / nw + 63) & ~(int64_t)63;
        const int64_t s0 = (int64_t)wv * seg, s1 = min(n, s0 + seg);
        uint32_t cnt = 0u;
        for (int64_t v0 = s0; v0 < s1; v0 += 64) {
            const int64_t v = v0 + lane;
            cnt += (uint32_t)__popcll(__ballot(v < s1 && order_key(row[v]) == K));
        }
        if (lane == 0) scan[wv] = cnt;
        __syncthreads();
        uint32_t rank = 0u;
        for (int w = 0; w < wv; ++w) rank += scan[w];
        for (int64_t v0 = s0; v0 < s1 && rank < take_eq; v0 += 64) {
            const int64_t v = v0 + lane;
            const bool eq = v < s1 && order_key(row[v]) == K;
            const uint64_t m = __ballot(eq);
            const uint32_t r = rank + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            if (eq && r < take_eq) {
                skey[above + r] = K;
                sidx[above + r] = (int32_t)v;
            }
            rank += (uint32_t)__popcll(m);
        }
    }
    __syncthreads();
    // bitonic sort of the k pairs (padded to a power of two)
    int p2 = 1;
    while (p2 < k) p2 <<= 1;
    for (int i = tid; i < p2; i += blockDim.x)
        if (i >= k) {
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
    for (int i = tid; i < k; i += blockDim.x) {
        const int32_t v = sidx[i];
        idx_out[(int64_t)blockIdx.x * k + i] = v;
        val_out[(int64_t)blockIdx.x * k + i] = row[v];
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

extern "C" tpa_status tpa_topk(const float *vals, int64_t rows, int64_t n, int k, int32_t *idx_out,
                               float *val_out, hipStream_t st) {
    if (rows < 0 || n < 1 || k < 1 || k > kTopkMax || k > n)
        return fail(TPA_ERR_INVALID_ARG, "need rows >= 0, n >= 1 and 1 <= k <= min(n, 1024)");
    if (rows == 0) return TPA_OK;
    if (!vals || !idx_out || !val_out) return fail(TPA_ERR_INVALID_ARG, "NULL argument");
    if (n > INT32_MAX) return fail(TPA_ERR_INDEX_OVERFLOW, "rows longer than 2^31 - 1");
    if (rows > INT32_MAX) return fail(TPA_ERR_INDEX_OVERFLOW, "too many rows for one launch");
    topk_kernel<<<(unsigned)rows, kTopkThreads, 0, st>>>(vals, n, k, idx_out, val_out);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
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
