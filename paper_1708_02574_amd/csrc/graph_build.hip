// Graph store construction on the GPU: R-MAT sampling, sort + dedupe,
// dangling self-loops, CSR of A~ and A~^T, 1/outdeg weights, edge-logit
// softmax, block-diagonal packing, and the wave work schedule.
//
// The graph is the row-normalised adjacency A~ of the paper's Section 2
// (Table 1); every row of A~ must sum to 1 (Theorem 1, Lemma 2), hence the
// self-loop on each node without out-edges.

#include <cstring>

#include <rocprim/rocprim.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "tpa_internal.h"

namespace tpa {

int key_bits(int64_t n) {
    int b = 1;
    while (b < 62 && (int64_t(1) << b) < n) ++b;
    return b;
}

// ------------------------------------------------------------------ kernels
namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n, int block = kBlock) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, int64_t(1) << 22));  // grid-stride kernels
}

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output j of the generator
// seeded with `seed` is the mixing function applied to seed + (j+1)*gamma.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t j) {
    uint64_t z = seed + (j + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One raw R-MAT sample per thread; key = (u << bits) | v.
__global__ void rmat_kernel(uint64_t seed, int scale, int64_t raw_begin, int64_t count,
                            uint32_t t0, uint32_t t1, uint32_t t2, int64_t n_nodes, int bits,
                            uint64_t *keys, int64_t *accept) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t e = (uint64_t)(raw_begin + i);
        uint64_t u = 0, v = 0;
        for (int l = 0; l < scale; ++l) {
            const uint32_t r = (uint32_t)(splitmix64_at(seed, e * (uint64_t)scale + (uint64_t)l) >> 32);
            const uint32_t q = (uint32_t)(r >= t0) + (uint32_t)(r >= t1) + (uint32_t)(r >= t2);
            u = (u << 1) | (q >> 1);
            v = (v << 1) | (q & 1u);
        }
        const bool ok = (int64_t)u < n_nodes && (int64_t)v < n_nodes;
        keys[i] = ok ? ((u << bits) | v) : 0;
        if (accept) accept[i] = ok ? 1 : 0;
    }
}

__global__ void pack_edges_kernel(const int32_t *src, const int32_t *dst, int64_t m, int bits,
                                  int64_t n, uint64_t *keys, int32_t *bad) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = src[i], v = dst[i];
        if (u < 0 || u >= n || v < 0 || v >= n) {
            *bad = 1;
            keys[i] = 0;
        } else {
            keys[i] = ((uint64_t)u << bits) | (uint64_t)v;
        }
    }
}

// out[pos[i]] = in[i] where flag[i] (pos = exclusive scan of flags).
__global__ void compact_kernel(const uint64_t *in, const int64_t *flag, const int64_t *pos,
                               int64_t count, int64_t limit, int64_t out_base, uint64_t *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (flag[i]) {
            const int64_t p = out_base + pos[i];
            if (p < limit) out[p] = in[i];
        }
    }
}

__global__ void unique_flags_kernel(const uint64_t *k, int64_t count, int64_t *flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = (i == 0 || k[i] != k[i - 1]) ? 1 : 0;
}

__global__ void count_rows_kernel(const uint64_t *k, int64_t count, int bits, int32_t *deg) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&deg[k[i] >> bits], 1);
}

__global__ void count_cols_kernel(const int32_t *col, int64_t count, int32_t *deg) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&deg[col[i]], 1);
}

// deg -> (deg64, deg2 = max(deg,1), padded, 1/deg2); entry n is 0.
__global__ void degree_kernel(const int32_t *deg, int64_t n, int64_t *deg64, int64_t *deg2,
                              uint8_t *padded, float *inv) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u <= n;
         u += (int64_t)gridDim.x * blockDim.x) {
        if (u == n) {
            deg64[n] = 0;
            deg2[n] = 0;
        } else {
            const int32_t d = deg[u];
            deg64[u] = d;
            deg2[u] = d > 0 ? d : 1;
            padded[u] = d == 0;
            inv[u] = 1.0f / (float)(d > 0 ? d : 1);
        }
    }
}

__global__ void max_deg_kernel(const int64_t *deg, int64_t n, unsigned long long *out) {
    unsigned long long mx = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        mx = max(mx, (unsigned long long)deg[i]);
    atomicMax(out, mx);
}

__global__ void widen_kernel(const int32_t *in, int64_t n, int64_t *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = i < n ? in[i] : 0;
}

// Place unique edge i at its A~ slot and emit its transposed key.
__global__ void fill_a_kernel(const uint64_t *uk, int64_t mu, int bits, const int64_t *a_rowptr,
                              const int64_t *ustart, int32_t *a_col, uint64_t *tkeys) {
    const uint64_t mask = (bits >= 64) ? ~0ull : ((1ull << bits) - 1);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < mu;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = uk[i];
        const int64_t u = (int64_t)(k >> bits), v = (int64_t)(k & mask);
        const int64_t p = a_rowptr[u] + (i - ustart[u]);
        a_col[p] = (int32_t)v;
        tkeys[p] = ((uint64_t)v << bits) | (uint64_t)u;
    }
}

__global__ void fill_selfloops_kernel(const uint8_t *padded, int64_t n, int bits,
                                      const int64_t *a_rowptr, int32_t *a_col, uint64_t *tkeys) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        if (padded[u]) {
            const int64_t p = a_rowptr[u];
            a_col[p] = (int32_t)u;
            tkeys[p] = ((uint64_t)u << bits) | (uint64_t)u;
        }
    }
}

__global__ void low_bits_kernel(const uint64_t *k, int64_t count, int bits, int32_t *out) {
    const uint64_t mask = (1ull << bits) - 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int32_t)(k[i] & mask);
}

// Transposed keys + A~ edge ids, one thread per row of A~.
__global__ void tkeys_with_ids_kernel(const int64_t *a_rowptr, const int32_t *a_col, int64_t n,
                                      int bits, uint64_t *tkeys, int64_t *ids) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        for (int64_t e = a_rowptr[u]; e < a_rowptr[u + 1]; ++e) {
            tkeys[e] = ((uint64_t)a_col[e] << bits) | (uint64_t)u;
            ids[e] = e;
        }
    }
}

// Row softmax of the logits over A~'s rows, waves striding over the rows
// (fixed-order reductions, so the weights are deterministic).
__global__ void softmax_rows_kernel(const int64_t *rowptr, int64_t n, const float *theta,
                                    float *w) {
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t row = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; row < n; row += nwaves) {
        const int64_t b = rowptr[row], e = rowptr[row + 1];
        float mx = -INFINITY;
        for (int64_t i = b + lane; i < e; i += 64) mx = fmaxf(mx, theta[i]);
        for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
        float s = 0.0f;
        for (int64_t i = b + lane; i < e; i += 64) s += expf(theta[i] - mx);
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
        for (int64_t i = b + lane; i < e; i += 64) w[i] = expf(theta[i] - mx) / s;
    }
}

__global__ void gather_w_kernel(const float *aw, const int64_t *t2a, int64_t m, float *tw) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        tw[i] = aw[t2a[i]];
}

__global__ void uniform_w_kernel(const int64_t *rowptr, const int32_t *col, const float *inv,
                                 int64_t n, int transpose, float *w) {
    // transpose == 0: w[e] = inv[row]; transpose == 1: w[e] = inv[col[e]]
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x)
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) w[e] = transpose ? inv[col[e]] : inv[r];
}

__global__ void offset_i64_kernel(const int64_t *in, int64_t count, int64_t add, int64_t *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i] + add;
}

__global__ void offset_i32_kernel(const int32_t *in, int64_t count, int32_t add, int32_t *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i] + add;
}

__global__ void fill_block_kernel(int32_t *node_block, float *restart, int64_t begin, int64_t count,
                                  int32_t b, float inv_nb) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        node_block[begin + i] = b;
        restart[begin + i] = inv_nb;
    }
}

struct Plus64 {
    __host__ __device__ int64_t operator()(int64_t a, int64_t b) const { return a + b; }
};

// Exclusive prefix sum of count int64 values (rocPRIM device scan).
tpa_status exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t count, hipStream_t st) {
    size_t bytes = 0;
    TPA_TRY_HIP(rocprim::exclusive_scan(nullptr, bytes, in, out, int64_t(0), (size_t)count,
                                        Plus64(), st));
    void *tmp = nullptr;
    TPA_TRY(dmalloc(&tmp, std::max<size_t>(bytes, 16), st));
    hipError_t e = rocprim::exclusive_scan(tmp, bytes, in, out, int64_t(0), (size_t)count,
                                           Plus64(), st);
    dfree(tmp);
    TPA_TRY_HIP(e);
    return TPA_OK;
}

// Sort keys (bits [0, end_bit)); returns the buffer holding the result and
// frees the other one.
tpa_status sort_keys(uint64_t *keys, int64_t count, int end_bit, hipStream_t st, uint64_t **result) {
    uint64_t *alt = nullptr;
    TPA_TRY(dalloc(&alt, std::max<int64_t>(count, 1), st));
    rocprim::double_buffer<uint64_t> db(keys, alt);
    size_t bytes = 0;
    hipError_t e = rocprim::radix_sort_keys(nullptr, bytes, db, (size_t)count, 0u,
                                            (unsigned)end_bit, st);
    if (e != hipSuccess) { dfree(alt); TPA_TRY_HIP(e); }
    void *tmp = nullptr;
    tpa_status s = dmalloc(&tmp, std::max<size_t>(bytes, 16), st);
    if (s != TPA_OK) { dfree(alt); return s; }
    e = rocprim::radix_sort_keys(tmp, bytes, db, (size_t)count, 0u, (unsigned)end_bit, st);
    TPA_TRY_HIP(hipStreamSynchronize(st));
    dfree(tmp);
    if (e != hipSuccess) { dfree(alt); TPA_TRY_HIP(e); }
    *result = db.current();
    dfree(db.alternate());
    return TPA_OK;
}

template <class T>
T read_back(const T *dptr, hipStream_t st) {
    T v{};
    if (hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, st) != hipSuccess) return v;
    (void)hipStreamSynchronize(st);
    return v;
}

}  // namespace

// ------------------------------------------------------------------ build
tpa_status graph_alloc_common(tpa_graph *g, hipStream_t st) {
    TPA_TRY(dalloc(&g->dev_err, 1, st));
    TPA_TRY_HIP(hipMemsetAsync(g->dev_err, 0, sizeof(int32_t), st));
    g->block_off = {0, g->n};
    g->nblocks = 1;
    return TPA_OK;
}

// Takes ownership of `keys` ((u << bits) | v, nkeys entries).
tpa_status build_from_keys(tpa_graph *g, uint64_t *keys, int64_t nkeys, hipStream_t st) {
    const int64_t n = g->n;
    const int bits = g->bits;
    uint64_t *sorted = keys;
    if (nkeys > 0) {
        tpa_status s = sort_keys(keys, nkeys, 2 * bits, st, &sorted);
        if (s != TPA_OK) { dfree(keys); return s; }
    }
    // unique
    int64_t *flag = nullptr, *pos = nullptr;
    uint64_t *uk = nullptr;
    int64_t mu = 0;
    if (nkeys > 0) {
        TPA_TRY(dalloc(&flag, nkeys + 1, st));
        TPA_TRY(dalloc(&pos, nkeys + 1, st));
        unique_flags_kernel<<<grid_for(nkeys), kBlock, 0, st>>>(sorted, nkeys, flag);
        TPA_TRY(exclusive_scan_i64(flag, pos, nkeys, st));
        mu = read_back(pos + nkeys - 1, st) + read_back(flag + nkeys - 1, st);
        TPA_TRY(dalloc(&uk, std::max<int64_t>(mu, 1), st));
        compact_kernel<<<grid_for(nkeys), kBlock, 0, st>>>(sorted, flag, pos, nkeys, mu, 0, uk);
        TPA_TRY_HIP(hipStreamSynchronize(st));
        dfree(flag);
        dfree(pos);
        dfree(sorted);
    } else {
        dfree(keys);  // no edges: only the dangling self-loops below
    }
    // out-degrees, dangling self-loops, A~ row offsets
    int32_t *deg = nullptr;
    int64_t *deg64 = nullptr, *deg2 = nullptr, *ustart = nullptr;
    TPA_TRY(dalloc(&deg, n, st));
    TPA_TRY(dalloc(&deg64, n + 1, st));
    TPA_TRY(dalloc(&deg2, n + 1, st));
    TPA_TRY(dalloc(&ustart, n + 1, st));
    TPA_TRY(dalloc(&g->a.rowptr, n + 1, st));
    TPA_TRY(dalloc(&g->padded, n, st));
    TPA_TRY(dalloc(&g->inv_deg, n, st));
    TPA_TRY_HIP(hipMemsetAsync(deg, 0, sizeof(int32_t) * n, st));
    if (mu > 0) count_rows_kernel<<<grid_for(mu), kBlock, 0, st>>>(uk, mu, bits, deg);
    degree_kernel<<<grid_for(n + 1), kBlock, 0, st>>>(deg, n, deg64, deg2, g->padded, g->inv_deg);
    TPA_TRY(exclusive_scan_i64(deg64, ustart, n + 1, st));
    TPA_TRY(exclusive_scan_i64(deg2, g->a.rowptr, n + 1, st));
    g->m = read_back(g->a.rowptr + n, st);
    {
        unsigned long long *mx = nullptr;
        TPA_TRY(dalloc(&mx, 1, st));
        TPA_TRY_HIP(hipMemsetAsync(mx, 0, sizeof(unsigned long long), st));
        max_deg_kernel<<<grid_for(n), kBlock, 0, st>>>(deg2, n, mx);
        g->max_outdeg = (int64_t)read_back(mx, st);
        dfree(mx);
    }
    const int64_t m = g->m;
    // A~ columns + transposed keys
    uint64_t *tkeys = nullptr;
    TPA_TRY(dalloc(&g->a.col, m, st));
    TPA_TRY(dalloc(&tkeys, m, st));
    if (mu > 0)
        fill_a_kernel<<<grid_for(mu), kBlock, 0, st>>>(uk, mu, bits, g->a.rowptr, ustart, g->a.col, tkeys);
    fill_selfloops_kernel<<<grid_for(n), kBlock, 0, st>>>(g->padded, n, bits, g->a.rowptr, g->a.col, tkeys);
    TPA_TRY_HIP(hipStreamSynchronize(st));
    dfree(uk);
    dfree(ustart);
    dfree(deg2);
    // A~^T: sort transposed keys; row offsets from in-degrees
    uint64_t *tsorted = nullptr;
    TPA_TRY(sort_keys(tkeys, m, 2 * bits, st, &tsorted));
    TPA_TRY(dalloc(&g->t.col, m, st));
    TPA_TRY(dalloc(&g->t.rowptr, n + 1, st));
    low_bits_kernel<<<grid_for(m), kBlock, 0, st>>>(tsorted, m, bits, g->t.col);
    TPA_TRY_HIP(hipMemsetAsync(deg, 0, sizeof(int32_t) * n, st));
    count_cols_kernel<<<grid_for(m), kBlock, 0, st>>>(g->a.col, m, deg);
    widen_kernel<<<grid_for(n + 1), kBlock, 0, st>>>(deg, n, deg64);
    TPA_TRY(exclusive_scan_i64(deg64, g->t.rowptr, n + 1, st));
    TPA_TRY_HIP(hipStreamSynchronize(st));
    dfree(tsorted);
    dfree(deg);
    dfree(deg64);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status ensure_t2a(tpa_graph *g, hipStream_t st) {
    if (g->t2a) return TPA_OK;
    const int64_t n = g->n, m = g->m;
    uint64_t *k0 = nullptr, *k1 = nullptr;
    int64_t *v0 = nullptr, *v1 = nullptr;
    TPA_TRY(dalloc(&k0, m, st));
    TPA_TRY(dalloc(&k1, m, st));
    TPA_TRY(dalloc(&v0, m, st));
    TPA_TRY(dalloc(&v1, m, st));
    tkeys_with_ids_kernel<<<grid_for(n), kBlock, 0, st>>>(g->a.rowptr, g->a.col, n, g->bits, k0, v0);
    rocprim::double_buffer<uint64_t> kb(k0, k1);
    rocprim::double_buffer<int64_t> vb(v0, v1);
    size_t bytes = 0;
    TPA_TRY_HIP(rocprim::radix_sort_pairs(nullptr, bytes, kb, vb, (size_t)m, 0u, (unsigned)(2 * g->bits), st));
    void *tmp = nullptr;
    TPA_TRY(dmalloc(&tmp, std::max<size_t>(bytes, 16), st));
    TPA_TRY_HIP(rocprim::radix_sort_pairs(tmp, bytes, kb, vb, (size_t)m, 0u, (unsigned)(2 * g->bits), st));
    TPA_TRY_HIP(hipStreamSynchronize(st));
    dfree(tmp);
    g->t2a = vb.current();
    dfree(vb.alternate());
    dfree(k0);
    dfree(k1);
    return TPA_OK;
}

namespace {

__global__ void hub_keys_kernel(const int64_t *rowptr, int64_t n, int64_t maxd, uint32_t *keys, int32_t *ids) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        keys[v] = (uint32_t)(maxd - (rowptr[v + 1] - rowptr[v]));
        ids[v] = (int32_t)v;
    }
}

__global__ void invert_perm_kernel(const int32_t *order, int64_t n, int32_t *rank) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        rank[order[i]] = (int32_t)i;
}

__global__ void map_cols_kernel(const int32_t *col, int64_t m, const int32_t *rank, int32_t *out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = rank[col[e]];
}

__global__ void row_col_keys_kernel(const int64_t *rowptr, int64_t n, const int32_t *colz, uint64_t *keys,
                                    int32_t *loc) {
    const int lane = threadIdx.x & 63;
    const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t v = w0; v < n; v += nw)
        for (int64_t e = rowptr[v] + lane; e < rowptr[v + 1]; e += 64) {
            keys[e] = ((uint64_t)v << 32) | (uint32_t)colz[e];
            loc[e] = (int32_t)(e - rowptr[v]);
        }
}

// Weights of A~^T in the re-sorted row order: wz[e'] = w[rowptr[v] + loc[e']].
__global__ void gather_row_w_kernel(const int64_t *rowptr, int64_t n, const int32_t *loc, const float *w,
                                    float *wz) {
    const int lane = threadIdx.x & 63;
    const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t v = w0; v < n; v += nw) {
        const int64_t b = rowptr[v];
        for (int64_t e = b + lane; e < rowptr[v + 1]; e += 64) wz[e] = w[b + loc[e]];
    }
}

__global__ void low32_kernel(const uint64_t *keys, int64_t m, int32_t *out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = (int32_t)(uint32_t)keys[e];
}

// One block per group item (grid-stride over the items): the item's edges
// sorted by gather row, ties by position, with a bitonic sort of kGroupEdges
// (row, position) keys in LDS, padded with all-ones keys; each entry then
// holds its row and, above it, its position in the item.
__global__ __launch_bounds__(256) void group_order_kernel(const Item *items, int64_t n_items, const int32_t *colz,
                                                          int32_t *colg) {
    __shared__ uint64_t key[kGroupEdges];
    for (int64_t b = blockIdx.x; b < n_items; b += gridDim.x) {
        const Item it = items[b];
        if (item_kind(it.meta) != kItemGroup) continue;  // block-uniform
        const int nnz = (int)item_nnz(it.meta);
        for (int k = threadIdx.x; k < kGroupEdges; k += 256)
            key[k] = k < nnz ? ((uint64_t)(uint32_t)colz[it.e0 + k] << 32) | (uint32_t)k : ~0ull;
        __syncthreads();
        for (int size = 2; size <= kGroupEdges; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = threadIdx.x; t < kGroupEdges / 2; t += 256) {
                    const int i = 2 * t - (t & (stride - 1)), j = i + stride;
                    const uint64_t x = key[i], y = key[j];
                    if ((x > y) == ((i & size) == 0)) {
                        key[i] = y;
                        key[j] = x;
                    }
                }
                __syncthreads();
            }
        }
        for (int k = threadIdx.x; k < nnz; k += 256) {
            const uint64_t x = key[k];
            colg[it.e0 + k] = (int32_t)((uint32_t)(x >> 32) | ((uint32_t)x << kGroupSlotShift));
        }
        __syncthreads();  // the keys are read before the next item overwrites them
    }
}

}  // namespace

// Rank of every node by descending out-degree (a stable radix sort keeps
// ties in id order), and A~^T's column ids mapped through it with each row
// re-sorted by rank.
tpa_status ensure_zlayout(tpa_graph *g, hipStream_t st) {
    if (g->zperm) return TPA_OK;
    const int64_t n = g->n, m = g->m;
    int end_bit = 1;
    while (end_bit < 32 && ((int64_t)1 << end_bit) <= g->max_outdeg) ++end_bit;
    uint32_t *k0 = nullptr, *k1 = nullptr;
    int32_t *v0 = nullptr, *v1 = nullptr, *rank = nullptr, *colz = nullptr;
    void *tmp = nullptr;
    auto cleanup = [&]() { dfree(k0); dfree(k1); dfree(v0); dfree(v1); dfree(tmp); };
    tpa_status rc = TPA_OK;
    if ((rc = dalloc(&k0, n, st)) != TPA_OK || (rc = dalloc(&k1, n, st)) != TPA_OK ||
        (rc = dalloc(&v0, n, st)) != TPA_OK || (rc = dalloc(&v1, n, st)) != TPA_OK) {
        cleanup();
        return rc;
    }
    hub_keys_kernel<<<grid_for(n), kBlock, 0, st>>>(g->a.rowptr, n, g->max_outdeg, k0, v0);
    rocprim::double_buffer<uint32_t> kb(k0, k1);
    rocprim::double_buffer<int32_t> vb(v0, v1);
    size_t bytes = 0;
    hipError_t e = rocprim::radix_sort_pairs(nullptr, bytes, kb, vb, (size_t)n, 0u, (unsigned)end_bit, st);
    if (e == hipSuccess) rc = dmalloc(&tmp, std::max<size_t>(bytes, 16), st);
    if (e == hipSuccess && rc == TPA_OK)
        e = rocprim::radix_sort_pairs(tmp, bytes, kb, vb, (size_t)n, 0u, (unsigned)end_bit, st);
    if (e != hipSuccess) rc = fail(TPA_ERR_HIP, std::string("radix_sort_pairs: ") + hipGetErrorString(e));
    if (rc == TPA_OK) rc = dalloc(&rank, n, st);
    if (rc == TPA_OK) rc = dalloc(&colz, m, st);
    if (rc != TPA_OK) {
        dfree(rank);
        cleanup();
        return rc;
    }
    invert_perm_kernel<<<grid_for(n), kBlock, 0, st>>>(vb.current(), n, rank);
    map_cols_kernel<<<grid_for(m), kBlock, 0, st>>>(g->t.col, m, rank, colz);
    e = hipStreamSynchronize(st);
    // the sorted ids are the node at each gather row: kept
    int32_t *zinv = vb.current();
    if (zinv == v0) v0 = nullptr;
    else v1 = nullptr;
    cleanup();
    // each row's edges in ascending hub rank: the first edges of every row
    // then read the same few cache lines of the gathered vector; each edge's
    // position in its row of A~^T is kept (loc) to re-sort per-edge weights
    int32_t *loc = nullptr;
    if (e == hipSuccess) {
        uint64_t *k2a = nullptr, *k2b = nullptr;
        int32_t *l2b = nullptr;
        void *tmp2 = nullptr;
        if ((rc = dalloc(&k2a, m, st)) == TPA_OK && (rc = dalloc(&k2b, m, st)) == TPA_OK &&
            (rc = dalloc(&loc, m, st)) == TPA_OK && (rc = dalloc(&l2b, m, st)) == TPA_OK) {
            row_col_keys_kernel<<<grid_for(n * 64), kBlock, 0, st>>>(g->t.rowptr, n, colz, k2a, loc);
            rocprim::double_buffer<uint64_t> kb2(k2a, k2b);
            rocprim::double_buffer<int32_t> lb2(loc, l2b);
            size_t bytes2 = 0;
            e = rocprim::radix_sort_pairs(nullptr, bytes2, kb2, lb2, (size_t)m, 0u, (unsigned)(32 + g->bits), st);
            if (e == hipSuccess) rc = dmalloc(&tmp2, std::max<size_t>(bytes2, 16), st);
            if (e == hipSuccess && rc == TPA_OK)
                e = rocprim::radix_sort_pairs(tmp2, bytes2, kb2, lb2, (size_t)m, 0u, (unsigned)(32 + g->bits), st);
            if (e == hipSuccess && rc == TPA_OK) {
                low32_kernel<<<grid_for(m), kBlock, 0, st>>>(kb2.current(), m, colz);
                e = hipStreamSynchronize(st);
            }
            // keep the sorted positions, free the other buffer
            int32_t *keep = lb2.current();
            int32_t *other = lb2.alternate();
            loc = keep;
            dfree(other);
        } else {
            dfree(l2b);
        }
        dfree(k2a);
        dfree(k2b);
        dfree(tmp2);
        if (e != hipSuccess && rc == TPA_OK) rc = fail(TPA_ERR_HIP, std::string("row sort: ") + hipGetErrorString(e));
        if (rc != TPA_OK) { dfree(rank); dfree(zinv); dfree(colz); dfree(loc); return rc; }
    }
    if (e != hipSuccess) {
        dfree(rank);
        dfree(zinv);
        dfree(colz);
        dfree(loc);
        return fail(TPA_ERR_HIP, std::string("gather layout: ") + hipGetErrorString(e));
    }
    g->zperm = rank;
    g->zinv = zinv;
    g->t_colz = colz;
    g->t_locz = loc;
    g->t_wz_valid = false;
    return TPA_OK;
}

// Per-edge weights in the gather layout's row order, after the weights
// change (weighted graphs only).
tpa_status ensure_wz(tpa_graph *g, hipStream_t st) {
    if (!g->weighted || !g->t_locz || g->t_wz_valid) return TPA_OK;
    if (!g->t_wz) TPA_TRY(dalloc(&g->t_wz, g->m, st));
    gather_row_w_kernel<<<grid_for(g->n * 64), kBlock, 0, st>>>(g->t.rowptr, g->n, g->t_locz, g->t.w, g->t_wz);
    TPA_TRY_HIP(hipGetLastError());
    g->t_wz_valid = true;
    return TPA_OK;
}

tpa_status ensure_group_order(tpa_graph *g, const Schedule *cs, hipStream_t st, bool over_a) {
    Schedule *s = const_cast<Schedule *>(cs);  // an entry of g's schedule cache
    // forward: hub-first ids of A~^T (gather rows); adjoint: A~'s destination ids
    const int32_t *src = over_a ? (g->a_colr ? g->a_colr : g->a.col) : g->t_colz;
    if (g->gather_layout != 2 || !src || s->n_items == 0) return TPA_OK;
    if (s->colg) {  // built before, set aside by a layout change
        if (s->colg_from == src) s->colg_src = src;
        return TPA_OK;
    }
    if (g->n >= kGroupSlotMaxN || s->ew > kGroupEdges) return TPA_OK;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return TPA_OK;
    // an optional copy: built only when it takes at most a quarter of the free memory
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || (size_t)g->m * sizeof(int32_t) > free_b / 4) return TPA_OK;
    int32_t *colg = nullptr;
    if (dalloc(&colg, g->m, st) != TPA_OK) return TPA_OK;  // optional: the kernels read t_colz instead
    hipError_t e = hipMemcpyAsync(colg, src, sizeof(int32_t) * g->m, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) {
        const unsigned grid = (unsigned)std::min<int64_t>(s->n_items, int64_t(1) << 20);
        group_order_kernel<<<grid, 256, 0, st>>>(s->items, s->n_items, src, colg);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        dfree(colg);
        return fail(TPA_ERR_HIP, std::string("group order: ") + hipGetErrorString(e));
    }
    s->colg = colg;
    s->colg_src = src;
    s->colg_from = src;
    return TPA_OK;
}

// Rank of every node by descending in-degree (the rows of A~^T), and A~'s
// destination ids mapped through it.
tpa_status ensure_lam_layout(tpa_graph *g, hipStream_t st) {
    if (g->lrank) return TPA_OK;
    const int64_t n = g->n, m = g->m;
    if (m >= (int64_t(1) << 32)) return TPA_OK;  // in-degree keys are 32 bits
    uint32_t *k0 = nullptr, *k1 = nullptr;
    int32_t *v0 = nullptr, *v1 = nullptr, *rank = nullptr, *colr = nullptr;
    void *tmp = nullptr;
    auto cleanup = [&]() { dfree(k0); dfree(k1); dfree(v0); dfree(v1); dfree(tmp); };
    tpa_status rc = TPA_OK;
    if ((rc = dalloc(&k0, n, st)) != TPA_OK || (rc = dalloc(&k1, n, st)) != TPA_OK ||
        (rc = dalloc(&v0, n, st)) != TPA_OK || (rc = dalloc(&v1, n, st)) != TPA_OK) {
        cleanup();
        return rc;
    }
    hub_keys_kernel<<<grid_for(n), kBlock, 0, st>>>(g->t.rowptr, n, m, k0, v0);
    rocprim::double_buffer<uint32_t> kb(k0, k1);
    rocprim::double_buffer<int32_t> vb(v0, v1);
    size_t bytes = 0;
    const unsigned end_bit = (unsigned)std::min(32, key_bits(m + 1));
    hipError_t e = rocprim::radix_sort_pairs(nullptr, bytes, kb, vb, (size_t)n, 0u, end_bit, st);
    if (e == hipSuccess) rc = dmalloc(&tmp, std::max<size_t>(bytes, 16), st);
    if (e == hipSuccess && rc == TPA_OK) e = rocprim::radix_sort_pairs(tmp, bytes, kb, vb, (size_t)n, 0u, end_bit, st);
    if (e != hipSuccess) rc = fail(TPA_ERR_HIP, std::string("radix_sort_pairs: ") + hipGetErrorString(e));
    if (rc == TPA_OK) rc = dalloc(&rank, n, st);
    if (rc == TPA_OK) rc = dalloc(&colr, std::max<int64_t>(m, 1), st);
    if (rc == TPA_OK) {
        invert_perm_kernel<<<grid_for(n), kBlock, 0, st>>>(vb.current(), n, rank);
        map_cols_kernel<<<grid_for(m), kBlock, 0, st>>>(g->a.col, m, rank, colr);
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(TPA_ERR_HIP, std::string("adjoint layout: ") + hipGetErrorString(e));
    }
    cleanup();
    if (rc != TPA_OK) {
        dfree(rank);
        dfree(colr);
        return rc;
    }
    g->lrank = rank;
    g->a_colr = colr;
    return TPA_OK;
}

namespace {

constexpr int kSliceSegment = 8192;  // edges of a long row per counting wave

// Edges per source slice of each segment of a long row (one wave per
// segment; cnt[seg][x]).
__global__ __launch_bounds__(256) void slice_count_kernel(const int64_t *__restrict__ seg_e0,
                                                          const int32_t *__restrict__ seg_len, int64_t nseg,
                                                          const int32_t *__restrict__ col, int32_t *__restrict__ cnt) {
    const int lane = threadIdx.x & 63;
    const int64_t sg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (sg >= nseg) return;
    const int64_t e0 = seg_e0[sg];
    const int len = seg_len[sg];
    int c[kSliceCount] = {};
    for (int b = 0; b < len; b += 64) {
        const int e = b + lane;
        const int x = e < len ? gather_slice(col[e0 + e]) : -1;
#pragma unroll
        for (int k = 0; k < kSliceCount; ++k) c[k] += __popcll(__ballot(x == k));
    }
    int mine = 0;
#pragma unroll
    for (int k = 0; k < kSliceCount; ++k)
        if (lane == k) mine = c[k];
    if (lane < kSliceCount) cnt[sg * kSliceCount + lane] = mine;
}

// Stable partition of each segment's edges by source slice: slice x's
// edges of segment sg go, in order, from colx[seg_out[sg][x]] on.
__global__ __launch_bounds__(256) void slice_scatter_kernel(const int64_t *__restrict__ seg_e0,
                                                            const int32_t *__restrict__ seg_len, int64_t nseg,
                                                            const int64_t *__restrict__ seg_out,
                                                            const int32_t *__restrict__ col,
                                                            int32_t *__restrict__ colx) {
    const int lane = threadIdx.x & 63;
    const int64_t sg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (sg >= nseg) return;
    const int64_t e0 = seg_e0[sg];
    const int len = seg_len[sg];
    int64_t o[kSliceCount];
#pragma unroll
    for (int k = 0; k < kSliceCount; ++k) o[k] = seg_out[sg * kSliceCount + k];
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int b = 0; b < len; b += 64) {
        const int e = b + lane;
        const int32_t u = e < len ? col[e0 + e] : 0;
        const int x = e < len ? gather_slice(u) : -1;
#pragma unroll
        for (int k = 0; k < kSliceCount; ++k) {
            const uint64_t mk = __ballot(x == k);
            if (x == k) colx[o[k] + __popcll(mk & below)] = u;
            o[k] += __popcll(mk);
        }
    }
}

// The inverse of slice_scatter_kernel's placement for per-edge values:
// edge k of segment sg (original order) takes the value at the position the
// scatter gave it.
__global__ __launch_bounds__(256) void slice_gather_back_kernel(const int64_t *__restrict__ seg_e0,
                                                                const int32_t *__restrict__ seg_len, int64_t nseg,
                                                                const int64_t *__restrict__ seg_out,
                                                                const int32_t *__restrict__ col,
                                                                const float *__restrict__ vx,
                                                                float *__restrict__ v) {
    const int lane = threadIdx.x & 63;
    const int64_t sg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (sg >= nseg) return;
    const int64_t e0 = seg_e0[sg];
    const int len = seg_len[sg];
    int64_t o[kSliceCount];
#pragma unroll
    for (int k = 0; k < kSliceCount; ++k) o[k] = seg_out[sg * kSliceCount + k];
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int b = 0; b < len; b += 64) {
        const int e = b + lane;
        const int x = e < len ? gather_slice(col[e0 + e]) : -1;
#pragma unroll
        for (int k = 0; k < kSliceCount; ++k) {
            const uint64_t mk = __ballot(x == k);
            if (x == k) v[e0 + e] = vx[o[k] + __popcll(mk & below)];
            o[k] += __popcll(mk);
        }
    }
}

// Short rows' edges into their section of the sliced ids (grid-stride
// over rows; rows flagged foreign are placed by slice_scatter_kernel).
__global__ __launch_bounds__(256) void short_copy_kernel(const int64_t *__restrict__ rp,
                                                         const int64_t *__restrict__ rowx, int64_t n,
                                                         const int32_t *__restrict__ col,
                                                         int32_t *__restrict__ colx) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rx = rowx[r];
        if ((rx >> kRowxForeignBit) & 1) continue;
        const int64_t b = rp[r], d = rp[r + 1] - b, o = rx & kRowxMask;
        for (int64_t k = 0; k < d; ++k) colx[o + k] = col[b + k];
    }
}

}  // namespace

namespace {
bool takes_sliced_sweep(const tpa_graph *g) {
    if (g->sliced_sweep == 0 || (g->sliced_sweep == 1 && g->n < kSliceMinN)) return false;
    return g->gather_layout && g->zperm && g->t_colz && !g->weighted && g->n > 0;
}
}  // namespace

const Schedule *find_sliced_sweep(const tpa_graph *g, const int32_t **col) {
    *col = nullptr;
    if (!takes_sliced_sweep(g) || g->sched_x_none || !g->sched_x.items || !g->t_colx ||
        g->sched_x_ew != choose_shape(g, 1).ew)
        return nullptr;
    *col = g->t_colx;
    return &g->sched_x;
}

tpa_status ensure_sliced_sweep(tpa_graph *g, hipStream_t st, const Schedule **out, const int32_t **out_col) {
    *out = nullptr;
    *out_col = nullptr;
    if (!takes_sliced_sweep(g)) return TPA_OK;
    const int ew = choose_shape(g, 1).ew;
    if (g->sched_x_ew == ew && (g->sched_x_none || g->sched_x.items)) {
        *out = find_sliced_sweep(g, out_col);
        return TPA_OK;
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return TPA_OK;
    const int64_t n = g->n, m = g->m;
    const int64_t lm = std::min<int64_t>(kSliceShortRow, ew);
    std::vector<int64_t> rp(n + 1);
    TPA_TRY_HIP(hipMemcpyAsync(rp.data(), g->t.rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, st));
    TPA_TRY_HIP(hipStreamSynchronize(st));
    // medium rows (one counting segment each) and long rows (segments of
    // kSliceSegment edges), in row order
    std::vector<int32_t> mrows, lrows;
    std::vector<int64_t> first_seg, seg_e0;
    std::vector<int32_t> seg_len;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t d = rp[r + 1] - rp[r];
        if (d > lm && d <= ew) {
            mrows.push_back((int32_t)r);
            seg_e0.push_back(rp[r]);
            seg_len.push_back((int32_t)d);
        }
    }
    for (int64_t r = 0; r < n; ++r) {
        const int64_t d = rp[r + 1] - rp[r];
        if (d <= ew) continue;
        lrows.push_back((int32_t)r);
        first_seg.push_back((int64_t)seg_e0.size());
        for (int64_t off = 0; off < d; off += kSliceSegment) {
            seg_e0.push_back(rp[r] + off);
            seg_len.push_back((int32_t)std::min<int64_t>(kSliceSegment, d - off));
        }
    }
    first_seg.push_back((int64_t)seg_e0.size());
    if (lrows.empty() && mrows.empty()) {
        g->sched_x.release();
        g->sched_x = Schedule();
        g->sched_x_ew = ew;
        g->sched_x_none = true;
        return TPA_OK;
    }
    // an optional copy: built only when it (and the row offsets) take at
    // most a quarter of the free memory
    size_t free_b = 0, total_b = 0;
    const size_t extra = (g->t_colx ? 0 : (size_t)m * sizeof(int32_t)) + (size_t)(n + 1) * sizeof(int64_t);
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || extra > free_b / 4) return TPA_OK;
    const int64_t nseg = (int64_t)seg_e0.size();
    int64_t *d_e0 = nullptr, *d_out = nullptr;
    int32_t *d_len = nullptr, *d_cnt = nullptr;
    auto cleanup = [&]() { dfree(d_e0); dfree(d_out); dfree(d_len); dfree(d_cnt); };
    tpa_status rc = TPA_OK;
    if ((rc = dalloc(&d_e0, nseg, st)) != TPA_OK || (rc = dalloc(&d_len, nseg, st)) != TPA_OK ||
        (rc = dalloc(&d_cnt, nseg * kSliceCount, st)) != TPA_OK || (rc = dalloc(&d_out, nseg * kSliceCount, st)) != TPA_OK) {
        cleanup();
        return rc == TPA_ERR_OUT_OF_MEMORY ? TPA_OK : rc;  // optional: the sweep runs unsliced
    }
    std::vector<int32_t> cnt((size_t)nseg * kSliceCount);
    hipError_t e = hipMemcpyAsync(d_e0, seg_e0.data(), sizeof(int64_t) * nseg, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_len, seg_len.data(), sizeof(int32_t) * nseg, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        slice_count_kernel<<<(unsigned)((nseg + 3) / 4), 256, 0, st>>>(d_e0, d_len, nseg, g->t_colz, d_cnt);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(cnt.data(), d_cnt, sizeof(int32_t) * cnt.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        cleanup();
        return fail(TPA_ERR_HIP, std::string("sliced sweep: ") + hipGetErrorString(e));
    }
    for (int64_t sg = 0; sg < nseg; ++sg) {
        int64_t sum = 0;
        for (int x = 0; x < kSliceCount; ++x) sum += cnt[(size_t)sg * kSliceCount + x];
        if (sum != seg_len[sg]) {
            cleanup();
            return fail(TPA_ERR_HIP, "sliced sweep: slice counts do not add up to the segment length");
        }
    }
    // short section: offsets of the short rows, the others flagged
    std::vector<int64_t> rowx(n + 1);
    int64_t pos = 0;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t d = rp[r + 1] - rp[r];
        if (d <= lm) {
            rowx[r] = pos;
            pos += d;
        } else {
            rowx[r] = pos | (int64_t(1) << kRowxForeignBit);
        }
    }
    rowx[n] = pos;
    std::vector<int64_t> seg_out((size_t)nseg * kSliceCount);
    std::vector<Item> lists[kSliceCount];
    std::vector<int32_t> xrel;
    std::vector<LongRow> longs, longs8;
    int64_t slot = 0;
    // long rows' chunk slots first: slice x's run follows slices 0..x-1,
    // cut into chunks of at most 4*EW edges, slots in slice then chunk order
    const int64_t chunk = 4 * (int64_t)ew;
    int64_t lpos = 0;  // long rows' offset within their section (placed after the bands)
    std::vector<int64_t> lstart(lrows.size());
    for (size_t l = 0; l < lrows.size(); ++l) {
        lstart[l] = lpos;
        lpos += rp[lrows[l] + 1] - rp[lrows[l]];
    }
    // bands of consecutive medium rows: at most 63 rows and kGroupEdges
    // edges per slice
    const int64_t band_section = pos;
    // medium row k's slot of slice x is x * M + k (a band item stores its
    // rows' sums side by side); the long rows' slots follow
    const int64_t M = (int64_t)mrows.size();
    if (8 * M > INT32_MAX) {
        cleanup();
        return fail(TPA_ERR_INDEX_OVERFLOW, "too many sliced work items");
    }
    slot = 8 * M;
    for (size_t i = 0; i < mrows.size();) {
        int64_t bc[kSliceCount] = {};
        size_t j = i;
        while (j < mrows.size() && j - i < 63) {
            bool fits = true;
            for (int x = 0; x < kSliceCount; ++x)
                if (bc[x] + cnt[j * kSliceCount + x] > kGroupEdges) fits = false;
            if (!fits) break;
            for (int x = 0; x < kSliceCount; ++x) bc[x] += cnt[j * kSliceCount + x];
            ++j;
        }
        const int R = (int)(j - i);  // >= 1: a medium row has at most EW <= kGroupEdges edges
        if (R == 0) {
            cleanup();
            return fail(TPA_ERR_HIP, "sliced sweep: a medium row exceeds a band");
        }
        for (int x = 0; x < kSliceCount; ++x) {
            const int64_t tab = (int64_t)xrel.size();
            xrel.push_back((int32_t)(x * M + (int64_t)i));
            int64_t run = 0;
            for (size_t r = i; r < j; ++r) {
                xrel.push_back((int32_t)run);
                seg_out[r * kSliceCount + x] = pos + run;
                run += cnt[r * kSliceCount + x];
            }
            xrel.push_back((int32_t)run);
            lists[x].push_back({pos, (int32_t)tab, item_meta((uint32_t)R, (uint32_t)run, kItemGroup) | kItemBandBit});
            pos += run;
        }
        for (size_t r = i; r < j; ++r) longs8.push_back({mrows[r], 8, (int32_t)r, 0});
        if ((int64_t)xrel.size() > INT32_MAX) {
            cleanup();
            return fail(TPA_ERR_INDEX_OVERFLOW, "too many sliced work items");
        }
        i = j;
    }
    const int64_t long_section = pos;
    for (size_t l = 0; l < lrows.size(); ++l) {
        int64_t tot[kSliceCount] = {};
        for (int64_t sg = first_seg[l]; sg < first_seg[l + 1]; ++sg)
            for (int x = 0; x < kSliceCount; ++x) tot[x] += cnt[(size_t)sg * kSliceCount + x];
        const int64_t first_slot = slot;
        int64_t start = long_section + lstart[l];
        for (int x = 0; x < kSliceCount; ++x) {
            int64_t at = start;
            for (int64_t sg = first_seg[l]; sg < first_seg[l + 1]; ++sg) {
                seg_out[(size_t)sg * kSliceCount + x] = at;
                at += cnt[(size_t)sg * kSliceCount + x];
            }
            for (int64_t off = 0; off < tot[x]; off += chunk) {
                const int64_t len = std::min(chunk, tot[x] - off);
                lists[x].push_back({start + off, (int32_t)slot, item_meta(1, (uint32_t)len, kItemChunk)});
                ++slot;
            }
            start += tot[x];
        }
        if (slot > INT32_MAX) {
            cleanup();
            return fail(TPA_ERR_INDEX_OVERFLOW, "too many chunk items");
        }
        longs.push_back({lrows[l], (int32_t)(slot - first_slot), (int32_t)first_slot, 0});
    }
    if (long_section + lpos != m || band_section != rowx[n]) {
        cleanup();
        return fail(TPA_ERR_HIP, "sliced sweep: sections do not cover the edges");
    }
    // block b of the sliced region holds slice b % 8's items (empty group
    // items pad the shorter slices), then the group items of the short rows
    size_t per = 0;
    for (int x = 0; x < kSliceCount; ++x) per = std::max(per, (lists[x].size() + 3) / 4);
    const Item pad = {0, 0, item_meta(0, 0, kItemGroup)};
    std::vector<Item> all;
    all.reserve(per * 4 * kSliceCount + (size_t)(n / 32) + 64);
    for (size_t jb = 0; jb < per; ++jb)
        for (int x = 0; x < kSliceCount; ++x)
            for (size_t w = 0; w < 4; ++w) {
                const size_t i = jb * 4 + w;
                all.push_back(i < lists[x].size() ? lists[x][i] : pad);
            }
    // short rows: greedy groups of consecutive rows (at most 63 rows and EW
    // edges; medium and long rows inside add no edges), none without a
    // short row
    int64_t gstart = -1, gnnz = 0, gown = 0;
    auto close_group = [&](int64_t end) {
        if (gstart >= 0 && end > gstart && gown > 0)
            all.push_back({rowx[gstart] & kRowxMask, (int32_t)gstart,
                           item_meta((uint32_t)(end - gstart), (uint32_t)gnnz, kItemGroup)});
        gstart = -1;
        gnnz = 0;
        gown = 0;
    };
    for (int64_t r = 0; r < n; ++r) {
        const int64_t d = rp[r + 1] - rp[r];
        const bool shortrow = d <= lm;
        const int64_t ds = shortrow ? d : 0;
        if (gstart >= 0 && (r - gstart >= 63 || gnnz + ds > ew)) close_group(r);
        if (gstart < 0 && !shortrow) continue;
        if (gstart < 0) gstart = r;
        gnnz += ds;
        gown += shortrow ? 1 : 0;
    }
    close_group(n);
    if ((uint64_t)((all.size() + 3) / 4) * 256 > UINT32_MAX) {
        cleanup();
        return fail(TPA_ERR_INDEX_OVERFLOW, "too many work items for one launch");
    }
    if (!g->t_colx && (rc = dalloc(&g->t_colx, m, st)) != TPA_OK) {
        cleanup();
        return rc == TPA_ERR_OUT_OF_MEMORY ? TPA_OK : rc;
    }
    g->sched_x.release();
    g->sched_x = Schedule();
    g->sched_x_ew = 0;
    g->sched_x_none = false;
    Schedule sx;
    sx.ew = ew;
    sx.ds = std::min(32, ew);
    sx.el = ew;
    sx.chunk = (int)chunk;
    sx.eb = ew;
    sx.chunk_slot_in_item = true;
    sx.n_items = (int64_t)all.size();
    sx.n_chunk_items = slot;
    sx.n_long = (int64_t)longs.size();
    sx.n_long8 = (int64_t)longs8.size();
    rc = dalloc(&sx.items, sx.n_items, st);
    if (rc == TPA_OK && sx.n_long) rc = dalloc(&sx.longs, sx.n_long, st);
    if (rc == TPA_OK && sx.n_long8) rc = dalloc(&sx.longs8, sx.n_long8, st);
    if (rc == TPA_OK) rc = dalloc(&sx.rowptr_x, n + 1, st);
    if (rc == TPA_OK) rc = dalloc(&sx.xrel, std::max<size_t>(xrel.size(), 1), st);
    if (rc != TPA_OK) {
        sx.release();
        cleanup();
        return rc == TPA_ERR_OUT_OF_MEMORY ? TPA_OK : rc;
    }
    e = hipMemcpyAsync(d_out, seg_out.data(), sizeof(int64_t) * seg_out.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sx.rowptr_x, rowx.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        slice_scatter_kernel<<<(unsigned)((nseg + 3) / 4), 256, 0, st>>>(d_e0, d_len, nseg, d_out, g->t_colz, g->t_colx);
        short_copy_kernel<<<grid_for(n), kBlock, 0, st>>>(g->t.rowptr, sx.rowptr_x, n, g->t_colz, g->t_colx);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(sx.items, all.data(), sizeof(Item) * all.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && sx.n_long)
        e = hipMemcpyAsync(sx.longs, longs.data(), sizeof(LongRow) * longs.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && sx.n_long8)
        e = hipMemcpyAsync(sx.longs8, longs8.data(), sizeof(LongRow) * longs8.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !xrel.empty())
        e = hipMemcpyAsync(sx.xrel, xrel.data(), sizeof(int32_t) * xrel.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    cleanup();
    if (e != hipSuccess) {
        sx.release();
        return fail(TPA_ERR_HIP, std::string("sliced sweep: ") + hipGetErrorString(e));
    }
    g->sched_x = sx;
    g->sched_x_ew = ew;
    *out = &g->sched_x;
    *out_col = g->t_colx;
    return TPA_OK;
}

void SlicedAdj::release() {
    s.release();
    dfree(col);
    dfree(slot_row);
    dfree(seg_e0);
    dfree(seg_len);
    dfree(seg_out);
    *this = SlicedAdj();
}

tpa_status launch_unslice(const SlicedAdj &sa, const float *gx, float *G, hipStream_t st) {
    if (sa.nseg == 0) return TPA_OK;
    slice_gather_back_kernel<<<(unsigned)((sa.nseg + 3) / 4), 256, 0, st>>>(sa.seg_e0, sa.seg_len, sa.nseg, sa.seg_out,
                                                                              sa.from, gx, G);
    TPA_TRY_HIP(hipGetLastError());
    return TPA_OK;
}

tpa_status ensure_sliced_adj(tpa_graph *g, const int32_t *src, hipStream_t st, const SlicedAdj **out) {
    *out = nullptr;
    if (g->sliced_sweep == 0 || (g->sliced_sweep == 1 && g->n < kSliceMinN)) return TPA_OK;
    if (g->weighted || !src || g->n == 0) return TPA_OK;
    SlicedAdj &sa = g->sax;
    const int ew = choose_shape(g, 1).ew;
    if (sa.ew == ew && sa.from == src && (sa.none || sa.s.items)) {
        if (!sa.none) *out = &sa;
        return TPA_OK;
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return TPA_OK;
    const int64_t n = g->n, m = g->m;
    std::vector<int64_t> rp(n + 1);
    TPA_TRY_HIP(hipMemcpyAsync(rp.data(), g->a.rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, st));
    TPA_TRY_HIP(hipStreamSynchronize(st));
    std::vector<int32_t> lrows;
    std::vector<int64_t> first_seg, seg_e0;
    std::vector<int32_t> seg_len;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t d = rp[r + 1] - rp[r];
        if (d <= ew) continue;
        lrows.push_back((int32_t)r);
        first_seg.push_back((int64_t)seg_e0.size());
        for (int64_t off = 0; off < d; off += kSliceSegment) {
            seg_e0.push_back(rp[r] + off);
            seg_len.push_back((int32_t)std::min<int64_t>(kSliceSegment, d - off));
        }
    }
    first_seg.push_back((int64_t)seg_e0.size());
    sa.release();
    if (lrows.empty()) {
        sa.ew = ew;
        sa.from = src;
        sa.none = true;
        return TPA_OK;
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || (size_t)m * sizeof(int32_t) > free_b / 4) return TPA_OK;
    SlicedAdj nx;
    const int64_t nseg = (int64_t)seg_e0.size();
    int32_t *d_cnt = nullptr;
    auto bail = [&](tpa_status rc) {
        dfree(d_cnt);
        nx.release();
        // optional: without the memory the steps run unsliced
        return rc == TPA_ERR_OUT_OF_MEMORY ? TPA_OK : rc;
    };
    tpa_status rc = TPA_OK;
    if ((rc = dalloc(&nx.seg_e0, nseg, st)) != TPA_OK || (rc = dalloc(&nx.seg_len, nseg, st)) != TPA_OK ||
        (rc = dalloc(&d_cnt, nseg * kSliceCount, st)) != TPA_OK ||
        (rc = dalloc(&nx.seg_out, nseg * kSliceCount, st)) != TPA_OK)
        return bail(rc);
    nx.nseg = nseg;
    std::vector<int32_t> cnt((size_t)nseg * kSliceCount);
    hipError_t e = hipMemcpyAsync(nx.seg_e0, seg_e0.data(), sizeof(int64_t) * nseg, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(nx.seg_len, seg_len.data(), sizeof(int32_t) * nseg, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        slice_count_kernel<<<(unsigned)((nseg + 3) / 4), 256, 0, st>>>(nx.seg_e0, nx.seg_len, nseg, src, d_cnt);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(cnt.data(), d_cnt, sizeof(int32_t) * cnt.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bail(fail(TPA_ERR_HIP, std::string("sliced adjoint: ") + hipGetErrorString(e)));
    // in place: slice x's run of a long row follows slices 0..x-1 within
    // the row, cut into chunks of at most 4*EW edges
    const int64_t chunk = 4 * (int64_t)ew;
    std::vector<int64_t> seg_out((size_t)nseg * kSliceCount);
    std::vector<Item> lists[kSliceCount];
    std::vector<int32_t> slot_row;
    std::vector<LongRow> longs;
    int64_t slot = 0;
    for (size_t l = 0; l < lrows.size(); ++l) {
        const int64_t r = lrows[l], d = rp[r + 1] - rp[r];
        int64_t tot[kSliceCount] = {};
        for (int64_t sg = first_seg[l]; sg < first_seg[l + 1]; ++sg)
            for (int x = 0; x < kSliceCount; ++x) tot[x] += cnt[(size_t)sg * kSliceCount + x];
        int64_t sum = 0;
        for (int x = 0; x < kSliceCount; ++x) sum += tot[x];
        if (sum != d) return bail(fail(TPA_ERR_HIP, "sliced adjoint: slice counts do not add up to the row length"));
        const int64_t first_slot = slot;
        int64_t start = rp[r];
        for (int x = 0; x < kSliceCount; ++x) {
            int64_t at = start;
            for (int64_t sg = first_seg[l]; sg < first_seg[l + 1]; ++sg) {
                seg_out[(size_t)sg * kSliceCount + x] = at;
                at += cnt[(size_t)sg * kSliceCount + x];
            }
            for (int64_t off = 0; off < tot[x]; off += chunk) {
                const int64_t len = std::min(chunk, tot[x] - off);
                lists[x].push_back({start + off, (int32_t)slot, item_meta(1, (uint32_t)len, kItemChunk)});
                slot_row.push_back((int32_t)r);
                ++slot;
            }
            start += tot[x];
        }
        if (slot > INT32_MAX) return bail(fail(TPA_ERR_INDEX_OVERFLOW, "too many chunk items"));
        longs.push_back({(int32_t)r, (int32_t)(slot - first_slot), (int32_t)first_slot, 0});
    }
    size_t per = 0;
    for (int x = 0; x < kSliceCount; ++x) per = std::max(per, (lists[x].size() + 3) / 4);
    const Item pad = {0, 0, item_meta(0, 0, kItemGroup)};
    std::vector<Item> all;
    all.reserve(per * 4 * kSliceCount + (size_t)(m / std::max(ew, 1)) + 64);
    for (size_t jb = 0; jb < per; ++jb)
        for (int x = 0; x < kSliceCount; ++x)
            for (size_t w = 0; w < 4; ++w) {
                const size_t i = jb * 4 + w;
                all.push_back(i < lists[x].size() ? lists[x][i] : pad);
            }
    int64_t gstart = -1, gnnz = 0;
    auto close_group = [&](int64_t end) {
        if (gstart >= 0 && end > gstart)
            all.push_back({rp[gstart], (int32_t)gstart, item_meta((uint32_t)(end - gstart), (uint32_t)gnnz, kItemGroup)});
        gstart = -1;
        gnnz = 0;
    };
    for (int64_t r = 0; r < n; ++r) {
        const int64_t d = rp[r + 1] - rp[r];
        if (d > ew) {
            close_group(r);
            continue;
        }
        if (gstart >= 0 && (r - gstart >= 63 || gnnz + d > ew)) close_group(r);
        if (gstart < 0) gstart = r;
        gnnz += d;
    }
    close_group(n);
    if ((uint64_t)((all.size() + 3) / 4) * 256 > UINT32_MAX)
        return bail(fail(TPA_ERR_INDEX_OVERFLOW, "too many work items for one launch"));
    Schedule &sx = nx.s;
    sx.ew = ew;
    sx.ds = std::min(32, ew);
    sx.el = ew;
    sx.chunk = (int)chunk;
    sx.eb = 0;
    sx.chunk_slot_in_item = true;
    sx.n_items = (int64_t)all.size();
    sx.n_chunk_items = slot;
    sx.n_long = (int64_t)longs.size();
    if ((rc = dalloc(&sx.items, sx.n_items, st)) != TPA_OK || (rc = dalloc(&sx.longs, sx.n_long, st)) != TPA_OK ||
        (rc = dalloc(&nx.slot_row, (size_t)std::max<int64_t>(slot, 1), st)) != TPA_OK ||
        (rc = dalloc(&nx.col, m, st)) != TPA_OK)
        return bail(rc);
    e = hipMemcpyAsync(nx.seg_out, seg_out.data(), sizeof(int64_t) * seg_out.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(nx.col, src, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) {
        slice_scatter_kernel<<<(unsigned)((nseg + 3) / 4), 256, 0, st>>>(nx.seg_e0, nx.seg_len, nseg, nx.seg_out, src,
                                                                          nx.col);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(sx.items, all.data(), sizeof(Item) * all.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sx.longs, longs.data(), sizeof(LongRow) * longs.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(nx.slot_row, slot_row.data(), sizeof(int32_t) * slot_row.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(d_cnt);
    d_cnt = nullptr;
    if (e != hipSuccess) return bail(fail(TPA_ERR_HIP, std::string("sliced adjoint: ") + hipGetErrorString(e)));
    nx.from = src;
    nx.ew = ew;
    sa = nx;
    *out = &sa;
    return TPA_OK;
}

void drop_group_order(tpa_graph *g) {
    // the copies stay allocated (query graphs captured before may read them)
    for (auto &kv : g->sched_t) kv.second.colg_src = nullptr;
    for (auto &kv : g->sched_a) kv.second.colg_src = nullptr;
}

// ------------------------------------------------------------------ schedule
void Schedule::release() {
    dfree(items);
    dfree(longs);
    dfree(colg);
    dfree(rowptr_x);
    dfree(xrel);
    dfree(longs8);
    items = nullptr;
    longs = nullptr;
    colg = nullptr;
    rowptr_x = nullptr;
    xrel = nullptr;
    longs8 = nullptr;
    colg_src = nullptr;
    colg_from = nullptr;
}

// Rows of A~^T are cut into wave items, heaviest first so they start early:
//   * rows of EL+1..EB edges: one block item per row (4 aligned slots);
//   * rows longer than max(EL, EB) edges: chunks of CH edges (chunk items);
//   * rows of EW+1..EL edges: one item per row;
//   * runs of rows with <= EW edges: greedy groups of at most 63 rows and
//     EW edges (rows of <= DS = 32 edges are summed one lane per row, longer
//     ones by the whole wave).
const Schedule *find_schedule(const tpa_graph *g, SchedShape shape, bool over_a) {
    const auto &cache = over_a ? g->sched_a : g->sched_t;
    auto it = cache.find(shape);
    return it == cache.end() ? nullptr : &it->second;
}

tpa_status get_schedule(tpa_graph *g, SchedShape shape, hipStream_t st, const Schedule **out, bool over_a) {
    auto &cache = over_a ? g->sched_a : g->sched_t;
    const int64_t *rowptr_dev = over_a ? g->a.rowptr : g->t.rowptr;
    auto it = cache.find(shape);
    if (it != cache.end()) { *out = &it->second; return TPA_OK; }
    const int64_t n = g->n;
    const int ew = shape.ew, el = shape.el, chunk = shape.chunk;
    const int64_t eb = std::max(shape.eb, el);
    if (ew < 1 || el < ew || chunk < 1 || el > (1 << 16) || chunk > (1 << 16) || eb > (1 << 17) - 1)
        return fail(TPA_ERR_INVALID_ARG, "bad schedule shape");
    const int ds = std::min(32, ew);
    std::vector<int64_t> rp(n + 1);
    TPA_TRY_HIP(hipMemcpyAsync(rp.data(), rowptr_dev, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, st));
    TPA_TRY_HIP(hipStreamSynchronize(st));
    std::vector<Item> blocks, chunks, rows, groups;
    std::vector<LongRow> longs;
    int64_t gstart = -1, gnnz = 0;
    auto close_group = [&](int64_t end) {
        if (gstart >= 0 && end > gstart)
            groups.push_back({rp[gstart], (int32_t)gstart, item_meta((uint32_t)(end - gstart), (uint32_t)gnnz, kItemGroup)});
        gstart = -1;
        gnnz = 0;
    };
    for (int64_t r = 0; r < n; ++r) {
        const int64_t d = rp[r + 1] - rp[r];
        if (d > el && d <= eb) {
            close_group(r);
            const Item b = {rp[r], (int32_t)r, item_meta(1, (uint32_t)d, kItemBlock)};
            for (int k = 0; k < 4; ++k) blocks.push_back(b);
        } else if (d > el) {
            close_group(r);
            const int64_t nch = (d + chunk - 1) / chunk;
            if ((int64_t)chunks.size() + nch > INT32_MAX) return fail(TPA_ERR_INDEX_OVERFLOW, "too many chunk items");
            longs.push_back({(int32_t)r, (int32_t)nch, (int32_t)chunks.size(), 0});
            for (int64_t ch = 0; ch < nch; ++ch) {
                const int64_t e0 = rp[r] + ch * chunk;
                const int64_t len = std::min<int64_t>(chunk, rp[r + 1] - e0);
                chunks.push_back({e0, (int32_t)(longs.size() - 1), item_meta(1, (uint32_t)len, kItemChunk)});
            }
        } else if (d > ew) {
            close_group(r);
            rows.push_back({rp[r], (int32_t)r, item_meta(1, (uint32_t)d, kItemRow)});
        } else {
            if (gstart >= 0 && (r - gstart >= 63 || gnnz + d > ew)) close_group(r);
            if (gstart < 0) gstart = r;
            gnnz += d;
        }
    }
    close_group(n);
    Schedule s;
    s.ew = ew;
    s.ds = ds;
    s.el = el;
    s.chunk = chunk;
    s.eb = (int)eb;
    // block items first (4-aligned), then chunks: chunk item i sits at index
    // blocks.size() + i, which the finish pass's first_item must include
    for (auto &lr : longs) lr.first_item += (int32_t)blocks.size();
    std::vector<Item> all;
    all.reserve(blocks.size() + chunks.size() + rows.size() + groups.size());
    all.insert(all.end(), blocks.begin(), blocks.end());
    all.insert(all.end(), chunks.begin(), chunks.end());
    all.insert(all.end(), rows.begin(), rows.end());
    all.insert(all.end(), groups.begin(), groups.end());
    s.n_items = (int64_t)all.size();
    s.n_chunk_items = (int64_t)(blocks.size() + chunks.size());  // partial slots are item indices
    s.n_long = (int64_t)longs.size();
    if (s.n_items > 0) {
        TPA_TRY(dalloc(&s.items, s.n_items, st));
        TPA_TRY_HIP(hipMemcpyAsync(s.items, all.data(), sizeof(Item) * s.n_items, hipMemcpyHostToDevice, st));
    }
    if (s.n_long > 0) {
        TPA_TRY(dalloc(&s.longs, s.n_long, st));
        TPA_TRY_HIP(hipMemcpyAsync(s.longs, longs.data(), sizeof(LongRow) * s.n_long, hipMemcpyHostToDevice, st));
    }
    TPA_TRY_HIP(hipStreamSynchronize(st));
    auto ins = cache.emplace(shape, s);
    *out = &ins.first->second;
    return TPA_OK;
}

void graph_release(tpa_graph *g) {
    dfree(g->node_block); dfree(g->restart_pr);
    dfree(g->a.rowptr); dfree(g->a.col); dfree(g->a.w);
    dfree(g->t.rowptr); dfree(g->t.col); dfree(g->t.w);
    dfree(g->t2a); dfree(g->inv_deg); dfree(g->padded);
    dfree(g->zperm); dfree(g->zinv); dfree(g->t_colz); dfree(g->t_locz); dfree(g->t_wz);
    g->zinv = nullptr;
    dfree(g->lrank); dfree(g->a_colr);
    g->lrank = nullptr;
    g->a_colr = nullptr;
    dfree(g->t_colx);
    g->t_colx = nullptr;
    g->sax.release();
    g->sched_x.release();
    g->sched_x_ew = 0;
    g->sched_x_none = false;
    g->zperm = nullptr;
    g->t_colz = nullptr;
    g->t_locz = nullptr;
    g->t_wz = nullptr;
    dfree(g->str); dfree(g->ws); dfree(g->dev_err); dfree(g->xiter);
    tile_buf_free(&g->tbuf);
    for (auto &b : g->adj_cache) dfree(b.first);
    g->adj_cache.clear();
    g->xiter = nullptr;
    g->xiter_K = 0;
    g->xiter_cap = 0;
    for (auto &kv : g->sched_t) kv.second.release();
    for (auto &kv : g->sched_a) kv.second.release();
    g->sched_t.clear();
    g->sched_a.clear();
}

}  // namespace tpa

using namespace tpa;

// ==================================================================== C ABI
extern "C" tpa_status tpa_graph_rmat(int scale, int64_t n_nodes, int64_t samples, uint64_t seed,
                                     double a, double b, double c, hipStream_t st,
                                     tpa_graph_t *out) {
    if (!out) return fail(TPA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (scale < 1 || scale > 31) return fail(TPA_ERR_INVALID_ARG, "scale must be in 1..31");
    if (samples < 0) return fail(TPA_ERR_INVALID_ARG, "samples must be >= 0");
    if (!(a >= 0 && b >= 0 && c >= 0 && a + b + c <= 1.0))
        return fail(TPA_ERR_INVALID_ARG, "R-MAT probabilities must be >= 0 with a+b+c <= 1");
    const int64_t full = int64_t(1) << scale;
    if (n_nodes == 0) n_nodes = full;
    if (n_nodes < 1 || n_nodes > full) return fail(TPA_ERR_INVALID_ARG, "n_nodes must be in 1..2^scale");
    if (n_nodes > INT32_MAX) return fail(TPA_ERR_INDEX_OVERFLOW, "node ids must fit int32");
    const uint32_t t0 = (uint32_t)std::llround(a * 4294967296.0);
    const uint32_t t1 = (uint32_t)std::llround((a + b) * 4294967296.0);
    const uint32_t t2 = (uint32_t)std::llround((a + b + c) * 4294967296.0);

    tpa_graph *g = new tpa_graph();
    TPA_TRY_HIP(hipGetDevice(&g->device));
    g->n = n_nodes;
    g->bits = key_bits(n_nodes);
    uint64_t *keys = nullptr;
    tpa_status s = dalloc(&keys, std::max<int64_t>(samples, 1), st);
    if (s != TPA_OK) { delete g; return s; }
    if (n_nodes == full) {
        if (samples > 0)
            rmat_kernel<<<grid_for(samples), kBlock, 0, st>>>(seed, scale, 0, samples, t0, t1, t2,
                                                             n_nodes, g->bits, keys, nullptr);
    } else {
        // rejection: raw batches, keep accepted samples in counter order
        int64_t got = 0, raw = 0;
        const int64_t max_raw = 64 * samples + 1024;
        while (got < samples && raw < max_raw) {
            const int64_t batch = std::min<int64_t>(max_raw - raw, std::max<int64_t>(2 * (samples - got), 1 << 16));
            uint64_t *bk = nullptr;
            int64_t *fl = nullptr, *ps = nullptr;
            if ((s = dalloc(&bk, batch, st)) != TPA_OK || (s = dalloc(&fl, batch, st)) != TPA_OK ||
                (s = dalloc(&ps, batch, st)) != TPA_OK) {
                dfree(bk); dfree(fl); dfree(ps); dfree(keys); delete g; return s;
            }
            rmat_kernel<<<grid_for(batch), kBlock, 0, st>>>(seed, scale, raw, batch, t0, t1, t2, n_nodes,
                                                           g->bits, bk, fl);
            s = exclusive_scan_i64(fl, ps, batch, st);
            if (s == TPA_OK) {
                const int64_t acc = read_back(ps + batch - 1, st) + read_back(fl + batch - 1, st);
                compact_kernel<<<grid_for(batch), kBlock, 0, st>>>(bk, fl, ps, batch, samples, got, keys);
                (void)hipStreamSynchronize(st);
                got = std::min(samples, got + acc);
            }
            dfree(bk); dfree(fl); dfree(ps);
            if (s != TPA_OK) { dfree(keys); delete g; return s; }
            raw += batch;
        }
        if (got < samples) {
            dfree(keys); delete g;
            return fail(TPA_ERR_INVALID_ARG, "R-MAT rejection did not reach the requested sample count");
        }
    }
    if ((s = graph_alloc_common(g, st)) != TPA_OK || (s = build_from_keys(g, keys, samples, st)) != TPA_OK) {
        graph_release(g); delete g; return s;
    }
    *out = g;
    return TPA_OK;
}

extern "C" tpa_status tpa_graph_from_edges(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                                           int device_ptrs, hipStream_t st, tpa_graph_t *out) {
    if (!out) return fail(TPA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || m < 0) return fail(TPA_ERR_INVALID_ARG, "need n >= 1 and m >= 0");
    if (n > INT32_MAX) return fail(TPA_ERR_INDEX_OVERFLOW, "node ids must fit int32");
    if (m > 0 && (!src || !dst)) return fail(TPA_ERR_INVALID_ARG, "src/dst is NULL");
    tpa_graph *g = new tpa_graph();
    TPA_TRY_HIP(hipGetDevice(&g->device));
    g->n = n;
    g->bits = key_bits(n);
    uint64_t *keys = nullptr;
    int32_t *ds = nullptr, *dd = nullptr, *bad = nullptr;
    tpa_status s = TPA_OK;
    auto bail = [&](tpa_status e) {
        dfree(keys); if (!device_ptrs) { dfree(ds); dfree(dd); } dfree(bad);
        graph_release(g); delete g; return e;
    };
    if ((s = dalloc(&keys, std::max<int64_t>(m, 1), st)) != TPA_OK) return bail(s);
    if ((s = dalloc(&bad, 1, st)) != TPA_OK) return bail(s);
    if (m > 0) {
        if (device_ptrs) {
            ds = const_cast<int32_t *>(src);
            dd = const_cast<int32_t *>(dst);
        } else {
            if ((s = dalloc(&ds, m, st)) != TPA_OK || (s = dalloc(&dd, m, st)) != TPA_OK) return bail(s);
            if (hipMemcpyAsync(ds, src, sizeof(int32_t) * m, hipMemcpyHostToDevice, st) != hipSuccess ||
                hipMemcpyAsync(dd, dst, sizeof(int32_t) * m, hipMemcpyHostToDevice, st) != hipSuccess)
                return bail(fail(TPA_ERR_HIP, "edge upload failed"));
        }
        (void)hipMemsetAsync(bad, 0, sizeof(int32_t), st);
        pack_edges_kernel<<<grid_for(m), kBlock, 0, st>>>(ds, dd, m, g->bits, n, keys, bad);
        const int32_t isbad = read_back(bad, st);
        if (!device_ptrs) { dfree(ds); dfree(dd); }
        ds = dd = nullptr;
        if (isbad) return bail(fail(TPA_ERR_INVALID_ARG, "edge endpoint outside [0, n)"));
    }
    dfree(bad);
    bad = nullptr;
    if ((s = graph_alloc_common(g, st)) != TPA_OK) return bail(s);
    s = build_from_keys(g, keys, m, st);
    keys = nullptr;
    if (s != TPA_OK) return bail(s);
    *out = g;
    return TPA_OK;
}

extern "C" tpa_status tpa_graph_pack(const tpa_graph_t *gs, int count, hipStream_t st, tpa_graph_t *out) {
    if (!out) return fail(TPA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!gs || count < 1) return fail(TPA_ERR_INVALID_ARG, "need at least one graph");
    int64_t n = 0, m = 0;
    int64_t maxd = 0;
    for (int i = 0; i < count; ++i) {
        if (!gs[i]) return fail(TPA_ERR_INVALID_ARG, "NULL graph handle");
        n += gs[i]->n;
        m += gs[i]->m;
        maxd = std::max(maxd, gs[i]->max_outdeg);
    }
    if (n > INT32_MAX) return fail(TPA_ERR_INDEX_OVERFLOW, "packed node ids must fit int32");
    tpa_graph *g = new tpa_graph();
    TPA_TRY_HIP(hipGetDevice(&g->device));
    g->n = n;
    g->m = m;
    g->max_outdeg = maxd;
    g->bits = key_bits(n);
    tpa_status s;
    auto bail = [&](tpa_status e) { graph_release(g); delete g; return e; };
    if ((s = graph_alloc_common(g, st)) != TPA_OK) return bail(s);
    if ((s = dalloc(&g->a.rowptr, n + 1, st)) != TPA_OK || (s = dalloc(&g->a.col, m, st)) != TPA_OK ||
        (s = dalloc(&g->t.rowptr, n + 1, st)) != TPA_OK || (s = dalloc(&g->t.col, m, st)) != TPA_OK ||
        (s = dalloc(&g->inv_deg, n, st)) != TPA_OK || (s = dalloc(&g->padded, n, st)) != TPA_OK ||
        (s = dalloc(&g->node_block, n, st)) != TPA_OK || (s = dalloc(&g->restart_pr, n, st)) != TPA_OK)
        return bail(s);
    g->nblocks = count;
    g->block_off.assign(count + 1, 0);
    int64_t no = 0, eo = 0;
    for (int i = 0; i < count; ++i) {
        const tpa_graph *h = gs[i];
        offset_i64_kernel<<<grid_for(h->n), kBlock, 0, st>>>(h->a.rowptr, h->n, eo, g->a.rowptr + no);
        offset_i64_kernel<<<grid_for(h->n), kBlock, 0, st>>>(h->t.rowptr, h->n, eo, g->t.rowptr + no);
        offset_i32_kernel<<<grid_for(h->m), kBlock, 0, st>>>(h->a.col, h->m, (int32_t)no, g->a.col + eo);
        offset_i32_kernel<<<grid_for(h->m), kBlock, 0, st>>>(h->t.col, h->m, (int32_t)no, g->t.col + eo);
        if (hipMemcpyAsync(g->inv_deg + no, h->inv_deg, sizeof(float) * h->n, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(g->padded + no, h->padded, h->n, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return bail(fail(TPA_ERR_HIP, "pack copy failed"));
        fill_block_kernel<<<grid_for(h->n), kBlock, 0, st>>>(g->node_block, g->restart_pr, no, h->n, i,
                                                            (float)(1.0 / (double)h->n));
        no += h->n;
        eo += h->m;
        g->block_off[i + 1] = no;
    }
    const int64_t tail[1] = {m};
    TPA_TRY_HIP(hipMemcpyAsync(g->a.rowptr + n, tail, sizeof(int64_t), hipMemcpyHostToDevice, st));
    TPA_TRY_HIP(hipMemcpyAsync(g->t.rowptr + n, tail, sizeof(int64_t), hipMemcpyHostToDevice, st));
    TPA_TRY_HIP(hipStreamSynchronize(st));
    TPA_TRY_HIP(hipGetLastError());
    *out = g;
    return TPA_OK;
}

extern "C" tpa_status tpa_graph_destroy(tpa_graph_t g) {
    if (!g) return TPA_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();
    graph_release(g);
    if (cur != g->device) (void)hipSetDevice(cur);
    delete g;
    return TPA_OK;
}

extern "C" tpa_status tpa_graph_info(tpa_graph_t g, int64_t *n, int64_t *m, int64_t *nblocks) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (nblocks) *nblocks = g->nblocks;
    return TPA_OK;
}

extern "C" tpa_status tpa_graph_device_bytes(tpa_graph_t g, size_t *bytes) {
    if (!g || !bytes) return fail(TPA_ERR_INVALID_ARG, "NULL argument");
    const size_t n = (size_t)g->n, m = (size_t)g->m;
    size_t b = 0;
    auto add = [&b](const void *p, size_t sz) {
        if (p) b += sz;
    };
    for (const Csr *c : {&g->a, &g->t}) {
        add(c->rowptr, sizeof(int64_t) * (n + 1));
        add(c->col, sizeof(int32_t) * m);
        add(c->w, sizeof(float) * m);
    }
    add(g->t2a, sizeof(int64_t) * m);
    add(g->inv_deg, sizeof(float) * n);
    add(g->padded, n);
    add(g->node_block, sizeof(int32_t) * n);
    add(g->restart_pr, sizeof(float) * n);
    add(g->zperm, sizeof(int32_t) * n);
    add(g->zinv, sizeof(int32_t) * n);
    add(g->t_colz, sizeof(int32_t) * m);
    add(g->t_locz, sizeof(int32_t) * m);
    add(g->t_wz, sizeof(float) * m);
    add(g->lrank, sizeof(int32_t) * n);
    add(g->a_colr, sizeof(int32_t) * m);
    add(g->t_colx, sizeof(int32_t) * m);
    add(g->sched_x.items, sizeof(Item) * (size_t)g->sched_x.n_items);
    add(g->sched_x.longs, sizeof(LongRow) * (size_t)g->sched_x.n_long);
    add(g->sched_x.longs8, sizeof(LongRow) * (size_t)g->sched_x.n_long8);
    add(g->sched_x.rowptr_x, sizeof(int64_t) * (n + 1));
    add(g->sax.col, sizeof(int32_t) * m);
    add(g->sax.s.items, sizeof(Item) * (size_t)g->sax.s.n_items);
    add(g->str, sizeof(float) * n);
    add(g->dev_err, sizeof(int32_t));
    add(g->ws, g->ws_bytes);
    add(g->tbuf.base, g->tbuf.bytes);
    add(g->xiter, sizeof(float) * g->xiter_cap);
    for (const auto &c : g->adj_cache) add(c.first, c.second);
    for (const auto *cache : {&g->sched_t, &g->sched_a}) {
        for (const auto &kv : *cache) {
            const Schedule &s = kv.second;
            add(s.items, sizeof(Item) * (size_t)s.n_items);
            add(s.longs, sizeof(LongRow) * (size_t)s.n_long);
            add(s.colg, sizeof(int32_t) * m);
        }
    }
    *bytes = b;
    return TPA_OK;
}

extern "C" tpa_status tpa_graph_version(tpa_graph_t g, uint64_t *version) {
    if (!g || !version) return fail(TPA_ERR_INVALID_ARG, "NULL argument");
    *version = g->version;
    return TPA_OK;
}

extern "C" tpa_status tpa_graph_blocks(tpa_graph_t g, int64_t *offsets) {
    if (!g || !offsets) return fail(TPA_ERR_INVALID_ARG, "NULL argument");
    std::copy(g->block_off.begin(), g->block_off.end(), offsets);
    return TPA_OK;
}

extern "C" tpa_status tpa_graph_export(tpa_graph_t g, int transpose, int64_t *row_ptr, int32_t *col,
                                       float *w, hipStream_t st) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    const Csr &c = transpose ? g->t : g->a;
    if (row_ptr)
        TPA_TRY_HIP(hipMemcpyAsync(row_ptr, c.rowptr, sizeof(int64_t) * (g->n + 1), hipMemcpyDeviceToDevice, st));
    if (col) TPA_TRY_HIP(hipMemcpyAsync(col, c.col, sizeof(int32_t) * g->m, hipMemcpyDeviceToDevice, st));
    if (w) {
        if (c.w) {
            TPA_TRY_HIP(hipMemcpyAsync(w, c.w, sizeof(float) * g->m, hipMemcpyDeviceToDevice, st));
        } else {
            uniform_w_kernel<<<grid_for(g->n), kBlock, 0, st>>>(c.rowptr, c.col, g->inv_deg, g->n, transpose, w);
            TPA_TRY_HIP(hipGetLastError());
        }
    }
    return TPA_OK;
}

extern "C" tpa_status tpa_graph_padded(tpa_graph_t g, uint8_t *mask, hipStream_t st) {
    if (!g || !mask) return fail(TPA_ERR_INVALID_ARG, "NULL argument");
    TPA_TRY_HIP(hipMemcpyAsync(mask, g->padded, g->n, hipMemcpyDeviceToDevice, st));
    return TPA_OK;
}

extern "C" tpa_status tpa_graph_set_logits(tpa_graph_t g, const float *theta, hipStream_t st) {
    if (!g) return fail(TPA_ERR_INVALID_ARG, "graph is NULL");
    g->preprocessed = false;
    g->xiter_K = 0;
    ++g->version;
    if (!theta) {
        dfree(g->a.w); dfree(g->t.w);
        g->a.w = g->t.w = nullptr;
        g->weighted = false;
        return TPA_OK;
    }
    TPA_TRY(ensure_t2a(g, st));
    if (!g->a.w) TPA_TRY(dalloc(&g->a.w, g->m, st));
    if (!g->t.w) TPA_TRY(dalloc(&g->t.w, g->m, st));
    const int64_t threads = g->n * 64;
    softmax_rows_kernel<<<grid_for(threads), kBlock, 0, st>>>(g->a.rowptr, g->n, theta, g->a.w);
    gather_w_kernel<<<grid_for(g->m), kBlock, 0, st>>>(g->a.w, g->t2a, g->m, g->t.w);
    TPA_TRY_HIP(hipGetLastError());
    g->weighted = true;
    g->t_wz_valid = false;
    return TPA_OK;
}
