/*
 * TPA oracle -- plain, slow, single-threaded FP64 reference of the TPA hot
 * path (Yoon, Jung, Kang, "TPA: Fast, Scalable, and Accurate Method for
 * Approximate Random Walk with Restart on Billion Scale Graphs").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it (through oracle/__init__.py).
 * It shares no code, header, table or helper with the HIP path.
 *
 * Every function follows the paper's notation:
 *   A~    row-normalised adjacency (Section 2, Table 1)
 *   x(i)  interim score vector of cumulative power iteration (Section 2.3)
 *   r     accumulated score vector, family / neighbor / stranger parts
 *         (Section 3, the three-part split of the CPI sum)
 *
 * Graph construction (a synthetic stand-in for the paper's input graphs):
 *   R-MAT edge sampling with a counter-based SplitMix64 hash, duplicate
 *   edges merged, one self-loop added on every node without out-edges
 *   (so that A~ is row stochastic, which Theorem 1 and Lemma 2 assume).
 *
 * Parity status of each function is documented in oracle/__init__.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Counter-based hash: the SplitMix64 output function (Steele, Lea, Flood,  */
/* "Fast splittable pseudorandom number generators", OOPSLA 2014).          */
/* The j-th output (j = 0, 1, ...) of a SplitMix64 generator seeded with    */
/* `seed` is mix(seed + (j + 1) * golden_gamma).                            */
/* ------------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t seed, uint64_t j)
{
    uint64_t z = seed + (j + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* R-MAT quadrant thresholds over [0, 2^32): round(cumulative p * 2^32). */
static void rmat_thresholds(double a, double b, double c, uint32_t th[3])
{
    th[0] = (uint32_t)llround(a * 4294967296.0);
    th[1] = (uint32_t)llround((a + b) * 4294967296.0);
    th[2] = (uint32_t)llround((a + b + c) * 4294967296.0);
}

/*
 * R-MAT sampling.  Raw sample e draws `scale` quadrants, most significant
 * bit first; level l uses the top 32 bits of hash(seed, e*scale + l).
 * Quadrant 0 (prob a) = (u bit 0, v bit 0), 1 (b) = (0,1), 2 (c) = (1,0),
 * 3 (d) = (1,1).  A sample whose endpoint is >= n_nodes is rejected and the
 * raw counter moves on.  Stops when `want` samples are accepted or
 * `max_raw` raw samples were drawn.  Returns the number accepted.
 */
int64_t orc_rmat(int scale, int64_t n_nodes, int64_t want, uint64_t seed,
                 double a, double b, double c, int64_t max_raw,
                 int32_t *src, int32_t *dst, int64_t *raw_used)
{
    uint32_t th[3];
    rmat_thresholds(a, b, c, th);
    int64_t got = 0, e = 0;
    for (; e < max_raw && got < want; ++e) {
        uint64_t u = 0, v = 0;
        for (int l = 0; l < scale; ++l) {
            uint32_t r = (uint32_t)(orc_splitmix64(seed, (uint64_t)e * (uint64_t)scale + (uint64_t)l) >> 32);
            int q = (r >= th[0]) + (r >= th[1]) + (r >= th[2]);
            u = (u << 1) | (uint64_t)(q >> 1);
            v = (v << 1) | (uint64_t)(q & 1);
        }
        if ((int64_t)u < n_nodes && (int64_t)v < n_nodes) {
            src[got] = (int32_t)u;
            dst[got] = (int32_t)v;
            ++got;
        }
    }
    if (raw_used) *raw_used = e;
    return got;
}

/* ------------------------------------------------------------------------ */
/* Graph: A~ stored by rows (out-edges of u, ascending v) and A~^T stored by */
/* rows (in-edges of v, ascending u), plus the map from an A~^T entry to    */
/* the same edge's A~ entry.  Weights live in A~ order.                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n, m;
    int64_t *a_rowptr; /* n+1 */
    int32_t *a_col;    /* m   */
    double  *a_w;      /* m, A~_uv */
    int64_t *t_rowptr; /* n+1 */
    int32_t *t_col;    /* m   */
    int64_t *t2a;      /* m   */
    uint8_t *padded;   /* n: 1 if a self-loop was added (no out-edges) */
} orc_graph;

static int cmp_u64(const void *x, const void *y)
{
    uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return (a > b) - (a < b);
}

void orc_graph_free(orc_graph *g)
{
    if (!g) return;
    free(g->a_rowptr); free(g->a_col); free(g->a_w);
    free(g->t_rowptr); free(g->t_col); free(g->t2a); free(g->padded);
    free(g);
}

/* Row-normalised weights A~_uv = 1 / outdeg(u). */
static void uniform_weights(orc_graph *g)
{
    for (int64_t u = 0; u < g->n; ++u) {
        int64_t d = g->a_rowptr[u + 1] - g->a_rowptr[u];
        for (int64_t e = g->a_rowptr[u]; e < g->a_rowptr[u + 1]; ++e)
            g->a_w[e] = 1.0 / (double)d;
    }
}

/*
 * Build from an edge list (node ids in [0, n)): sort the (u, v) pairs,
 * drop duplicates, add (u, u) for every u with no out-edge, then lay out
 * A~ by rows and A~^T by rows.  Returns NULL on bad input / no memory.
 */
orc_graph *orc_graph_build(int64_t n, int64_t m_in, const int32_t *src, const int32_t *dst)
{
    if (n <= 0 || m_in < 0) return NULL;
    for (int64_t i = 0; i < m_in; ++i)
        if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return NULL;

    uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m_in > 0 ? m_in : 1));
    if (!key) return NULL;
    for (int64_t i = 0; i < m_in; ++i)
        key[i] = ((uint64_t)(uint32_t)src[i] << 32) | (uint64_t)(uint32_t)dst[i];
    qsort(key, (size_t)m_in, sizeof(uint64_t), cmp_u64);
    int64_t mu = 0;
    for (int64_t i = 0; i < m_in; ++i)
        if (i == 0 || key[i] != key[i - 1]) key[mu++] = key[i];

    orc_graph *g = (orc_graph *)calloc(1, sizeof(orc_graph));
    if (!g) { free(key); return NULL; }
    g->n = n;
    g->padded = (uint8_t *)calloc((size_t)n, 1);
    int64_t *deg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    for (int64_t i = 0; i < mu; ++i) deg[key[i] >> 32]++;
    int64_t npad = 0;
    for (int64_t u = 0; u < n; ++u)
        if (deg[u] == 0) { g->padded[u] = 1; npad++; }
    g->m = mu + npad;

    g->a_rowptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    g->a_col = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->m);
    g->a_w = (double *)malloc(sizeof(double) * (size_t)g->m);
    g->t_rowptr = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    g->t_col = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->m);
    g->t2a = (int64_t *)malloc(sizeof(int64_t) * (size_t)g->m);
    if (!g->padded || !deg || !g->a_rowptr || !g->a_col || !g->a_w ||
        !g->t_rowptr || !g->t_col || !g->t2a) {
        free(deg); free(key); orc_graph_free(g); return NULL;
    }

    /* A~ by rows: walk sorted unique keys, emit the self-loop for padded rows. */
    int64_t k = 0, pos = 0;
    for (int64_t u = 0; u < n; ++u) {
        g->a_rowptr[u] = pos;
        if (g->padded[u]) {
            g->a_col[pos++] = (int32_t)u;
        } else {
            while (k < mu && (int64_t)(key[k] >> 32) == u)
                g->a_col[pos++] = (int32_t)(key[k++] & 0xffffffffu);
        }
    }
    g->a_rowptr[n] = pos;

    /* A~^T by rows: count in-degrees, prefix sum, then place edges while
       walking A~ in (u asc, v asc) order, so each row of A~^T is u-ascending. */
    for (int64_t e = 0; e < g->m; ++e) g->t_rowptr[g->a_col[e] + 1]++;
    for (int64_t v = 0; v < n; ++v) g->t_rowptr[v + 1] += g->t_rowptr[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    memcpy(fill, g->t_rowptr, sizeof(int64_t) * (size_t)n);
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = g->a_rowptr[u]; e < g->a_rowptr[u + 1]; ++e) {
            int64_t p = fill[g->a_col[e]]++;
            g->t_col[p] = (int32_t)u;
            g->t2a[p] = e;
        }
    free(fill);
    free(deg);
    free(key);
    uniform_weights(g);
    return g;
}

int64_t orc_graph_n(const orc_graph *g) { return g->n; }
int64_t orc_graph_m(const orc_graph *g) { return g->m; }

void orc_graph_export(const orc_graph *g, int64_t *a_rowptr, int32_t *a_col, double *a_w,
                      int64_t *t_rowptr, int32_t *t_col, int64_t *t2a, uint8_t *padded)
{
    if (a_rowptr) memcpy(a_rowptr, g->a_rowptr, sizeof(int64_t) * (size_t)(g->n + 1));
    if (a_col) memcpy(a_col, g->a_col, sizeof(int32_t) * (size_t)g->m);
    if (a_w) memcpy(a_w, g->a_w, sizeof(double) * (size_t)g->m);
    if (t_rowptr) memcpy(t_rowptr, g->t_rowptr, sizeof(int64_t) * (size_t)(g->n + 1));
    if (t_col) memcpy(t_col, g->t_col, sizeof(int32_t) * (size_t)g->m);
    if (t2a) memcpy(t2a, g->t2a, sizeof(int64_t) * (size_t)g->m);
    if (padded) memcpy(padded, g->padded, (size_t)g->n);
}

/*
 * Per-edge logits theta (A~ order) -> row-softmax weights:
 * A~_uv = exp(theta_uv) / sum_{w in out(u)} exp(theta_uw).
 * theta == NULL restores A~_uv = 1/outdeg(u).
 */
void orc_graph_set_logits(orc_graph *g, const double *theta)
{
    if (!theta) { uniform_weights(g); return; }
    for (int64_t u = 0; u < g->n; ++u) {
        int64_t b = g->a_rowptr[u], e = g->a_rowptr[u + 1];
        double mx = -INFINITY, s = 0.0;
        for (int64_t i = b; i < e; ++i) if (theta[i] > mx) mx = theta[i];
        for (int64_t i = b; i < e; ++i) s += exp(theta[i] - mx);
        for (int64_t i = b; i < e; ++i) g->a_w[i] = exp(theta[i] - mx) / s;
    }
}

/* y = (1-c) A~^T x, pulled row by row over A~^T with in-edges summed in
   ascending source order (Section 2.3, one CPI step). */
static void cpi_step(const orc_graph *g, double c, const double *x, double *y)
{
    for (int64_t v = 0; v < g->n; ++v) {
        double s = 0.0;
        for (int64_t p = g->t_rowptr[v]; p < g->t_rowptr[v + 1]; ++p)
            s += g->a_w[g->t2a[p]] * x[g->t_col[p]];
        y[v] = (1.0 - c) * s;
    }
}

/* y = (1-c) A~ x : the transposed step used by the adjoint. */
static void adj_step(const orc_graph *g, double c, const double *x, double *y)
{
    for (int64_t u = 0; u < g->n; ++u) {
        double s = 0.0;
        for (int64_t e = g->a_rowptr[u]; e < g->a_rowptr[u + 1]; ++e)
            s += g->a_w[e] * x[g->a_col[e]];
        y[u] = (1.0 - c) * s;
    }
}

static double l1(const double *x, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += fabs(x[i]);
    return s;
}

/*
 * Cumulative power iteration (Section 2.3, Algorithm 1).
 *   x(0) = c q ;  x(i) = (1-c) A~^T x(i-1)
 *   r = sum of x(i) for s_iter <= i <= t_iter ; stop after the first i whose
 *   ||x(i)||_1 < eps (checked after accumulating x(i)).
 * t_iter < 0 means "no terminal iteration".  Reading: x(0) is part of the
 * sum when s_iter == 0 (the text states the sum runs over s_iter..t_iter and
 * that s_iter = 0, t_iter = inf gives exact RWR).  Returns the last
 * iteration index computed, or -1 on allocation failure.
 */
int64_t orc_cpi(const orc_graph *g, const double *q, double c, double eps,
                int64_t s_iter, int64_t t_iter, double *r)
{
    int64_t n = g->n;
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    if (!x || !y) { free(x); free(y); return -1; }
    for (int64_t v = 0; v < n; ++v) x[v] = c * q[v];
    for (int64_t v = 0; v < n; ++v) r[v] = (s_iter == 0) ? x[v] : 0.0;
    int64_t last = 0;
    for (int64_t i = 1; t_iter < 0 || i <= t_iter; ++i) {
        cpi_step(g, c, x, y);
        if (i >= s_iter)
            for (int64_t v = 0; v < n; ++v) r[v] += y[v];
        double *t = x; x = y; y = t;
        last = i;
        if (l1(x, n) < eps) break;
    }
    free(x); free(y);
    return last;
}

/*
 * Preprocessing phase (Section 3.1, Algorithm 2): the stranger part of
 * PageRank, CPI with q = (1/n) 1, s_iter = T, t_iter = infinity.
 * Writes r~_stranger; returns the last iteration K (or -1).
 */
int64_t orc_preprocess(const orc_graph *g, double c, int64_t T, double eps, double *str)
{
    int64_t n = g->n;
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    if (!q) return -1;
    for (int64_t v = 0; v < n; ++v) q[v] = 1.0 / (double)n;
    int64_t K = orc_cpi(g, q, c, eps, T, -1, str);
    free(q);
    return K;
}

/*
 * Neighbor-approximation scale (Section 3.2):
 *   ||r_neighbor||_1 / ||r_family||_1 = ((1-c)^S - (1-c)^T) / (1 - (1-c)^S),
 * both norms taken in closed form (Lemma 2).
 */
double orc_neighbor_scale(double c, int64_t S, int64_t T)
{
    double pS = pow(1.0 - c, (double)S), pT = pow(1.0 - c, (double)T);
    return (pS - pT) / (1.0 - pS);
}

/*
 * Online phase (Section 3, Algorithm 3) for a restart vector q:
 *   r_family   = CPI(q, 0, S-1)
 *   r~_neighbor = scale * r_family
 *   r_TPA      = r_family + r~_neighbor + r~_stranger
 * Optional outputs r_family / r_neighbor_approx may be NULL.
 */
int orc_query_q(const orc_graph *g, const double *q, double c, int64_t S, int64_t T,
                double eps, const double *str, double *out, double *fam_out)
{
    int64_t n = g->n;
    double *fam = (double *)malloc(sizeof(double) * (size_t)n);
    if (!fam) return -1;
    if (orc_cpi(g, q, c, eps, 0, S - 1, fam) < 0) { free(fam); return -1; }
    double sc = orc_neighbor_scale(c, S, T);
    for (int64_t v = 0; v < n; ++v) {
        double nb = sc * fam[v];
        out[v] = fam[v] + nb + str[v];
    }
    if (fam_out) memcpy(fam_out, fam, sizeof(double) * (size_t)n);
    free(fam);
    return 0;
}

/* Online phase for a single seed node s (q = e_s). */
int orc_query(const orc_graph *g, int64_t s, double c, int64_t S, int64_t T,
              double eps, const double *str, double *out)
{
    int64_t n = g->n;
    if (s < 0 || s >= n) return -2;
    double *q = (double *)calloc((size_t)n, sizeof(double));
    if (!q) return -1;
    q[s] = 1.0;
    int rc = orc_query_q(g, q, c, S, T, eps, str, out, NULL);
    free(q);
    return rc;
}

/*
 * Reverse-mode derivative of one CPI chain.
 *   forward:  x(0) = x0,  x(i) = (1-c) A~^T x(i-1),  i = 1..N
 *   loss:     L = sum_i beta_i <gv, x(i)>
 * The adjoint lambda(i) = dL/dx(i) obeys
 *   lambda(N) = beta_N gv,  lambda(i) = beta_i gv + (1-c) A~ lambda(i+1),
 * and dL/dA~_uv = (1-c) sum_{i=1..N} x(i-1)[u] lambda(i)[v] is added into
 * G (A~ order).  lambda(0) is written to lam0 when it is not NULL.
 * All N+1 iterates are stored (plain, no checkpointing).
 */
int orc_chain_adjoint(const orc_graph *g, const double *x0, int64_t N, double c,
                      const double *beta, const double *gv, double *G, double *lam0)
{
    int64_t n = g->n;
    double *xs = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(N + 1));
    double *lam = (double *)malloc(sizeof(double) * (size_t)n);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
    if (!xs || !lam || !tmp) { free(xs); free(lam); free(tmp); return -1; }
    memcpy(xs, x0, sizeof(double) * (size_t)n);
    for (int64_t i = 1; i <= N; ++i) cpi_step(g, c, xs + (size_t)(i - 1) * n, xs + (size_t)i * n);

    for (int64_t v = 0; v < n; ++v) lam[v] = beta[N] * gv[v];
    for (int64_t i = N; i >= 1; --i) {
        const double *xp = xs + (size_t)(i - 1) * n;
        for (int64_t u = 0; u < n; ++u)
            for (int64_t e = g->a_rowptr[u]; e < g->a_rowptr[u + 1]; ++e)
                G[e] += (1.0 - c) * xp[u] * lam[g->a_col[e]];
        adj_step(g, c, lam, tmp);
        for (int64_t u = 0; u < n; ++u) lam[u] = beta[i - 1] * gv[u] + tmp[u];
    }
    if (lam0) memcpy(lam0, lam, sizeof(double) * (size_t)n);
    free(xs); free(lam); free(tmp);
    return 0;
}

/*
 * Gradient of L = <gv, r_TPA(q)> for one restart vector q, with the
 * stranger part recomputed from the current weights (K stranger steps).
 *   family chain:   x(0) = c q,        N = S-1, beta_i = 1 + scale
 *   stranger chain: x(0) = (c/n) 1,    N = K,   beta_i = [i >= T]
 * dA (A~ order) accumulates dL/dA~; dq (may be NULL) receives c lambda_fam(0).
 * include_stranger = 0 skips the stranger chain (used when summing several
 * seeds: the stranger's gradient is linear in gv and can be taken once for
 * the summed gv).
 */
int orc_backward_q(const orc_graph *g, const double *q, double c, int64_t S, int64_t T,
                   int64_t K, const double *gv, int include_family, int include_stranger,
                   double *dA, double *dq)
{
    int64_t n = g->n;
    int rc = 0;
    if (include_family) {
        double alpha = 1.0 + orc_neighbor_scale(c, S, T);
        double *x0 = (double *)malloc(sizeof(double) * (size_t)n);
        double *beta = (double *)malloc(sizeof(double) * (size_t)S);
        double *lam0 = (double *)malloc(sizeof(double) * (size_t)n);
        if (!x0 || !beta || !lam0) { free(x0); free(beta); free(lam0); return -1; }
        for (int64_t v = 0; v < n; ++v) x0[v] = c * q[v];
        for (int64_t i = 0; i < S; ++i) beta[i] = alpha;
        rc = orc_chain_adjoint(g, x0, S - 1, c, beta, gv, dA, lam0);
        if (dq) for (int64_t v = 0; v < n; ++v) dq[v] = c * lam0[v];
        free(x0); free(beta); free(lam0);
        if (rc) return rc;
    }
    if (include_stranger) {
        double *x0 = (double *)malloc(sizeof(double) * (size_t)n);
        double *beta = (double *)malloc(sizeof(double) * (size_t)(K + 1));
        if (!x0 || !beta) { free(x0); free(beta); return -1; }
        for (int64_t v = 0; v < n; ++v) x0[v] = c / (double)n;
        for (int64_t i = 0; i <= K; ++i) beta[i] = (i >= T) ? 1.0 : 0.0;
        rc = orc_chain_adjoint(g, x0, K, c, beta, gv, dA, NULL);
        free(x0); free(beta);
    }
    return rc;
}

/* Row-softmax backward: dtheta_uv = A~_uv (dA_uv - sum_w A~_uw dA_uw). */
void orc_softmax_backward(const orc_graph *g, const double *dA, double *dtheta)
{
    for (int64_t u = 0; u < g->n; ++u) {
        int64_t b = g->a_rowptr[u], e = g->a_rowptr[u + 1];
        double s = 0.0;
        for (int64_t i = b; i < e; ++i) s += g->a_w[i] * dA[i];
        for (int64_t i = b; i < e; ++i) dtheta[i] = g->a_w[i] * (dA[i] - s);
    }
}
