"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these compare the oracle with itself: the expected values come from
a dense linear solve (Theorem 1), dense matrix powers built straight from the
edge list, closed-form graphs, the per-iterate norms of Lemma 2, the bound
values printed in Table 3, the bounds of Lemma 1 / Lemma 3 / Theorem 2, the
published SplitMix64 output sequence, and central finite differences.
"""
import os

import numpy as np
import pytest

import oracle
import tpa_inputs as ti

GOLD = os.path.join(os.path.dirname(__file__), "golden")
c, S, T, EPS = ti.C, ti.S, ti.T, ti.EPS


# ---------------------------------------------------------------- helpers
def dense_At_from_edges(n, src, dst, theta_of=None):
    """Dense A~^T written out from the edge list: unique edges, a self-loop on
    each node without out-edges, rows of A~ normalised to sum 1."""
    A = np.zeros((n, n))
    for u, v in set(zip(np.asarray(src).tolist(), np.asarray(dst).tolist())):
        A[u, v] = 1.0
    for u in range(n):
        if A[u].sum() == 0:
            A[u, u] = 1.0
    if theta_of is not None:
        E = np.where(A > 0, np.exp(theta_of), 0.0)
        A = E / E.sum(axis=1, keepdims=True)
    else:
        A = A / A.sum(axis=1, keepdims=True)
    return A.T.copy()


def dense_cpi_window(At, q, s, t):
    """c * sum_{i=s..t} ((1-c) A~^T)^i q by explicit matrix powers."""
    x = c * np.asarray(q, float)
    r = np.zeros_like(x)
    for i in range(0, t + 1):
        if i >= s:
            r += x
        x = (1 - c) * At @ x
    return r


def small_rmat(scale, samples, seed):
    s, d, _ = oracle.rmat(scale, samples, seed)
    return (1 << scale), s, d


def e(n, s):
    q = np.zeros(n)
    q[s] = 1.0
    return q


# ---------------------------------------------------------------- generator
def test_splitmix64_published_sequence():
    rows = [l.split() for l in open(os.path.join(GOLD, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    for j, hx in rows:
        assert oracle.splitmix64(0, int(j)) == int(hx, 16)


def test_rmat_quadrant_orientation_and_rates():
    # asymmetric probabilities so that a swap of u/v bits or of b/c shows
    abcd = (0.1, 0.6, 0.2, 0.1)
    n = 200_000
    s, d, raw = oracle.rmat(1, n, 12345, abcd=abcd)
    assert raw == n and s.size == n
    freq = np.array([np.mean((s == u) & (d == v)) for u, v in ((0, 0), (0, 1), (1, 0), (1, 1))])
    sig = np.sqrt(np.array(abcd) * (1 - np.array(abcd)) / n)
    assert np.all(np.abs(freq - np.array(abcd)) < 6 * sig), freq


def test_rmat_levels_independent():
    # two levels: P(u=0, v=0) = a^2 (both quadrant draws hit "a")
    a = 0.57
    n = 200_000
    s, d, _ = oracle.rmat(2, n, 777)
    p = np.mean((s == 0) & (d == 0))
    assert abs(p - a * a) < 6 * np.sqrt(a * a * (1 - a * a) / n)
    # top bit of u is 0 with probability a + b
    p_top = np.mean(s < 2)
    assert abs(p_top - 0.76) < 6 * np.sqrt(0.76 * 0.24 / n)


def test_rmat_rejection_respects_node_count():
    s, d, raw = oracle.rmat(10, 5000, 99, n_nodes=700)
    assert s.size == 5000 and raw > 5000
    assert s.max() < 700 and d.max() < 700 and s.min() >= 0


# ---------------------------------------------------------------- builder
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_build_matches_brute_force(seed):
    r = np.random.default_rng(seed)
    n = 37
    m_in = 120
    src = r.integers(0, n, m_in).astype(np.int32)
    dst = r.integers(0, n, m_in).astype(np.int32)
    src[:10] = 3  # duplicates
    dst[:10] = 5
    src = np.where(src == 7, 8, src)  # node 7 has no out-edge
    g = oracle.Graph(n, src, dst)
    ex = g.export()
    out = {u: sorted({v for a, v in zip(src.tolist(), dst.tolist()) if a == u}) for u in range(n)}
    padded = [u for u in range(n) if not out[u]]
    for u in padded:
        out[u] = [u]
    assert 7 in padded
    exp_rowptr = np.cumsum([0] + [len(out[u]) for u in range(n)])
    assert np.array_equal(ex["a_rowptr"], exp_rowptr)
    assert np.array_equal(ex["a_col"], np.concatenate([out[u] for u in range(n)]))
    assert np.array_equal(np.flatnonzero(ex["padded"]), padded)
    inn = {v: sorted(u for u in range(n) if v in out[u]) for v in range(n)}
    assert np.array_equal(ex["t_rowptr"], np.cumsum([0] + [len(inn[v]) for v in range(n)]))
    assert np.array_equal(ex["t_col"], np.concatenate([inn[v] for v in range(n) if inn[v]]))
    # t2a points at the same edge
    rows = np.repeat(np.arange(n), np.diff(ex["a_rowptr"]))
    trows = np.repeat(np.arange(n), np.diff(ex["t_rowptr"]))
    assert np.array_equal(rows[ex["t2a"]], ex["t_col"])
    assert np.array_equal(ex["a_col"][ex["t2a"]], trows)
    assert np.allclose(ex["a_w"], 1.0 / np.diff(ex["a_rowptr"])[rows], rtol=0, atol=0)


def test_build_rmat13_invariants():
    g = oracle.Graph.rmat(*ti.GRAPHS["rmat13"])
    ex = g.export()
    n = g.n
    deg = np.diff(ex["a_rowptr"])
    assert deg.min() >= 1
    rows = np.repeat(np.arange(n), deg)
    assert np.allclose(np.bincount(rows, weights=ex["a_w"], minlength=n), 1.0, atol=1e-15)
    # strictly ascending columns within each row (sorted and unique)
    key = rows.astype(np.int64) * n + ex["a_col"]
    assert np.all(np.diff(key) > 0)
    padded = ex["padded"].astype(bool)
    assert np.all(deg[padded] == 1)
    assert np.all(ex["a_col"][ex["a_rowptr"][:-1][padded]] == np.flatnonzero(padded))
    # about 30 % of nodes have no R-MAT out-edge at this size
    assert 0.2 < padded.mean() < 0.4


# ---------------------------------------------------------------- CPI
@pytest.mark.parametrize("scale,samples,n_nodes", [(8, 2000, None), (10, 12000, None), (11, 20000, 1500)])
def test_cpi_equals_dense_solve(scale, samples, n_nodes):
    """Theorem 1: CPI with s_iter=0, t_iter=inf solves r = (1-c) A~^T r + c q."""
    n = (1 << scale) if n_nodes is None else n_nodes
    s, d, _ = oracle.rmat(scale, samples, 4242 + scale, n_nodes=n)
    g = oracle.Graph(n, s, d)
    At = dense_At_from_edges(n, s, d)
    rng = np.random.default_rng(scale)
    for q in (e(n, int(rng.integers(n))), rng.random(n) / n):
        r, last = g.cpi(q, c, 1e-15, 0, -1)
        r_solve = np.linalg.solve(np.eye(n) - (1 - c) * At, c * q)
        assert np.abs(r - r_solve).sum() < 1e-12 * max(1.0, q.sum())
        assert last > 100


@pytest.mark.parametrize("s_iter,t_iter", [(0, 0), (0, 4), (1, 4), (3, 3), (2, 9), (5, 4)])
def test_cpi_window_matches_matrix_powers(s_iter, t_iter):
    n, s, d = small_rmat(7, 700, 31)
    g = oracle.Graph(n, s, d)
    At = dense_At_from_edges(n, s, d)
    q = e(n, 17)
    r, _ = g.cpi(q, c, 0.0, s_iter, t_iter)
    assert np.abs(r - dense_cpi_window(At, q, s_iter, t_iter)).sum() < 1e-14


def test_lemma2_iterate_norms():
    """Lemma 2: ||x(i)||_1 = c (1-c)^i, so ||r_family||_1 = 1 - (1-c)^S."""
    g = oracle.Graph.rmat(*ti.GRAPHS["rmat13"])
    q = e(g.n, 123)
    for i in range(0, 25):
        xi, _ = g.cpi(q, c, 0.0, i, i)
        assert abs(np.abs(xi).sum() - c * (1 - c) ** i) < 1e-14
        assert xi.min() >= 0
    fam, _ = g.cpi(q, c, 0.0, 0, S - 1)
    assert abs(fam.sum() - (1 - (1 - c) ** S)) < 1e-14


# ---------------------------------------------------------------- preprocess
def test_preprocess_K_from_l1_break():
    """Algorithm 1's L1 break at eps=1e-9: c(1-c)^115 > 1e-9 > c(1-c)^116."""
    g = oracle.Graph.rmat(*ti.GRAPHS["rmat13"])
    g.preprocess(c, T, EPS)
    assert g.K == 116
    assert c * (1 - c) ** 115 > EPS > c * (1 - c) ** 116


def test_stranger_equals_pagerank_tail():
    """r~_stranger = PageRank minus its first T terms (Section 3.1)."""
    n, s, d = small_rmat(10, 12000, 5)
    g = oracle.Graph(n, s, d)
    At = dense_At_from_edges(n, s, d)
    st = g.preprocess(c, T, EPS)
    b = np.full(n, 1.0 / n)
    p = np.linalg.solve(np.eye(n) - (1 - c) * At, c * b)
    head = dense_cpi_window(At, b, 0, T - 1)
    trunc = (1 - c) ** (g.K + 1)
    assert np.abs(st - (p - head)).sum() <= trunc + 1e-12
    assert abs(st.sum() - ((1 - c) ** T - (1 - c) ** (g.K + 1))) < 1e-13


# ---------------------------------------------------------------- online
def test_neighbor_scale_reproduces_table3():
    """Table 3 prints 2||r_neighbor||_1 = 2(1-c)^S - 2(1-c)^T; scale *
    ||r_family||_1 must equal half of it (Section 3.2, Lemma 2)."""
    rows = [l.split() for l in open(os.path.join(GOLD, "table3_bounds.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 7
    for name, Ss, Ts, nb, stb, tpab in rows:
        Ss, Ts = int(Ss), int(Ts)
        fam_norm = 1 - (1 - c) ** Ss
        assert round(2 * oracle.neighbor_scale(c, Ss, Ts) * fam_norm, 4) == pytest.approx(float(nb), abs=1e-12), name
        assert round(2 * (1 - c) ** Ts, 4) == pytest.approx(float(stb), abs=1e-12), name
        assert round(2 * (1 - c) ** Ss, 4) == pytest.approx(float(tpab), abs=1e-12), name


def test_neighbor_scale_at_defaults():
    # T = 2S makes the ratio (1-c)^S exactly
    assert oracle.neighbor_scale(0.15, 5, 10) == pytest.approx(0.85 ** 5, rel=1e-14)
    assert oracle.neighbor_scale(0.15, 5, 5) == 0.0


def test_query_matches_dense_brute_force():
    n, s, d = small_rmat(9, 5000, 77)
    g = oracle.Graph(n, s, d)
    At = dense_At_from_edges(n, s, d)
    st = g.preprocess(c, T, EPS)
    b = np.full(n, 1.0 / n)
    st_dense = dense_cpi_window(At, b, T, g.K)
    assert np.abs(st - st_dense).sum() < 1e-13
    alpha = (1 - (1 - c) ** T) / (1 - (1 - c) ** S)
    for seed in (0, 3, 200, 511):
        fam = dense_cpi_window(At, e(n, seed), 0, S - 1)
        expect = alpha * fam + st_dense
        assert np.abs(g.query(seed, c, S, T) - expect).sum() < 1e-13


def test_closed_form_cycle():
    n = 50
    src = np.arange(n, dtype=np.int32)
    dst = ((np.arange(n) + 1) % n).astype(np.int32)
    g = oracle.Graph(n, src, dst)
    st = g.preprocess(c, T, EPS)
    K = g.K
    assert np.allclose(st, ((1 - c) ** T - (1 - c) ** (K + 1)) / n, rtol=1e-13, atol=0)
    s0 = 45
    _, fam = g.query_q(e(n, s0), c, S, T, return_family=True)
    expect = np.zeros(n)
    for j in range(S):
        expect[(s0 + j) % n] = c * (1 - c) ** j
    assert np.abs(fam - expect).sum() < 1e-15
    r = g.query(s0, c, S, T)
    alpha = (1 - (1 - c) ** T) / (1 - (1 - c) ** S)
    assert np.abs(r - (alpha * expect + st)).sum() < 1e-14


def test_closed_form_complete_digraph():
    n = 12
    u, v = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    g = oracle.Graph(n, u.ravel().astype(np.int32), v.ravel().astype(np.int32))
    st = g.preprocess(c, T, EPS)
    K = g.K
    assert np.allclose(st, ((1 - c) ** T - (1 - c) ** (K + 1)) / n, rtol=1e-13, atol=0)
    _, fam = g.query_q(e(n, 4), c, S, T, return_family=True)
    expect = c * e(n, 4) + ((1 - c) - (1 - c) ** S) / n
    assert np.abs(fam - expect).sum() < 1e-15


def test_closed_form_single_node():
    g = oracle.Graph(1, np.zeros(0, np.int32), np.zeros(0, np.int32))
    g.preprocess(c, T, EPS)
    r = g.query(0, c, S, T)
    assert r[0] == pytest.approx(1 - (1 - c) ** (g.K + 1), abs=1e-15)


def test_mass_invariant_and_nonnegativity():
    g = oracle.Graph.rmat(*ti.GRAPHS["rmat13"])
    g.preprocess(c, T, EPS)
    for seed in (0, 1, 100, 4000, 8191):
        r = g.query(seed, c, S, T)
        assert r.min() >= 0
        assert abs(r.sum() - (1 - (1 - c) ** (g.K + 1))) < 1e-13


def test_error_bounds_against_exact_cpi():
    """Lemma 1, Lemma 3 and Theorem 2 against exact CPI parts."""
    n, s, d = small_rmat(10, 12000, 8)
    g = oracle.Graph(n, s, d)
    st = g.preprocess(c, T, EPS)
    for seed in (1, 10, 700):
        q = e(n, seed)
        fam, _ = g.cpi(q, c, 0.0, 0, S - 1)
        nb_exact, _ = g.cpi(q, c, 0.0, S, T - 1)
        st_exact, _ = g.cpi(q, c, 1e-16, T, -1)
        nb_approx = oracle.neighbor_scale(c, S, T) * fam
        assert np.abs(st_exact - st).sum() <= 2 * (1 - c) ** T
        assert np.abs(nb_exact - nb_approx).sum() <= 2 * (1 - c) ** S - 2 * (1 - c) ** T
        exact, _ = g.cpi(q, c, 1e-16, 0, -1)
        assert np.abs(exact - g.query(seed, c, S, T)).sum() <= 2 * (1 - c) ** S


# ---------------------------------------------------------------- logit weights
def test_softmax_weights_query_and_cpi_match_dense():
    """Row-softmax weights from per-edge logits (the weighted A~ of the
    adjoint's forward pass): the oracle's weights equal the dense softmax
    written out from the edge list, its weighted TPA equals dense brute force
    (family by matrix powers, stranger as dense PageRank minus its first T
    terms), and weighted CPI to eps solves the RWR system (Theorem 1)."""
    n, s, d = small_rmat(8, 1500, 606)
    g = oracle.Graph(n, s, d)
    ex = g.export()
    rows = np.repeat(np.arange(n), np.diff(ex["a_rowptr"]))
    theta = 0.5 * np.random.default_rng(607).standard_normal(g.m)
    theta_mat = np.zeros((n, n))
    theta_mat[rows, ex["a_col"]] = theta
    At = dense_At_from_edges(n, s, d, theta_of=theta_mat)
    g.set_logits(theta)
    w = g.export()["a_w"]
    # weights: A~_uv = exp(theta_uv) / sum_w exp(theta_uw), read off the dense matrix
    assert np.abs(w - At.T[rows, ex["a_col"]]).max() < 1e-15
    assert np.abs(w - 1.0 / np.diff(ex["a_rowptr"])[rows]).max() > 1e-3  # not the uniform weights
    st = g.preprocess(c, T, EPS)
    b = np.full(n, 1.0 / n)
    p = np.linalg.solve(np.eye(n) - (1 - c) * At, c * b)
    assert np.abs(st - (p - dense_cpi_window(At, b, 0, T - 1))).sum() <= (1 - c) ** (g.K + 1) + 1e-12
    alpha = (1 - (1 - c) ** T) / (1 - (1 - c) ** S)
    st_dense = dense_cpi_window(At, b, T, g.K)
    for seed in (0, 7, 100, 255):
        expect = alpha * dense_cpi_window(At, e(n, seed), 0, S - 1) + st_dense
        assert np.abs(g.query(seed, c, S, T) - expect).sum() < 1e-13
        r, _ = g.cpi(e(n, seed), c, 1e-15, 0, -1)
        r_solve = np.linalg.solve(np.eye(n) - (1 - c) * At, c * e(n, seed))
        assert np.abs(r - r_solve).sum() < 1e-12
    g.set_logits(None)
    assert np.array_equal(g.export()["a_w"], ex["a_w"])


# ---------------------------------------------------------------- adjoint
def test_adjoint_matches_central_differences():
    """Oracle gradient of L = sum_j <w_j, r_TPA(q_j)> w.r.t. edge logits and
    restart vectors against central differences (h = 1e-3, FP64)."""
    n, s, d = small_rmat(6, 300, 11)
    g = oracle.Graph(n, s, d)
    m = g.m
    theta = 0.1 * np.random.default_rng(0).standard_normal(m)
    g.set_logits(theta)
    rng = np.random.default_rng(1)
    Q = np.stack([e(n, 3), e(n, 40), rng.random(n) / n])
    W = rng.standard_normal((3, n))

    def loss(th, Qm):
        g.set_logits(th)
        R, _ = g.tpa_forward(Qm, c, S, T, EPS)
        return float((W * R).sum())

    g.set_logits(theta)
    _, K = g.tpa_forward(Q, c, S, T, EPS)
    dtheta, _, dq = g.backward(Q, W, c, S, T, K)
    h = 1e-3
    # sampled edges
    for idx in rng.choice(m, 12, replace=False):
        tp = theta.copy(); tp[idx] += h
        tm = theta.copy(); tm[idx] -= h
        fd = (loss(tp, Q) - loss(tm, Q)) / (2 * h)
        assert abs(fd - dtheta[idx]) <= 1e-6 * np.abs(dtheta).max() + 1e-9, idx
    # random direction
    dirn = rng.standard_normal(m)
    fd = (loss(theta + h * dirn, Q) - loss(theta - h * dirn, Q)) / (2 * h)
    assert abs(fd - dtheta @ dirn) <= 1e-6 * np.abs(dtheta @ dirn) + 1e-9
    # restart vector (L is linear in q)
    g.set_logits(theta)
    for j, v in ((0, 3), (1, 7), (2, 50)):
        Qp = Q.copy(); Qp[j, v] += h
        Qm_ = Q.copy(); Qm_[j, v] -= h
        fd = (loss(theta, Qp) - loss(theta, Qm_)) / (2 * h)
        assert abs(fd - dq[j, v]) <= 1e-9 * max(1.0, abs(dq[j, v]))


def test_topk_defining_properties():
    """oracle.topk against the properties that fix a top-k list uniquely:
    k entries; values non-increasing with NaN last; every unselected entry
    no larger than the smallest selected one; among entries equal to the
    cut value, the smallest indices are taken; equal values in index order."""
    rng = np.random.default_rng(44)
    for n, k in ((1, 1), (9, 4), (300, 7), (300, 300), (2000, 64)):
        pool = np.array([0.5, 0.25, 0.0, -0.0, 1e-7, np.nan, 3.0], np.float32)
        vals = np.where(rng.random((4, n)) < 0.6, rng.choice(pool, (4, n)),
                        rng.random((4, n)).astype(np.float32))
        idx, val = oracle.topk(vals, k)
        for r in range(4):
            row, sel = vals[r], idx[r]
            assert len(set(sel.tolist())) == k
            assert np.array_equal(val[r], row[sel], equal_nan=True)
            key = np.where(np.isnan(row), -np.inf, row.astype(np.float64))
            ks = key[sel]
            assert np.all(ks[1:] <= ks[:-1])
            rest = np.setdiff1d(np.arange(n), sel)
            if len(rest):
                assert key[rest].max() <= ks.min()
            cut = ks[-1]
            tied = np.flatnonzero(key == cut)
            chosen = np.sort(sel[ks == cut])
            assert np.array_equal(chosen, tied[:len(chosen)])
            for v in np.unique(ks):
                pos = sel[ks == v]
                assert np.all(np.diff(pos) > 0)


# ---------------------------------------------------------------- structured closed form
def test_structured_closed_form_helper_matches_oracle():
    """The O(n) closed-form helper that checks the GPU path on a graph with
    more than 2^31 edges (tests/closed_form.py: complete digraph block,
    two-successor circulant, isolated nodes), pinned on a small instance of
    the same structure against the oracle: CSR offsets, stranger, TPA for
    seeds in each part and a dense restart, restart and logit gradients."""
    from closed_form import Structured
    cf = Structured(nc=12, L=9, D=3)
    src, dst = cf.edge_list(order_seed=5)
    g = oracle.Graph(cf.n, src.astype(np.int32), dst.astype(np.int32))
    assert (g.n, g.m) == (cf.n, cf.m)
    ex = g.export()
    assert np.array_equal(ex["a_rowptr"], cf.a_rowptr())
    rows = np.repeat(np.arange(cf.n), np.diff(ex["a_rowptr"]))
    sel = rows < cf.i0
    assert np.array_equal(cf.edge_index(rows[sel], ex["a_col"][sel]), np.flatnonzero(sel))
    st = g.preprocess(c, T, EPS)
    assert np.abs(st - cf.stranger(c, T, g.K)).sum() < 1e-15
    rng = np.random.default_rng(6)
    qd = rng.random(cf.n)
    qd /= qd.sum()
    Q = np.stack([e(cf.n, 3), e(cf.n, cf.c0 + 7), e(cf.n, cf.i0 + 1), qd])
    for q in Q:
        assert np.abs(g.query_q(q, c, S, T) - cf.tpa(q, c, S, T, g.K)).sum() < 1e-14
    W = rng.standard_normal((4, cf.n))
    dth, _, dq = g.backward(Q, W, c, S, T, g.K)
    dQ, dtheta = cf.backward(Q, W, c, S, T, g.K)
    assert np.abs(dq - dQ).max() < 1e-13 * np.abs(dQ).max()
    assert np.abs(dth[sel] - dtheta(rows[sel], ex["a_col"][sel])).max() < 1e-12 * np.abs(dth).max()
    assert np.all(dth[~sel] == 0.0)
