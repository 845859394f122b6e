"""Exact values on a graph with more than 2^31 edges (int64 edge offsets).

The graph (tests/closed_form.py) is a complete digraph with self-loops on
46,341 nodes (46,341^2 = 2,147,488,281 edges), then a two-successor
circulant on 5,000 nodes and 37 isolated nodes (self-loops added by the
builder).  The circulant and isolated rows sit past edge offset 2^31 in both
orientations.  Every expected value is a closed form or an O(n) recursion of
the structure (block mean, shifts, identity), pinned on a small instance of
the same structure against the oracle in test_oracle.py: CSR arrays exactly,
and TPA (stranger, single seeds through the pulled and the pushed second
step, seed tiles of 16 and 64, dense restarts) and gradients (restart
vectors and sampled edge logits) within the parity bar.
"""
import numpy as np
import pytest

import tpa_inputs as ti
from closed_form import Structured

pytestmark = pytest.mark.gpu

c, S, T = ti.C, ti.S, ti.T
TOL = 1e-5
NC, L, D = 46341, 5000, 37


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a HIP device"
    return _t


@pytest.fixture(scope="module")
def tpa(torch):
    import paper_1708_02574_amd as _tpa
    _tpa.load_library()
    return _tpa


def say(msg):
    print(f"large closed form: {msg}", flush=True)


@pytest.fixture(scope="module")
def big(tpa, torch):
    cf = Structured(NC, L, D)
    assert cf.m > 2 ** 31
    say(f"edge list n={cf.n} m={cf.m} on the device")
    mb = NC * NC
    cs, cd = cf.circ_succ()
    src = torch.empty(mb + cs.size, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    # circulant edges first, block edges after them (the builder sorts)
    src[:cs.size] = torch.from_numpy(cs.astype(np.int32)).cuda()
    dst[:cs.size] = torch.from_numpy(cd.astype(np.int32)).cuda()
    step = 1 << 28
    for e0 in range(0, mb, step):
        e = torch.arange(e0, min(mb, e0 + step), dtype=torch.int64, device="cuda")
        src[cs.size + e0:cs.size + e0 + e.numel()] = (e // NC).to(torch.int32)
        dst[cs.size + e0:cs.size + e0 + e.numel()] = (e % NC).to(torch.int32)
        del e
    say("tpa_graph_from_edges (device pointers)")
    g = tpa.Graph.from_edges(cf.n, src, dst)
    del src, dst
    torch.cuda.empty_cache()
    say(f"built: n={g.n} m={g.m}; preprocess")
    g.preprocess(c, T)
    yield cf, g
    g.close()
    torch.cuda.empty_cache()


def l1(a, b):
    return float(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)).sum())


def nl1(a, b):
    b = np.asarray(b, np.float64)
    return float(np.abs(np.asarray(a, np.float64) - b).sum() / max(np.abs(b).sum(), 1e-300))


def test_csr_arrays_exact(big, torch):
    """Both orientations' offsets, columns and FP32 weights equal the
    structure's, including every entry past offset 2^31."""
    cf, g = big
    assert (g.n, g.m) == (cf.n, cf.m)
    mb = NC * NC
    rp_expect = torch.from_numpy(cf.a_rowptr()).cuda()
    for transpose in (False, True):
        say(f"export transpose={transpose}")
        rp, col, w = g.export(transpose=transpose)
        # in-degrees equal out-degrees part by part, so A~^T has A~'s offsets
        assert torch.equal(rp, rp_expect)
        ar = torch.arange(NC, dtype=torch.int32, device="cuda")
        assert torch.equal(col[:mb].view(NC, NC), ar.expand(NC, NC))
        if transpose:
            i = np.arange(L)
            a, b = (i - 1) % L, (i - 2) % L
            circ = np.stack([np.minimum(a, b), np.maximum(a, b)], axis=1) + cf.c0
        else:
            circ = cf.circ_rows_cols()
        assert torch.equal(col[mb:mb + 2 * L].cpu(), torch.from_numpy(circ.reshape(-1).astype(np.int32)))
        assert torch.equal(col[mb + 2 * L:].cpu(), torch.arange(cf.i0, cf.n, dtype=torch.int32))
        inv = float(np.float32(1.0) / np.float32(NC))
        assert bool((w[:mb] == inv).all())
        assert bool((w[mb:mb + 2 * L] == 0.5).all()) and bool((w[mb + 2 * L:] == 1.0).all())
        del rp, col, w
        torch.cuda.empty_cache()


def test_stranger_and_queries(big, tpa, torch):
    cf, g = big
    K = 116
    st = g.stranger().cpu().numpy()
    assert l1(st, cf.stranger(c, T, K)) <= TOL
    # single seeds: block seeds (frontier = the block: step 2 pulled), a
    # circulant seed that wraps and an isolated seed (step 2 pushed)
    singles = [123, NC - 1, cf.c0 + L - 2, cf.c0 + 17, cf.i0 + D - 1]
    for s in singles:
        say(f"single-seed query {s}")
        r = g.query(torch.tensor([s], dtype=torch.int32), c, S, T)[0].cpu().numpy()
        q = np.zeros(cf.n)
        q[s] = 1.0
        assert l1(r, cf.tpa(q, c, S, T, K)) <= TOL, s
    rng = np.random.default_rng(71)
    for kt, k in ((16, 16), (64, 40)):
        seeds = np.concatenate([rng.integers(0, NC, k // 2), cf.c0 + rng.integers(0, L, k // 2 - 2),
                                cf.i0 + rng.integers(0, D, 2)]).astype(np.int32)
        say(f"seed tile {kt}, {k} seeds")
        g.set_tuning(seed_tile=kt)
        try:
            R = g.query(torch.from_numpy(seeds), c, S, T).cpu().numpy()
        finally:
            g.set_tuning(0, 0)
        for j, s in enumerate(seeds):
            q = np.zeros(cf.n)
            q[s] = 1.0
            assert l1(R[j], cf.tpa(q, c, S, T, K)) <= TOL, (kt, j, s)
    say("dense restarts")
    Q = rng.random((3, cf.n))
    Q[1, :NC] = 0.0  # mass only past the block
    Q /= Q.sum(axis=1, keepdims=True)
    R = g.query_dense(torch.from_numpy(Q.astype(np.float32)), c, S, T).cpu().numpy()
    for j in range(3):
        assert l1(R[j], cf.tpa(Q[j].astype(np.float32).astype(np.float64), c, S, T, K)) <= TOL, j


@pytest.mark.parametrize("form", ["seed", "seeds4", "dense2"])
def test_gradients(big, tpa, torch, form):
    """Restart gradients on every node and logit gradients on 4000 sampled
    block edges, every circulant edge and every isolated self-loop."""
    cf, g = big
    K = 116
    rng = np.random.default_rng({"seed": 81, "seeds4": 82, "dense2": 83}[form])
    if form == "dense2":
        Q = rng.random((2, cf.n))
        Q /= Q.sum(axis=1, keepdims=True)
        Q = Q.astype(np.float32).astype(np.float64)
        seeds = None
    else:
        if form == "seed":
            seeds = np.array([cf.c0 + rng.integers(0, L)], np.int32)
        else:
            seeds = np.array([rng.integers(0, NC), cf.c0 + rng.integers(0, L), cf.c0 + L - 1,
                              cf.i0 + rng.integers(0, D)], np.int32)
        k = seeds.size
        Q = np.zeros((k, cf.n))
        Q[np.arange(k), seeds] = 1.0
    W = ti.draw_loss_weights(Q.shape, 84)
    say(f"backward ({form})")
    Wd = torch.from_numpy(W).cuda()
    if seeds is not None:
        dth, dq = g.backward(Wd, c, S, T, seeds=torch.from_numpy(seeds).cuda())
    else:
        dth, dq = g.backward(Wd, c, S, T, q=torch.from_numpy(Q.astype(np.float32)).cuda())
    dQ, dtheta = cf.backward(Q, W.astype(np.float64), c, S, T, K)
    assert nl1(dq.cpu().numpy(), dQ) <= TOL
    bu = rng.integers(0, NC, 4000)
    bv = rng.integers(0, NC, 4000)
    cu = np.repeat(np.arange(cf.c0, cf.i0), 2)
    cv = cf.circ_rows_cols().reshape(-1)
    u = np.concatenate([bu, cu])
    v = np.concatenate([bv, cv])
    idx = torch.from_numpy(cf.edge_index(u, v)).cuda()
    got = dth[idx].cpu().numpy()
    assert nl1(got, dtheta(u, v)) <= TOL
    assert nl1(got[:4000], dtheta(bu, bv)) <= TOL  # the block alone
    iso = dth[NC * NC + 2 * L:].cpu().numpy()
    assert np.all(iso == 0.0)
    del dth, dq
    torch.cuda.empty_cache()
