"""HIP path vs the FP64 oracle, through the C ABI.

Integer graph construction must be bit-exact; r_TPA must agree within
L1 <= 1e-5 per seed (FP32 values and accumulation on the device).
"""
import numpy as np
import pytest

import oracle
import tpa_inputs as ti

pytestmark = pytest.mark.gpu

c, S, T, EPS = ti.C, ti.S, ti.T, ti.EPS
TOL = 1e-5


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


@pytest.fixture(scope="module")
def rmat13(tpa):
    scale, samples, seed = ti.GRAPHS["rmat13"]
    og = oracle.Graph.rmat(scale, samples, seed)
    og.preprocess(c, T, EPS)
    gg = tpa.Graph.rmat(scale, samples, seed)
    gg.preprocess(c, T)
    return og, gg


def l1_rows(a, b):
    return np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)).sum(axis=-1)


def compare_graph(og, gg, torch):
    ex = og.export()
    rp, col, w = gg.export(transpose=False)
    trp, tcol, tw = gg.export(transpose=True)
    torch.cuda.synchronize()
    assert gg.n == og.n and gg.m == og.m
    assert np.array_equal(rp.cpu().numpy(), ex["a_rowptr"])
    assert np.array_equal(col.cpu().numpy(), ex["a_col"])
    assert np.array_equal(trp.cpu().numpy(), ex["t_rowptr"])
    assert np.array_equal(tcol.cpu().numpy(), ex["t_col"])
    assert np.array_equal(gg.padded().cpu().numpy(), ex["padded"])
    deg = np.diff(ex["a_rowptr"]).astype(np.float32)
    w_expect = (np.float32(1.0) / deg)[np.repeat(np.arange(og.n), np.diff(ex["a_rowptr"]))]
    assert np.array_equal(w.cpu().numpy(), w_expect)  # IEEE FP32 division, bit for bit
    assert np.array_equal(tw.cpu().numpy(), w_expect[ex["t2a"]])


# ---------------------------------------------------------------- graph store
def test_rmat13_graph_bit_exact(rmat13, torch):
    og, gg = rmat13
    compare_graph(og, gg, torch)


def test_rmat_rejection_graph_bit_exact(tpa, torch):
    og = oracle.Graph.rmat(12, 48000, 0xABC, n_nodes=3000)
    gg = tpa.Graph.rmat(12, 48000, 0xABC, n_nodes=3000)
    compare_graph(og, gg, torch)


@pytest.mark.parametrize("device_edges", [False, True])
def test_from_edges_bit_exact(tpa, torch, device_edges):
    r = np.random.default_rng(5)
    n, m = 1000, 6000
    src = r.integers(0, n, m).astype(np.int32)
    dst = r.integers(0, n, m).astype(np.int32)
    src[:500] = src[500:1000]          # duplicates
    dst[:500] = dst[500:1000]
    src[src % 7 == 3] = 0              # many nodes without out-edges
    og = oracle.Graph(n, src, dst)
    if device_edges:
        gg = tpa.Graph.from_edges(n, torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda())
    else:
        gg = tpa.Graph.from_edges(n, src, dst)
    compare_graph(og, gg, torch)


def test_from_edges_rejects_bad_ids(tpa):
    with pytest.raises(tpa.TPAError) as e:
        tpa.Graph.from_edges(10, np.array([1, 2], np.int32), np.array([3, 10], np.int32))
    assert e.value.status == -1


# ---------------------------------------------------------------- preprocess
def test_stranger_parity(rmat13, torch):
    og, gg = rmat13
    st = gg.stranger().cpu().numpy()
    assert l1_rows(st, og.str) <= TOL
    assert st.min() >= 0


@pytest.mark.parametrize("Tq", [0, 1, 10, 30])
def test_stranger_parity_various_T(tpa, torch, Tq):
    og = oracle.Graph.rmat(10, 12000, 3)
    ost = og.preprocess(c, Tq, EPS)
    gg = tpa.Graph.rmat(10, 12000, 3)
    gg.preprocess(c, Tq)
    assert l1_rows(gg.stranger().cpu().numpy(), ost) <= TOL


# ---------------------------------------------------------------- queries
def seeds_for(og, k, seed):
    return ti.draw_seeds(og.export()["padded"] == 0, k, seed)


def test_single_seed_queries(rmat13, torch):
    og, gg = rmat13
    seeds = seeds_for(og, 12, 101)
    for s in seeds:
        r = gg.query(torch.tensor([s]), c, S, T).cpu().numpy()[0]
        assert l1_rows(r, og.query(int(s), c, S, T)) <= TOL


@pytest.mark.parametrize("k,kt", [(1, 1), (3, 2), (17, 4), (64, 8), (100, 16), (70, 32), (130, 64), (5, 0)])
def test_batched_queries(rmat13, torch, k, kt):
    og, gg = rmat13
    seeds = seeds_for(og, k, 7 + k)
    gg.set_tuning(seed_tile=kt)
    try:
        R = gg.query(torch.from_numpy(seeds), c, S, T).cpu().numpy()
    finally:
        gg.set_tuning(0, 0)
    expect = np.stack([og.query(int(s), c, S, T) for s in seeds])
    assert np.all(l1_rows(R, expect) <= TOL)


@pytest.mark.parametrize("ew", [64, 128, 512, 1024])
@pytest.mark.parametrize("kt", [1, 4, 16, 64])
def test_schedules_with_long_rows(rmat13, torch, ew, kt):
    """Small edges-per-item makes the hub rows of A~^T long (chunks + finish)."""
    og, gg = rmat13
    seeds = seeds_for(og, 9, 55)
    gg.set_tuning(seed_tile=kt, edges_per_item=ew)
    try:
        R = gg.query(torch.from_numpy(seeds), c, S, T).cpu().numpy()
    finally:
        gg.set_tuning(0, 0)
    expect = np.stack([og.query(int(s), c, S, T) for s in seeds])
    assert np.all(l1_rows(R, expect) <= TOL)


@pytest.mark.parametrize("ew,kt", [(64, 1), (512, 1), (64, 4), (128, 64), (1024, 64), (1024, 1)])
def test_hub_rows_blocks_and_chunks(tpa, torch, ew, kt):
    """A graph whose hub has 20000 in-edges: with small items it becomes a
    chunked row (finish pass); with the default single-vector shape it is a
    block item shared by 4 waves."""
    n = 30000
    r = np.random.default_rng(9)
    src = np.concatenate([np.arange(1, 20001), r.integers(0, n, 150000)]).astype(np.int32)
    dst = np.concatenate([np.zeros(20000, np.int64), r.integers(0, n, 150000)]).astype(np.int32)
    dst[20000:20000 + 3000] = 7          # a second, mid-size hub
    og = oracle.Graph(n, src, dst)
    og.preprocess(c, T, EPS)
    gg = tpa.Graph.from_edges(n, src, dst)
    gg.set_tuning(seed_tile=kt, edges_per_item=ew)
    gg.preprocess(c, T)
    assert l1_rows(gg.stranger().cpu().numpy(), og.str) <= TOL
    seeds = np.array([5, 17, 20000, 29999, 7, 0], np.int32)
    R = gg.query(torch.from_numpy(seeds), c, S, T).cpu().numpy()
    expect = np.stack([og.query(int(s), c, S, T) for s in seeds])
    assert np.all(l1_rows(R, expect) <= TOL)


@pytest.mark.parametrize("Sq,Tq", [(1, 10), (2, 10), (5, 5), (3, 7), (8, 10)])
def test_query_S_T_cases(tpa, torch, Sq, Tq):
    og = oracle.Graph.rmat(11, 30000, 17)
    og.preprocess(c, Tq, EPS)
    gg = tpa.Graph.rmat(11, 30000, 17)
    gg.preprocess(c, Tq)
    seeds = seeds_for(og, 6, 3)
    R = gg.query(torch.from_numpy(seeds), c, Sq, Tq).cpu().numpy()
    expect = np.stack([og.query(int(s), c, Sq, Tq) for s in seeds])
    assert np.all(l1_rows(R, expect) <= TOL)


def test_dangling_seed_and_hub_seed(rmat13, torch):
    og, gg = rmat13
    ex = og.export()
    dangling = int(np.flatnonzero(ex["padded"])[0])
    hub = int(np.argmax(np.diff(ex["a_rowptr"])))
    for s in (dangling, hub, 0, og.n - 1):
        r = gg.query(torch.tensor([s]), c, S, T).cpu().numpy()[0]
        assert l1_rows(r, og.query(s, c, S, T)) <= TOL


def test_mass_and_determinism(rmat13, torch):
    og, gg = rmat13
    seeds = torch.from_numpy(seeds_for(og, 40, 9))
    a = gg.query(seeds, c, S, T)
    b = gg.query(seeds, c, S, T)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    mass = a.double().sum(dim=1).cpu().numpy()
    assert np.all(np.abs(mass - (1 - (1 - c) ** 117)) < 1e-5)


def test_cycle_closed_form_on_gpu(tpa, torch):
    n = 200
    src = np.arange(n, dtype=np.int32)
    dst = ((np.arange(n) + 1) % n).astype(np.int32)
    gg = tpa.Graph.from_edges(n, src, dst)
    gg.preprocess(c, T)
    K = 116
    st = gg.stranger().cpu().numpy()
    assert np.allclose(st, ((1 - c) ** T - (1 - c) ** (K + 1)) / n, rtol=1e-5, atol=0)
    r = gg.query(torch.tensor([190]), c, S, T).cpu().numpy()[0]
    alpha = (1 - (1 - c) ** T) / (1 - (1 - c) ** S)
    expect = st.astype(np.float64).copy()
    for j in range(S):
        expect[(190 + j) % n] += alpha * c * (1 - c) ** j
    assert l1_rows(r, expect) <= TOL


# ---------------------------------------------------------------- pushed step 2
def frontier_edges(ex, s):
    """Edges of A~ leaving F = out(s) + {s}: the work of a pushed step 2."""
    rp, col = ex["a_rowptr"], ex["a_col"]
    nb = col[rp[s]:rp[s + 1]]
    f = nb if s in nb else np.append(nb, s)
    return int(np.diff(rp)[f].sum())


def run_single(gg, torch, sd, Sq, order):
    out = [None] * len(order)
    for i in order:
        out[i] = gg.query(sd[i:i + 1], c, Sq, T)[0]
    return torch.stack(out)


@pytest.mark.parametrize("Sq", [4, 5, 8])
def test_second_step_push_and_pull(rmat13, torch, Sq):
    """Single-seed queries with step 2 always pushed (limit m), always pulled
    (limit 0) and chosen per seed (limit = the median frontier): all within
    L1 of the oracle, push and pull within FP32 rounding of each other,
    bitwise reproducible in any query order, and the per-seed choice equal
    bit for bit to the forced direction it picked."""
    og, gg = rmat13
    ex = og.export()
    seeds = [int(s) for s in seeds_for(og, 10, 303)]
    seeds += [int(np.argmax(np.diff(ex["a_rowptr"]))), int(np.flatnonzero(ex["padded"])[0])]
    W = np.array([frontier_edges(ex, s) for s in seeds])
    mid = int(np.median(W))
    assert (W <= mid).any() and (W > mid).any()
    expect = np.stack([og.query(s, c, Sq, T) for s in seeds])
    sd = torch.tensor(seeds, dtype=torch.int32).cuda()
    runs = {}
    try:
        for limit in (0, og.m, mid, -1):
            gg.set_push_limit(limit)
            assert gg.get_push_limit() == limit
            R = run_single(gg, torch, sd, Sq, list(range(len(seeds))))
            R2 = run_single(gg, torch, sd, Sq, list(reversed(range(len(seeds)))))
            assert torch.equal(R, R2), limit
            runs[limit] = R.cpu().numpy()
            assert np.all(l1_rows(runs[limit], expect) <= TOL), limit
    finally:
        gg.set_push_limit(-1)
    pushed, pulled, mixed = runs[og.m], runs[0], runs[mid]
    assert np.abs(pushed - pulled).max() <= 1e-6
    for i, w in enumerate(W):
        assert np.array_equal(mixed[i], (pushed if w <= mid else pulled)[i]), i


def test_second_step_push_weighted(tpa, torch):
    """Row-softmax edge weights: the pushed step multiplies each gathered
    value by its A~ edge weight."""
    og = oracle.Graph.rmat(10, 12000, 22)
    gg = tpa.Graph.rmat(10, 12000, 22)
    theta = ti.draw_logits(og.m, 7)
    og.set_logits(theta.astype(np.float64))
    gg.set_logits(torch.from_numpy(theta).cuda())
    og.preprocess(c, T, EPS)
    gg.preprocess(c, T)
    seeds = [int(s) for s in seeds_for(og, 8, 2)] + [int(np.argmax(np.diff(og.export()["a_rowptr"])))]
    expect = np.stack([og.query(s, c, S, T) for s in seeds])
    sd = torch.tensor(seeds, dtype=torch.int32).cuda()
    res = []
    for limit in (og.m, 0):
        gg.set_push_limit(limit)
        res.append(run_single(gg, torch, sd, S, list(range(len(seeds)))).cpu().numpy())
        assert np.all(l1_rows(res[-1], expect) <= TOL), limit
    gg.set_push_limit(-1)
    assert np.abs(res[0] - res[1]).max() <= 1e-6


def support_edges(ex, s):
    """Out-edges of y2's support F2 = out(F) + {s}, F = out(s) + {s}: the
    work of a pushed step 3 (every y2 term is positive, so F2 is exactly
    the support)."""
    rp, col = ex["a_rowptr"], ex["a_col"]
    nb = col[rp[s]:rp[s + 1]]
    f = nb if s in nb else np.append(nb, s)
    f2 = np.unique(np.concatenate([col[rp[u]:rp[u + 1]] for u in f] + [[s]]))
    return int(np.diff(rp)[f2].sum()), f.size


@pytest.mark.parametrize("Sq,layout", [(5, 2), (8, 2), (5, 0)])
def test_third_step_push_and_pull(rmat13, torch, Sq, layout):
    """Single seeds whose second step is pushed, with step 3 always pushed
    (a limit above every frontier), always pulled (0) and chosen per seed
    (the median frontier W3 = out-edges of y2's support): all within L1 of
    the oracle, push and pull within FP32 rounding of each other, the
    pushed queries bitwise reproducible in any order, and each seed of the
    per-seed choice equal bit for bit to the direction its W3 picks (seeds
    whose step 2 is pulled, F over 2048 nodes, pull step 3 too).  Layout 0
    lists y2's support by node id, layout 2 through the gather rows."""
    og, gg = rmat13
    ex = og.export()
    seeds = [int(s) for s in seeds_for(og, 12, 707)]
    seeds += [int(np.argmax(np.diff(ex["a_rowptr"]))), int(np.flatnonzero(ex["padded"])[0])]
    w3, nf = zip(*[support_edges(ex, s) for s in seeds])
    w3, step2_pushed = np.array(w3), np.array(nf) <= 2048
    mid, big = int(np.median(w3)), int(w3.max())
    assert (w3 <= mid).any() and (w3 > mid).any()
    expect = np.stack([og.query(s, c, Sq, T) for s in seeds])
    sd = torch.tensor(seeds, dtype=torch.int32).cuda()
    runs = {}
    try:
        gg.set_gather_layout(layout)
        gg.set_push_limit(og.m)
        for limit in (big, 0, mid):
            gg.set_third_push_limit(limit)
            assert gg.get_third_push_limit() == limit
            R = run_single(gg, torch, sd, Sq, list(range(len(seeds))))
            R2 = run_single(gg, torch, sd, Sq, list(reversed(range(len(seeds)))))
            assert torch.equal(R, R2), limit
            runs[limit] = R.cpu().numpy()
            assert np.all(l1_rows(runs[limit], expect) <= TOL), limit
    finally:
        gg.set_third_push_limit(-1)
        gg.set_push_limit(-1)
        gg.set_gather_layout(2)
    pushed, pulled, mixed = runs[big], runs[0], runs[mid]
    assert np.abs(pushed - pulled).max() <= 1e-6
    assert not np.array_equal(pushed, pulled)
    for i, w in enumerate(w3):
        if not step2_pushed[i]:
            assert np.array_equal(pushed[i], pulled[i]), i
        assert np.array_equal(mixed[i], (pushed if w <= mid else pulled)[i]), (i, w, mid)


def test_third_step_push_weighted(tpa, torch):
    """Row-softmax edge weights in the pushed third step."""
    og = oracle.Graph.rmat(10, 12000, 24)
    gg = tpa.Graph.rmat(10, 12000, 24)
    theta = ti.draw_logits(og.m, 10)
    og.set_logits(theta.astype(np.float64))
    gg.set_logits(torch.from_numpy(theta).cuda())
    og.preprocess(c, T, EPS)
    gg.preprocess(c, T)
    seeds = [int(s) for s in seeds_for(og, 8, 4)]
    expect = np.stack([og.query(s, c, S, T) for s in seeds])
    sd = torch.tensor(seeds, dtype=torch.int32).cuda()
    res = []
    gg.set_push_limit(og.m)
    try:
        for limit in (4 * og.m, 0):
            gg.set_third_push_limit(limit)
            res.append(run_single(gg, torch, sd, S, list(range(len(seeds)))).cpu().numpy())
            assert np.all(l1_rows(res[-1], expect) <= TOL), limit
    finally:
        gg.set_third_push_limit(-1)
        gg.set_push_limit(-1)
    assert np.abs(res[0] - res[1]).max() <= 1e-6


def test_push_plan_size_limit(tpa, torch):
    """Each block of the pushed first two steps plans the seed's frontier
    F = out(s) + {s} in LDS, up to 2048 nodes.  Seeds with 2047 out-edges
    (F fills the plan exactly), 2048 and 3000 (the plan does not fit: step 2
    is pulled) and a few out-edges must all match the oracle, under a push
    limit that admits every frontier."""
    rng = np.random.default_rng(99)
    n = 5000
    src = [np.zeros(3000, np.int64), np.full(2047, 1), np.full(2048, 2)]
    dst = [np.arange(1, 3001), np.arange(1001, 3048), np.arange(2000, 4048)]
    rest = np.arange(3, n)
    src.append(np.repeat(rest, 3))
    dst.append(rng.integers(0, n, size=3 * rest.size))
    src, dst = np.concatenate(src).astype(np.int32), np.concatenate(dst).astype(np.int32)
    og = oracle.Graph(n, src, dst)
    og.preprocess(c, T, EPS)
    gg = tpa.Graph.from_edges(n, src, dst)
    gg.preprocess(c, T)
    seeds = [0, 1, 2, 17, 4999]
    sd = torch.tensor(seeds, dtype=torch.int32).cuda()
    gg.set_push_limit(og.m)
    try:
        R = run_single(gg, torch, sd, S, list(range(len(seeds)))).cpu().numpy()
    finally:
        gg.set_push_limit(-1)
    expect = np.stack([og.query(s, c, S, T) for s in seeds])
    assert np.all(l1_rows(R, expect) <= TOL), l1_rows(R, expect)


@pytest.mark.parametrize("nn,scale,samples", [(3000, 12, 48000), (37, 6, 300), (64, 6, 500)])
def test_pushed_frontier_on_ragged_node_counts(tpa, torch, nn, scale, samples):
    """The conversion after a pushed step 2 writes the frontier bitmap one
    64-row round at a time; node counts that leave a partial last round
    (3000 = 46*64 + 56, 37 < 64) or fill it exactly (64) must mark every
    non-zero row.  A skipped live row would drop its terms from step 3, so
    the pushed queries must match the pulled ones (no push, no skip) to
    FP32 rounding element by element, and the oracle in L1."""
    og = oracle.Graph.rmat(scale, samples, 0xF00 + nn, n_nodes=nn)
    og.preprocess(c, T, EPS)
    gg = tpa.Graph.rmat(scale, samples, 0xF00 + nn, n_nodes=nn)
    gg.preprocess(c, T)
    seeds = [int(s) for s in seeds_for(og, 12, 505)] + [nn - 1, 0]
    sd = torch.tensor(seeds, dtype=torch.int32).cuda()
    res = []
    try:
        for limit in (og.m, 0):
            gg.set_push_limit(limit)
            res.append(run_single(gg, torch, sd, S, list(range(len(seeds)))).cpu().numpy().astype(np.float64))
    finally:
        gg.set_push_limit(-1)
    pushed, pulled = res
    assert np.all(np.abs(pushed - pulled) <= 1e-4 * np.abs(pulled) + 1e-9)
    expect = np.stack([og.query(s, c, S, T) for s in seeds])
    assert np.all(l1_rows(pushed, expect) <= TOL)


@pytest.mark.parametrize("kt", [1, 2, 16, 64])
def test_dense_restarts_ragged_nodes_and_tiles(tpa, torch, kt):
    """Dense restart vectors are transposed per tile into a node-major
    block (64 nodes per transpose block) that every step's epilogue reads:
    a node count that is not a multiple of 64 (1000) and a batch that
    leaves a ragged last tile (k = 70) must match the oracle."""
    og = oracle.Graph.rmat(10, 14000, 0xD15E, n_nodes=1000)
    og.preprocess(c, T, EPS)
    gg = tpa.Graph.rmat(10, 14000, 0xD15E, n_nodes=1000)
    gg.preprocess(c, T)
    rng = np.random.default_rng(77)
    k = 70
    Q = rng.random((k, og.n)) * (rng.random((k, og.n)) < 0.05)
    Q[:, 0] += 1e-3
    Q /= Q.sum(axis=1, keepdims=True)
    gg.set_tuning(seed_tile=kt)
    try:
        R = gg.query_dense(torch.from_numpy(Q.astype(np.float32)), c, S, T).cpu().numpy()
    finally:
        gg.set_tuning(0, 0)
    for j in (0, 1, kt - 1, kt, k - 1):
        if j < k:
            assert l1_rows(R[j], og.query_q(Q[j], c, S, T)) <= TOL, j


@pytest.mark.parametrize("kt,Sq", [(64, 5), (64, 3), (1, 3)])
def test_frontier_skip_is_bitwise_neutral(rmat13, torch, kt, Sq):
    """The pull after a pushed first step skips the rows the push left zero.
    The skipped terms are exact zeros, so the results equal the unskipped
    pull (push limit 0 turns the skip off) bit for bit, and match the
    oracle (tiles pull their second step here)."""
    og, gg = rmat13
    sd = seeds_for(og, 70 if kt == 64 else 6, 404)
    seeds = torch.from_numpy(sd).cuda()
    res = []
    try:
        gg.set_tuning(seed_tile=kt)
        gg.set_tile_push_limit(0)
        for limit in (-1, 0):
            gg.set_push_limit(limit)
            res.append(gg.query(seeds, c, Sq, T))
    finally:
        gg.set_push_limit(-1)
        gg.set_tile_push_limit(-1)
        gg.set_tuning(0, 0)
    assert torch.equal(res[0], res[1])
    expect = np.stack([og.query(int(s), c, Sq, T) for s in sd])
    assert np.all(l1_rows(res[0].cpu().numpy(), expect) <= TOL)


def tile_runs(gg, torch, seeds, kt, Sq, limits):
    """Queries of one batch under several tile push limits."""
    out = {}
    try:
        gg.set_tuning(seed_tile=kt)
        for limit in limits:
            gg.set_tile_push_limit(limit)
            assert gg.get_tile_push_limit() == limit
            out[limit] = gg.query(seeds, c, Sq, T)
    finally:
        gg.set_tile_push_limit(-1)
        gg.set_tuning(0, 0)
    return out


@pytest.mark.parametrize("kt,Sq", [(2, 5), (16, 4), (16, 5), (64, 5), (64, 8)])
def test_tile_second_step_push_and_pull(rmat13, torch, kt, Sq):
    """Seed tiles with step 2 always pushed (a tile limit above every tile's
    frontier), always pulled (0) and chosen per tile (the median tile
    frontier): all within L1 of the oracle, push and pull within FP32
    rounding of each other, the pushed batch bitwise reproducible, and each
    tile of the per-tile choice equal bit for bit to the direction its
    frontier picks.  70 seeds leave a ragged last tile; the largest
    out-degree's seed and a dangling node's seed are among them."""
    og, gg = rmat13
    ex = og.export()
    sd = np.concatenate([seeds_for(og, 68, 606),
                         [int(np.argmax(np.diff(ex["a_rowptr"]))), int(np.flatnonzero(ex["padded"])[0])]])
    sd = sd.astype(np.int32)
    k = sd.size
    tiles = [range(t, min(k, t + kt)) for t in range(0, k, kt)]
    W = np.array([sum(frontier_edges(ex, int(sd[i])) for i in t) for t in tiles])
    mid, big = int(np.median(W)), int(W.max())
    seeds = torch.from_numpy(sd).cuda()
    runs = tile_runs(gg, torch, seeds, kt, Sq, (big, 0, mid))
    again = tile_runs(gg, torch, seeds, kt, Sq, (big,))
    assert torch.equal(runs[big], again[big])
    expect = np.stack([og.query(int(s), c, Sq, T) for s in sd])
    res = {lim: r.cpu().numpy() for lim, r in runs.items()}
    for lim, r in res.items():
        assert np.all(l1_rows(r, expect) <= TOL), lim
    pushed, pulled, mixed = res[big], res[0], res[mid]
    assert np.abs(pushed - pulled).max() <= 1e-6
    assert not np.array_equal(pushed, pulled)  # the pushed sums round differently somewhere
    for t, w in zip(tiles, W):
        rows = list(t)
        assert np.array_equal(mixed[rows], (pushed if w <= mid else pulled)[rows]), (rows[0], w, mid)


@pytest.mark.parametrize("kt", [4, 64])
def test_tile_second_step_push_weighted(tpa, torch, kt):
    """Row-softmax edge weights: the tile's plan takes each y1 entry from
    its A~ edge weight and the push multiplies by the frontier edge's
    weight; pushed and pulled tiles match the oracle."""
    og = oracle.Graph.rmat(10, 12000, 23)
    gg = tpa.Graph.rmat(10, 12000, 23)
    theta = ti.draw_logits(og.m, 9)
    og.set_logits(theta.astype(np.float64))
    gg.set_logits(torch.from_numpy(theta).cuda())
    og.preprocess(c, T, EPS)
    gg.preprocess(c, T)
    sd = seeds_for(og, 40, 3)
    runs = tile_runs(gg, torch, torch.from_numpy(sd).cuda(), kt, S, (4 * og.m, 0))
    expect = np.stack([og.query(int(s), c, S, T) for s in sd])
    for lim, r in runs.items():
        assert np.all(l1_rows(r.cpu().numpy(), expect) <= TOL), lim
    assert (runs[4 * og.m] - runs[0]).abs().max().item() <= 1e-6


@pytest.mark.parametrize("kt", [4, 64])
def test_tile_push_with_invalid_seeds(rmat13, tpa, torch, kt):
    """A tile whose columns include out-of-range seeds: the plan gives those
    columns no entries, their rows come out NaN with the sticky error raised,
    and every valid column matches the oracle whether step 2 is pushed or
    pulled."""
    og, gg = rmat13
    sd = seeds_for(og, 10, 808).astype(np.int32)
    sd[2], sd[7] = -1, og.n  # invalid
    valid = [i for i in range(sd.size) if 0 <= sd[i] < og.n]
    runs = tile_runs(gg, torch, torch.from_numpy(sd).cuda(), kt, S, (1 << 40, 0))
    expect = np.stack([og.query(int(sd[i]), c, S, T) for i in valid])
    for lim, r in runs.items():
        r = r.cpu().numpy()
        assert np.all(np.isnan(r[2])) and np.all(np.isnan(r[7])), lim
        assert np.all(l1_rows(r[valid], expect) <= TOL), lim
    with pytest.raises(tpa.TPAError):
        gg.device_error()
    gg.device_error()  # cleared


def test_tile_push_plan_limit(tpa, torch):
    """The device plans a tile's push with one entry per frontier node, at
    most 16384: a tile of 64 seeds with 300 out-edges each (19264 entries)
    pulls, one of 54 of them (16254 entries) pushes.  Their out-neighbours
    include nodes of 600 out-edges, whose edges are pushed in three pieces.
    Both match the oracle; the first equals the pulled tile bit for bit,
    the second does not."""
    rng = np.random.default_rng(98)
    n = 20000
    src, dst = [], []
    for s in range(64):
        src.append(np.full(300, s))
        dst.append(np.concatenate([64 + rng.choice(36, 4, replace=False), 100 + rng.choice(n - 100, 296, replace=False)]))
    for h in range(64, 100):
        src.append(np.full(600, h))
        dst.append(rng.choice(n, 600, replace=False))
    rest = np.arange(100, n)
    src.append(np.repeat(rest, 3))
    dst.append(rng.integers(0, n, size=3 * rest.size))
    src, dst = np.concatenate(src).astype(np.int32), np.concatenate(dst).astype(np.int32)
    og = oracle.Graph(n, src, dst)
    og.preprocess(c, T, EPS)
    gg = tpa.Graph.from_edges(n, src, dst)
    gg.preprocess(c, T)
    ex = og.export()
    assert int(np.diff(ex["a_rowptr"])[:64].min()) == 300
    for cols in (64, 54):
        sd = np.arange(cols, dtype=np.int32)
        runs = tile_runs(gg, torch, torch.from_numpy(sd).cuda(), 64, S, (1 << 40, 0))
        expect = np.stack([og.query(int(s), c, S, T) for s in sd])
        for lim, r in runs.items():
            assert np.all(l1_rows(r.cpu().numpy(), expect) <= TOL), (cols, lim)
        same = torch.equal(runs[1 << 40], runs[0])
        assert same == (cols == 64), cols


# ---------------------------------------------------------------- gather layout
@pytest.mark.parametrize("weighted", [False, True])
def test_gather_layout_node_and_hub_order(tpa, torch, weighted):
    """Hub-first and node-order work vectors: stranger vector, single-seed
    queries (pushed and pulled step 2, S = 2 with a pulled first step), seed
    tiles 4 and 64 and dense restart vectors all match the oracle and agree
    with each other to FP32 rounding, with 1/outdeg and with logit weights
    (whose per-edge weights follow the re-sorted rows)."""
    og = oracle.Graph.rmat(12, 60000, 31)
    gg = tpa.Graph.rmat(12, 60000, 31)
    if weighted:
        theta = ti.draw_logits(gg.m, 8)
        og.set_logits(theta.astype(np.float64))
        gg.set_logits(torch.from_numpy(theta).cuda())
    og.preprocess(c, T, EPS)
    sd = ti.draw_seeds(og.export()["padded"] == 0, 70, 5)
    seeds = torch.from_numpy(sd).cuda()
    Q = np.random.default_rng(6).random((3, gg.n))
    Q /= Q.sum(axis=1, keepdims=True)
    Qt = torch.from_numpy(Q.astype(np.float32)).cuda()
    single = np.stack([og.query(int(s), c, S, T) for s in sd])
    expect = [og.str]
    for kt in (1, 4, 64):
        expect += [single[:9] if kt == 1 else single, np.stack([og.query_q(q, c, S, T) for q in Q])]
    expect += [single[:3], np.stack([og.query(int(s), c, 2, T) for s in sd[:3]])]
    res = []
    try:
        for hub in (True, False):
            gg.set_gather_layout(hub)
            assert gg.get_gather_layout() == (2 if hub else 0)
            gg.preprocess(c, T)
            out = [gg.stranger()]
            for kt in (1, 4, 64):
                gg.set_tuning(seed_tile=kt)
                out.append(gg.query(seeds[:9] if kt == 1 else seeds, c, S, T))
                out.append(gg.query_dense(Qt, c, S, T))
            gg.set_tuning(seed_tile=1)
            gg.set_push_limit(0)
            out.append(gg.query(seeds[:3], c, S, T))
            gg.set_push_limit(-1)
            out.append(gg.query(seeds[:3], c, 2, T))
            res.append(out)
    finally:
        gg.set_tuning(0, 0)
        gg.set_gather_layout(True)
    for i, (a, b, e) in enumerate(zip(res[0], res[1], expect)):
        assert np.all(l1_rows(a.cpu().numpy(), e) <= TOL), i
        assert np.all(l1_rows(b.cpu().numpy(), e) <= TOL), i
        assert float((a - b).abs().max()) <= 1e-6, i


@pytest.mark.parametrize("weighted", [False, True])
def test_group_order_is_bitwise_row_order(tpa, torch, weighted):
    """Layout 2 re-sorts each group item's edges by rank across its rows and
    sends each product to its row-order LDS slot: the stranger vector,
    single-seed queries (pushed, pulled, S = 2), exact CPI (seed and dense)
    and both gradients are bit for bit those of layout 1, with 1/outdeg and
    with logit weights (read through the slot).  The group-ordered ids are
    one more int32 per edge for each of the two single-vector schedules
    (the forward's over A~^T and the adjoint's over A~), held only under
    layout 2."""
    og = oracle.Graph.rmat(15, 300000, 41)
    gg = tpa.Graph.rmat(15, 300000, 41)
    if weighted:
        theta = ti.draw_logits(gg.m, 42)
        og.set_logits(theta.astype(np.float64))
        gg.set_logits(torch.from_numpy(theta).cuda())
    og.preprocess(c, T, EPS)
    sd = ti.draw_seeds(og.export()["padded"] == 0, 6, 43)
    seeds = torch.from_numpy(sd).cuda()
    q = np.random.default_rng(44).random(gg.n)
    q /= q.sum()
    qt = torch.from_numpy(q.astype(np.float32)).cuda()
    W = torch.from_numpy(ti.draw_loss_weights((1, gg.n), 45)).cuda()
    res, mem = [], []
    try:
        for layout in (1, 2):
            gg.set_gather_layout(layout)
            gg.preprocess(c, T)
            out = [gg.stranger()]
            for j in range(len(sd)):
                out.append(gg.query(seeds[j:j + 1], c, S, T))
            gg.set_push_limit(0)
            out.append(gg.query(seeds[:1], c, S, T))
            gg.set_push_limit(-1)
            out.append(gg.query(seeds[1:2], c, 2, T))
            out.append(gg.cpi(c, 0, -1, EPS, seed=int(sd[2])))
            out.append(gg.cpi(c, 3, 9, EPS, q=qt))
            out.extend(gg.backward(W, c, S, T, seeds=seeds[3:4]))
            res.append(out)
            mem.append(gg.device_bytes())
    finally:
        gg.set_gather_layout(2)
        gg.set_logits(None)
    assert res[1][-2] is not None
    for i, (a, b) in enumerate(zip(res[0], res[1])):
        assert (a is None) == (b is None), i
        assert a is None or torch.equal(a, b), i
    for sv, r in zip(sd, res[1][1:7]):
        assert np.all(l1_rows(r.cpu().numpy(), og.query(int(sv), c, S, T)[None]) <= TOL)
    assert mem[1] - mem[0] == 8 * gg.m


@pytest.mark.parametrize("n", [(1 << 23) - 1, 1 << 23])
def test_group_order_node_id_limit(tpa, torch, n):
    """The group-ordered ids keep 23 bits of gather row: a graph of 2^23 - 1
    nodes gets them (its highest rank, n - 1, still fits), one of 2^23 nodes
    keeps layout 1's ids; either way queries and the stranger vector are
    bitwise those of layout 1, each query's mass is 1, and both are within
    L1 <= 1e-5 of the oracle.  The edges join a dense core of 2048 nodes to
    the top node ids, so that gather rows near n - 1 appear in group items."""
    rng = np.random.default_rng(47)
    core = rng.integers(0, 2048, size=(2, 40000))
    top = n - 1 - rng.integers(0, 2048, size=20000)
    low = rng.integers(0, 2048, size=20000)
    src = np.concatenate([core[0], top, low]).astype(np.int32)
    dst = np.concatenate([core[1], low, top]).astype(np.int32)
    gg = tpa.Graph.from_edges(n, src, dst)
    seeds = torch.tensor([3, 100, n - 1, n - 7], dtype=torch.int32).cuda()
    res, mem = [], []
    try:
        for layout in (1, 2):
            gg.set_gather_layout(layout)
            gg.preprocess(c, T)
            out = [gg.stranger()] + [gg.query(seeds[j:j + 1], c, S, T) for j in range(4)]
            res.append(out)
            mem.append(gg.device_bytes())
    finally:
        gg.set_gather_layout(2)
    for i, (a, b) in enumerate(zip(res[0], res[1])):
        assert torch.equal(a, b), i
    for r in res[1][1:]:
        assert abs(float(r.double().sum()) - 1.0) < 1e-4
    assert mem[1] - mem[0] == (4 * gg.m if n < (1 << 23) else 0)
    # and against the oracle
    og = oracle.Graph(n, src, dst)
    assert og.m == gg.m
    og.preprocess(c, T, EPS)
    assert np.abs(res[1][0].cpu().numpy().astype(np.float64) - og.str).sum() <= 1e-5
    for j, s in enumerate(seeds.cpu().tolist()):
        got = res[1][1 + j][0].cpu().numpy().astype(np.float64)
        assert np.abs(got - og.query(int(s), c, S, T)).sum() <= 1e-5, s


# ---------------------------------------------------------------- packed
def test_packed_blocks_equal_separate_graphs(tpa, torch):
    params = [(9, 4000, 1, 400), (10, 9000, 2, 0), (8, 1500, 3, 200)]
    ogs, ggs = [], []
    for scale, samples, seed, nn in params:
        n_nodes = nn or (1 << scale)
        og = oracle.Graph.rmat(scale, samples, seed, n_nodes=n_nodes)
        og.preprocess(c, T, EPS)
        ogs.append(og)
        ggs.append(tpa.Graph.rmat(scale, samples, seed, n_nodes=n_nodes))
    pk = tpa.Graph.pack(ggs)
    off = pk.block_offsets()
    assert pk.nblocks == 3 and off[-1] == pk.n
    pk.preprocess(c, T)
    st = pk.stranger().cpu().numpy()
    P = 4
    seeds = np.stack([off[b] + seeds_for(ogs[b], P, 20 + b) for b in range(3)]).astype(np.int32)
    for kt in (1, 4, 0):
        pk.set_tuning(seed_tile=kt)
        R = pk.query_packed(torch.from_numpy(seeds), c, S, T).cpu().numpy()
        for b, og in enumerate(ogs):
            lo, hi = off[b], off[b + 1]
            assert l1_rows(st[lo:hi], og.str) <= TOL
            for j in range(P):
                assert l1_rows(R[j, lo:hi], og.query(int(seeds[b, j] - lo), c, S, T)) <= TOL


# ---------------------------------------------------------------- weights
def test_logit_weights_forward(tpa, torch):
    og = oracle.Graph.rmat(10, 12000, 21)
    gg = tpa.Graph.rmat(10, 12000, 21)
    theta = ti.draw_logits(og.m, 4)
    og.set_logits(theta.astype(np.float64))
    gg.set_logits(torch.from_numpy(theta).cuda())
    _, _, w = gg.export()
    assert np.abs(w.cpu().numpy() - og.export()["a_w"]).max() < 1e-6
    og.preprocess(c, T, EPS)
    gg.preprocess(c, T)
    assert l1_rows(gg.stranger().cpu().numpy(), og.str) <= TOL
    seeds = seeds_for(og, 8, 1)
    for kt in (1, 8):
        gg.set_tuning(seed_tile=kt)
        R = gg.query(torch.from_numpy(seeds), c, S, T).cpu().numpy()
        expect = np.stack([og.query(int(s), c, S, T) for s in seeds])
        assert np.all(l1_rows(R, expect) <= TOL)


# ---------------------------------------------------------------- errors
def test_query_errors(tpa, torch):
    gg = tpa.Graph.rmat(8, 2000, 1)
    s = torch.tensor([1], dtype=torch.int32)
    with pytest.raises(tpa.TPAError) as e:
        gg.query(s, c, S, T)
    assert e.value.status == -2
    gg.preprocess(c, T)
    for args, code in (((0.2, S, T), -3), ((c, S, 12), -3), ((c, 0, T), -1), ((c, 6, 5), -1), ((1.5, S, T), -1)):
        with pytest.raises(tpa.TPAError) as e:
            gg.query(s, *args)
        assert e.value.status == code
    gg.query(s, c, S, T)  # still usable


@pytest.mark.parametrize("limit", [-1, 0])
def test_bad_single_seed_gives_nan_row(tpa, torch, limit):
    """Seed tile 1 (pushed and pulled step 2): an out-of-range seed gives a
    NaN row and the sticky error, and the next valid query is unaffected."""
    gg = tpa.Graph.rmat(8, 2000, 1)
    gg.preprocess(c, T)
    gg.set_push_limit(limit)
    try:
        good = gg.query(torch.tensor([3], dtype=torch.int32), c, S, T)
        for bad in (256, -1):
            r = gg.query(torch.tensor([bad], dtype=torch.int32), c, S, T)
            assert bool(torch.isnan(r).all())
            with pytest.raises(tpa.TPAError):
                gg.device_error()
        again = gg.query(torch.tensor([3], dtype=torch.int32), c, S, T)
        assert torch.equal(good, again)
        gg.device_error()
    finally:
        gg.set_push_limit(-1)


def test_bad_seed_gives_nan_row_and_sticky_error(tpa, torch):
    gg = tpa.Graph.rmat(8, 2000, 1)
    gg.preprocess(c, T)
    R = gg.query(torch.tensor([3, 256, -1, 7], dtype=torch.int32), c, S, T).cpu().numpy()
    assert np.all(np.isnan(R[1])) and np.all(np.isnan(R[2]))
    assert np.all(np.isfinite(R[0])) and np.all(np.isfinite(R[3]))
    with pytest.raises(tpa.TPAError):
        gg.device_error()
    gg.device_error()  # cleared


# ---------------------------------------------------------------- XCD-sliced sweep
@pytest.mark.parametrize("nn,scale,samples,ew", [
    (None, 15, 1 << 19, 128), (None, 15, 1 << 19, 512), (20000, 15, 1 << 18, 64), (5000, 13, 1 << 17, 64)])
def test_sliced_sweep_stranger_parity(tpa, torch, nn, scale, samples, ew):
    """Rows of A~^T longer than a group item summed as 8 runs, one per
    source slice (ranks below 8192 by row mod 8, the others by blocks of
    1024), each slice's runs in the blocks of one XCD, then a finish pass in
    slice order: the stranger vector and queries against the oracle, with
    ragged node counts and group budgets from 32 to 512 edges; mode 0 gives
    back the unsliced sweep bit for bit."""
    kw = {} if nn is None else {"n_nodes": nn}
    og = oracle.Graph.rmat(scale, samples, 0x51C + scale, **kw)
    og.preprocess(c, T, EPS)
    gg = tpa.Graph.rmat(scale, samples, 0x51C + scale, **kw)
    gg.set_tuning(1, ew)
    gg.preprocess(c, T)
    assert gg.get_sliced_sweep() == (1, False)  # off below 2^23 nodes by default
    base = gg.stranger().cpu().numpy()
    gg.set_sliced_sweep(2)
    gg.preprocess(c, T)
    assert gg.get_sliced_sweep() == (2, True)
    st = gg.stranger().cpu().numpy()
    assert l1_rows(base, og.str) <= TOL
    assert l1_rows(st, og.str) <= TOL, l1_rows(st, og.str)
    assert st.min() >= 0
    assert np.all(np.abs(st - base) <= 1e-5 * base + 1e-12)
    seeds = seeds_for(og, 4, 31)
    gg.set_tuning(0, 0)
    R = gg.query(torch.from_numpy(seeds), c, S, T).cpu().numpy()
    for i, s in enumerate(seeds):
        assert l1_rows(R[i], og.query(int(s), c, S, T)) <= TOL
    gg.set_tuning(1, ew)
    gg.set_sliced_sweep(0)
    gg.preprocess(c, T)
    assert gg.get_sliced_sweep() == (0, False)
    assert np.array_equal(gg.stranger().cpu().numpy(), base)


def test_sliced_sweep_skips_weighted_and_node_order(tpa, torch):
    """Graphs with logit weights, and the node-order layout, keep the
    unsliced sweep (the sliced copy holds hub-first ids of 1/outdeg graphs)."""
    og = oracle.Graph.rmat(12, 1 << 16, 9)
    gg = tpa.Graph.rmat(12, 1 << 16, 9)
    gg.set_tuning(1, 64)
    gg.set_sliced_sweep(2)
    theta = ti.draw_logits(og.m, 3)
    og.set_logits(theta.astype(np.float64))
    gg.set_logits(torch.from_numpy(theta).cuda())
    og.preprocess(c, T, EPS)
    gg.preprocess(c, T)
    assert gg.get_sliced_sweep() == (2, False)
    assert l1_rows(gg.stranger().cpu().numpy(), og.str) <= TOL
    gg.set_logits(None)
    og.set_logits(None)
    gg.set_gather_layout(0)
    og.preprocess(c, T, EPS)
    gg.preprocess(c, T)
    assert gg.get_sliced_sweep() == (2, False)
    assert l1_rows(gg.stranger().cpu().numpy(), og.str) <= TOL
    gg.set_gather_layout(2)
    gg.preprocess(c, T)
    assert gg.get_sliced_sweep() == (2, True)
    assert l1_rows(gg.stranger().cpu().numpy(), og.str) <= TOL


@pytest.mark.parametrize("ew", [64, 512])
def test_sliced_single_seed_pulls(tpa, torch, ew):
    """Once preprocessing built the sliced schedule, single-seed queries pull
    their dense family steps with it: plain pulls, the pulls after pushed
    second and third steps (with their frontier skips), and dense restarts,
    against the oracle and against the unsliced pulls to FP32 rounding."""
    og = oracle.Graph.rmat(15, 1 << 19, 0x51D)
    og.preprocess(c, T, EPS)
    gg = tpa.Graph.rmat(15, 1 << 19, 0x51D)
    gg.set_tuning(1, ew)
    seeds = seeds_for(og, 6, 77)
    sd = torch.from_numpy(seeds).cuda()
    expect = np.stack([og.query(int(s), c, S, T) for s in seeds])
    rng = np.random.default_rng(78)
    Q = rng.random((2, og.n))
    Q /= Q.sum(axis=1, keepdims=True)
    expect_q = np.stack([og.query_q(q, c, S, T) for q in Q])
    res = {}
    try:
        for mode in (0, 2):
            gg.set_sliced_sweep(mode)
            gg.preprocess(c, T)
            assert gg.get_sliced_sweep() == (mode, mode == 2)
            for third in (0, og.m):
                gg.set_third_push_limit(third)
                for push in (-1, 0):
                    gg.set_push_limit(push)
                    R = gg.query(sd, c, S, T).cpu().numpy()
                    assert np.all(l1_rows(R, expect) <= TOL), (mode, third, push, l1_rows(R, expect))
                    res[(mode, third, push)] = R.astype(np.float64)
            Rq = gg.query_dense(torch.from_numpy(Q.astype(np.float32)), c, S, T).cpu().numpy()
            assert np.all(l1_rows(Rq, expect_q) <= TOL)
            res[(mode, "q")] = Rq.astype(np.float64)
    finally:
        gg.set_push_limit(-1)
        gg.set_third_push_limit(-1)
    for key, a in res.items():
        if key[0] == 2:
            b = res[(0,) + key[1:]]
            assert np.all(np.abs(a - b) <= 1e-5 * np.abs(b) + 1e-9), key
