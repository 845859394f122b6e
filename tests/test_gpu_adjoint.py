"""Adjoint CPI and dense restart vectors on the GPU vs the FP64 oracle.

Gradients have no unit mass, so they are compared by normalised L1,
||g - g*||_1 / ||g*||_1 <= 1e-5 (the oracle's gradient is itself pinned by
central finite differences in test_oracle.py).
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


def nl1(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300)


def l1_rows(a, b):
    return np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)).sum(axis=-1)


def onehot(n, seeds):
    q = np.zeros((len(seeds), n))
    q[np.arange(len(seeds)), seeds] = 1.0
    return q


@pytest.fixture(scope="module")
def g10(tpa):
    scale, samples, seed = 10, 12000, 77
    og = oracle.Graph.rmat(scale, samples, seed)
    gg = tpa.Graph.rmat(scale, samples, seed)
    return og, gg


def test_query_dense_parity(g10, torch):
    og, gg = g10
    og.set_logits(None)
    gg.set_logits(None)
    og.preprocess(c, T, EPS)
    gg.preprocess(c, T)
    rng = np.random.default_rng(3)
    Q = rng.random((5, og.n))
    Q /= Q.sum(axis=1, keepdims=True)
    Q[0] = 0.0
    Q[0, 17] = 1.0                      # one-hot column
    Q[1] = 0.0
    Q[1, [3, 9, 400]] = 1.0 / 3.0       # seed set
    for kt in (1, 4, 64):
        gg.set_tuning(seed_tile=kt)
        R = gg.query_dense(torch.from_numpy(Q.astype(np.float32)), c, S, T).cpu().numpy()
        expect = np.stack([og.query_q(q, c, S, T) for q in Q])
        assert np.all(l1_rows(R, expect) <= TOL), l1_rows(R, expect)
    gg.set_tuning(0, 0)


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("kt", [1, 4, 64])
def test_backward_seeds_vs_oracle(g10, tpa, torch, weighted, kt):
    og, gg = g10
    theta = ti.draw_logits(og.m, 5) if weighted else np.zeros(og.m, np.float32)
    og.set_logits(theta.astype(np.float64) if weighted else None)
    gg.set_logits(torch.from_numpy(theta).cuda() if weighted else None)
    og.preprocess(c, T, EPS)
    gg.preprocess(c, T)
    seeds = ti.draw_seeds(og.export()["padded"] == 0, 6, 11)
    W = ti.draw_loss_weights((6, og.n), 12)
    gg.set_tuning(seed_tile=kt)
    try:
        dth, dq = gg.backward(torch.from_numpy(W), c, S, T, seeds=torch.from_numpy(seeds))
    finally:
        gg.set_tuning(0, 0)
    odth, _, odq = og.backward(onehot(og.n, seeds), W.astype(np.float64), c, S, T, og.K)
    assert nl1(dth.cpu().numpy(), odth) <= TOL, nl1(dth.cpu().numpy(), odth)
    assert nl1(dq.cpu().numpy(), odq) <= TOL, nl1(dq.cpu().numpy(), odq)


def test_backward_dense_q_and_checkpoints(g10, tpa, torch):
    og, gg = g10
    theta = ti.draw_logits(og.m, 6)
    og.set_logits(theta.astype(np.float64))
    gg.set_logits(torch.from_numpy(theta).cuda())
    og.preprocess(c, T, EPS)
    gg.preprocess(c, T)
    rng = np.random.default_rng(8)
    Q = rng.random((3, og.n))
    Q /= Q.sum(axis=1, keepdims=True)
    W = ti.draw_loss_weights((3, og.n), 9)
    odth, _, odq = og.backward(Q, W.astype(np.float64), c, S, T, og.K)
    ref = None
    for ck in (0, 1, 7, 116, -1):
        dth, dq = gg.backward(torch.from_numpy(W), c, S, T, q=torch.from_numpy(Q.astype(np.float32)),
                              checkpoint_every=ck)
        dth = dth.cpu().numpy()
        assert nl1(dth, odth) <= TOL
        assert nl1(dq.cpu().numpy(), odq) <= TOL
        if ref is None:
            ref = dth
        else:
            assert np.array_equal(dth, ref)  # recomputed iterates are bit-identical


@pytest.mark.parametrize("Sq,Tq", [(1, 10), (2, 10), (5, 5), (3, 20)])
def test_backward_S_T_cases(tpa, torch, Sq, Tq):
    og = oracle.Graph.rmat(9, 5000, 21)
    gg = tpa.Graph.rmat(9, 5000, 21)
    theta = ti.draw_logits(og.m, 2)
    og.set_logits(theta.astype(np.float64))
    gg.set_logits(torch.from_numpy(theta).cuda())
    og.preprocess(c, Tq, EPS)
    gg.preprocess(c, Tq)
    seeds = ti.draw_seeds(og.export()["padded"] == 0, 3, 4)
    W = ti.draw_loss_weights((3, og.n), 5)
    dth, dq = gg.backward(torch.from_numpy(W), c, Sq, Tq, seeds=torch.from_numpy(seeds))
    odth, _, odq = og.backward(onehot(og.n, seeds), W.astype(np.float64), c, Sq, Tq, og.K)
    assert nl1(dth.cpu().numpy(), odth) <= TOL
    assert nl1(dq.cpu().numpy(), odq) <= TOL


def test_backward_long_rows(g10, tpa, torch):
    """Small items force chunked long rows in both orientations."""
    og, gg = g10
    og.set_logits(None)
    gg.set_logits(None)
    og.preprocess(c, T, EPS)
    gg.preprocess(c, T)
    seeds = ti.draw_seeds(og.export()["padded"] == 0, 5, 1)
    W = ti.draw_loss_weights((5, og.n), 2)
    odth, _, odq = og.backward(onehot(og.n, seeds), W.astype(np.float64), c, S, T, og.K)
    for kt in (1, 4):
        gg.set_tuning(seed_tile=kt, edges_per_item=64)
        try:
            dth, dq = gg.backward(torch.from_numpy(W), c, S, T, seeds=torch.from_numpy(seeds))
        finally:
            gg.set_tuning(0, 0)
        assert nl1(dth.cpu().numpy(), odth) <= TOL
        assert nl1(dq.cpu().numpy(), odq) <= TOL


@pytest.mark.parametrize("sliced", [False, True])
def test_backward_packed_blocks(tpa, torch, sliced):
    """A block-diagonal batch: the adjoint per block against the oracle of
    each graph; sliced: the XCD-sliced stranger sweep and adjoint steps
    forced on (64-edge group items, so many rows are split)."""
    params = [(9, 4000, 1, 400), (10, 9000, 2, 0), (8, 1500, 3, 200)]
    ogs, ggs = [], []
    for scale, samples, seed, nn in params:
        n_nodes = nn or (1 << scale)
        ogs.append(oracle.Graph.rmat(scale, samples, seed, n_nodes=n_nodes))
        ggs.append(tpa.Graph.rmat(scale, samples, seed, n_nodes=n_nodes))
    pk = tpa.Graph.pack(ggs)
    if sliced:
        pk.set_sliced_sweep(2)
        pk.set_tuning(0, 64)
    pk.preprocess(c, T)
    assert pk.get_sliced_sweep()[1] == sliced
    off = pk.block_offsets()
    P = 2
    loc = [ti.draw_seeds(og.export()["padded"] == 0, P, 30 + b) for b, og in enumerate(ogs)]
    seeds = np.stack([off[b] + loc[b] for b in range(3)]).astype(np.int32)
    W = ti.draw_loss_weights((P, pk.n), 31)
    dth, dq = pk.backward(torch.from_numpy(W), c, S, T, seeds=torch.from_numpy(seeds), packed=True)
    dth = dth.cpu().numpy()
    dq = dq.cpu().numpy()
    eoff = 0
    for b, og in enumerate(ogs):
        og.preprocess(c, T, EPS)
        lo, hi = off[b], off[b + 1]
        odth, _, odq = og.backward(onehot(og.n, loc[b]), W[:, lo:hi].astype(np.float64), c, S, T, og.K)
        assert nl1(dth[eoff:eoff + og.m], odth) <= TOL
        assert nl1(dq[:, lo:hi], odq) <= TOL
        eoff += og.m


def test_autograd_function(g10, tpa, torch):
    og, gg = g10
    theta = torch.from_numpy(ti.draw_logits(og.m, 13)).cuda().requires_grad_(True)
    rng = np.random.default_rng(14)
    Qn = rng.random((2, og.n))
    Qn /= Qn.sum(axis=1, keepdims=True)
    Q = torch.from_numpy(Qn.astype(np.float32)).cuda().requires_grad_(True)
    W = torch.from_numpy(ti.draw_loss_weights((2, og.n), 15)).cuda()
    R = tpa.TPAFunction.apply(theta, Q, gg, c, S, T)
    loss = (R * W).sum()
    loss.backward()
    og.set_logits(theta.detach().cpu().numpy().astype(np.float64))
    _, K = og.tpa_forward(Qn, c, S, T, EPS)
    odth, _, odq = og.backward(Qn, W.cpu().numpy().astype(np.float64), c, S, T, K)
    assert nl1(theta.grad.cpu().numpy(), odth) <= TOL
    assert nl1(Q.grad.cpu().numpy(), odq) <= TOL
    og.preprocess(c, T, EPS)
    expect = np.stack([og.query_q(q, c, S, T) for q in Qn])
    assert np.all(l1_rows(R.detach().cpu().numpy(), expect) <= TOL)


def test_autograd_two_applies_on_one_graph(g10, tpa, torch):
    """Two forward passes on one graph with different logits before either
    backward: each output's gradients are those of its own logits (the
    backward restores the weights and stranger part its forward used when
    the graph has changed since), checked against the oracle."""
    og, gg = g10
    rng = np.random.default_rng(16)
    Qn = rng.random((2, og.n))
    Qn /= Qn.sum(axis=1, keepdims=True)
    thetas = [torch.from_numpy(ti.draw_logits(og.m, 17 + i)).cuda().requires_grad_(True) for i in range(2)]
    Qs = [torch.from_numpy(Qn.astype(np.float32)).cuda().requires_grad_(True) for _ in range(2)]
    Ws = [torch.from_numpy(ti.draw_loss_weights((2, og.n), 19 + i)).cuda() for i in range(2)]
    try:
        Rs = [tpa.TPAFunction.apply(thetas[i], Qs[i], gg, c, S, T) for i in range(2)]
        v_after_second = gg.version()
        # the first output's backward runs while the graph holds the second theta
        (Rs[0] * Ws[0]).sum().backward()
        assert gg.version() != v_after_second
        (Rs[1] * Ws[1]).sum().backward()
        for i in range(2):
            th = thetas[i].detach().cpu().numpy().astype(np.float64)
            og.set_logits(th)
            _, K = og.tpa_forward(Qn, c, S, T, EPS)
            odth, _, odq = og.backward(Qn, Ws[i].cpu().numpy().astype(np.float64), c, S, T, K)
            assert nl1(thetas[i].grad.cpu().numpy(), odth) <= TOL, i
            assert nl1(Qs[i].grad.cpu().numpy(), odq) <= TOL, i
            og.preprocess(c, T, EPS)
            expect = np.stack([og.query_q(q, c, S, T) for q in Qn])
            assert np.all(l1_rows(Rs[i].detach().cpu().numpy(), expect) <= TOL), i
    finally:
        gg.set_keep_iterates(False)
        gg.set_logits(None)
        og.set_logits(None)


@pytest.mark.parametrize("weighted", [False, True])
def test_backward_with_kept_iterates_is_bitwise_equal(g10, tpa, torch, weighted):
    """With tpa_set_keep_iterates the adjoint reads the stranger chain's
    iterates kept by preprocessing instead of recomputing them: the same
    values, so the gradients are bit for bit those of the recomputing path
    (automatic and checkpointed), and set_logits drops the kept iterates."""
    og, gg = g10
    theta = ti.draw_logits(og.m, 91) if weighted else None
    gg.set_logits(torch.from_numpy(theta).cuda() if weighted else None)
    seeds = torch.from_numpy(ti.draw_seeds(og.export()["padded"] == 0, 6, 92)).cuda()
    W = torch.from_numpy(ti.draw_loss_weights((6, og.n), 93)).cuda()
    try:
        gg.set_keep_iterates(False)
        gg.preprocess(c, T)
        ref = gg.backward(W, c, S, T, seeds=seeds)
        ref_ck = gg.backward(W, c, S, T, seeds=seeds, checkpoint_every=11)
        gg.set_keep_iterates(True)
        gg.preprocess(c, T)
        kept = gg.backward(W, c, S, T, seeds=seeds)
        for a, b in zip(kept, ref):
            assert torch.equal(a, b)
        for a, b in zip(ref_ck, ref):
            assert torch.equal(a, b)
        # new weights: the iterates are dropped until the next preprocessing
        gg.set_logits(torch.from_numpy(ti.draw_logits(og.m, 94)).cuda())
        gg.preprocess(c, T)
        again = gg.backward(W, c, S, T, seeds=seeds)
        gg.set_keep_iterates(False)
        gg.preprocess(c, T)
        fresh = gg.backward(W, c, S, T, seeds=seeds)
        for a, b in zip(again, fresh):
            assert torch.equal(a, b)
    finally:
        gg.set_keep_iterates(False)
        gg.set_logits(None)


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("kt,epi", [(1, 0), (1, 64), (16, 0), (64, 0), (64, 64)])
def test_backward_lambda_order_is_bitwise_equal(g10, tpa, torch, weighted, kt, epi):
    """Gather layout 2 (on this small graph: the adjoint's group items read
    their column ids in gather order, each row's sum in edge order) gives
    gradients bit for bit those of layout 1, for seeds, dense restarts and
    checkpoints, with short and long (chunked) rows; and they stay within the
    bar of the oracle."""
    og, gg = g10
    theta = ti.draw_logits(og.m, 95) if weighted else None
    og.set_logits(theta.astype(np.float64) if weighted else None)
    gg.set_logits(torch.from_numpy(theta).cuda() if weighted else None)
    og.preprocess(c, T, EPS)
    k = 1 if kt == 1 else 5
    seeds_np = ti.draw_seeds(og.export()["padded"] == 0, k, 96)
    seeds = torch.from_numpy(seeds_np).cuda()
    W = ti.draw_loss_weights((k, og.n), 97)
    Wd = torch.from_numpy(W).cuda()
    rng = np.random.default_rng(98)
    Q = rng.random((2, og.n))
    Q /= Q.sum(axis=1, keepdims=True)
    Qd = torch.from_numpy(Q.astype(np.float32)).cuda()
    W2 = torch.from_numpy(ti.draw_loss_weights((2, og.n), 99)).cuda()
    gg.set_tuning(seed_tile=kt, edges_per_item=epi)
    try:
        out = {}
        for layout in (1, 2):
            gg.set_gather_layout(layout)
            gg.preprocess(c, T)
            out[layout] = (gg.backward(Wd, c, S, T, seeds=seeds),
                           gg.backward(Wd, c, S, T, seeds=seeds, checkpoint_every=7),
                           gg.backward(W2, c, S, T, q=Qd))
        for a2, b2 in zip(out[1], out[2]):
            for a, b in zip(a2, b2):
                assert torch.equal(a, b)
        dth, dq = out[2][0]
        odth, _, odq = og.backward(onehot(og.n, seeds_np), W.astype(np.float64), c, S, T, og.K)
        assert nl1(dth.cpu().numpy(), odth) <= TOL
        assert nl1(dq.cpu().numpy(), odq) <= TOL
    finally:
        gg.set_gather_layout(2)
        gg.set_tuning(0, 0)
        gg.set_logits(None)
        og.set_logits(None)


@pytest.mark.parametrize("weighted", [False, True])
def test_backward_lambda_rank_order_large_graph(tpa, torch, weighted):
    """From 2^23 nodes gather layout 2 keeps the adjoint's lambda vectors in
    descending in-degree order (rows looked up per store, A~'s column ids
    mapped): the gradients are bit for bit those of layout 1 (node order),
    for a single seed and a tile of 4, and within the bar of the oracle.  The
    edges join a dense core of 2048 nodes to the top node ids, so lambda
    rows at both ends of the order are gathered."""
    n = 1 << 23
    rng = np.random.default_rng(48)
    core = rng.integers(0, 2048, size=(2, 40000))
    top = n - 1 - rng.integers(0, 2048, size=20000)
    low = rng.integers(0, 2048, size=20000)
    src = np.concatenate([core[0], top, low]).astype(np.int32)
    dst = np.concatenate([core[1], low, top]).astype(np.int32)
    gg = tpa.Graph.from_edges(n, src, dst)
    og = oracle.Graph(n, src, dst)
    assert og.m == gg.m
    theta = ti.draw_logits(og.m, 49) if weighted else None
    og.set_logits(theta.astype(np.float64) if weighted else None)
    gg.set_logits(torch.from_numpy(theta).cuda() if weighted else None)
    seeds_np = np.array([3, 100, n - 1, n - 7], np.int32)
    seeds = torch.from_numpy(seeds_np).cuda()
    W = ti.draw_loss_weights((4, n), 50)
    Wd = torch.from_numpy(W).cuda()
    out = {}
    try:
        for layout in (1, 2):
            gg.set_gather_layout(layout)
            gg.preprocess(c, T)
            out[layout] = (gg.backward(Wd, c, S, T, seeds=seeds), gg.backward(Wd[:1], c, S, T, seeds=seeds[:1]))
    finally:
        gg.set_gather_layout(2)
    for a2, b2 in zip(out[1], out[2]):
        for a, b in zip(a2, b2):
            assert torch.equal(a, b)
    og.preprocess(c, T, EPS)
    odth, _, odq = og.backward(onehot(n, seeds_np), W.astype(np.float64), c, S, T, og.K)
    dth, dq = out[2][0]
    assert nl1(dth.cpu().numpy(), odth) <= TOL
    assert nl1(dq.cpu().numpy(), odq) <= TOL
    gg.close()


def test_backward_sliced_sweep(tpa, torch):
    """The adjoint recomputes the stranger chain in XCD slices as
    preprocessing computed it, and sums the long rows of A~ in slices too
    (the edge gradient put back in A~'s order after the chain): the
    gradients are bitwise equal with the iterates kept, recomputed or
    checkpointed, agree with the unsliced adjoint to FP32 rounding, and
    match the oracle's."""
    og = oracle.Graph.rmat(12, 1 << 16, 41)
    og.preprocess(c, T, EPS)
    gg = tpa.Graph.rmat(12, 1 << 16, 41)
    gg.set_tuning(1, 64)
    gg.set_sliced_sweep(2)
    seeds = ti.draw_seeds(og.export()["padded"] == 0, 4, 42)
    W = ti.draw_loss_weights((4, og.n), 43)
    Wt, sd = torch.from_numpy(W).cuda(), torch.from_numpy(seeds).cuda()
    try:
        gg.preprocess(c, T)
        assert gg.get_sliced_sweep() == (2, True)
        ref = gg.backward(Wt, c, S, T, seeds=sd)
        ck = gg.backward(Wt, c, S, T, seeds=sd, checkpoint_every=11)
        gg.set_keep_iterates(True)
        gg.preprocess(c, T)
        kept = gg.backward(Wt, c, S, T, seeds=sd)
        for a, b, d in zip(ref, ck, kept):
            assert torch.equal(a, b) and torch.equal(a, d)
        gg.set_keep_iterates(False)
        gg.set_sliced_sweep(0)
        gg.preprocess(c, T)
        plain = gg.backward(Wt, c, S, T, seeds=sd)
    finally:
        gg.set_keep_iterates(False)
    for a, b in zip(ref, plain):
        a, b = a.double().cpu().numpy(), b.double().cpu().numpy()
        assert nl1(a, b) <= 1e-6
    odth, _, odq = og.backward(onehot(og.n, seeds), W.astype(np.float64), c, S, T, og.K)
    assert nl1(ref[0].cpu().numpy(), odth) <= TOL
    assert nl1(ref[1].cpu().numpy(), odq) <= TOL


def test_backward_sliced_adjoint_large_graph(tpa, torch):
    """From 2^23 nodes the stranger chain's adjoint sums the rows of A~
    longer than a group item (here hub sources of 600..5000 out-edges, whose
    destinations spread over lambda's rank order) in XCD slices, with the
    edge gradient put back in A~'s order after the chain: against the
    oracle, against the unsliced adjoint to FP32 rounding, and bitwise
    between checkpointed and recomputed iterates."""
    n = 1 << 23
    rng = np.random.default_rng(58)
    core = rng.integers(0, 2048, size=(2, 30000))
    hubs = np.array([5, 700, 2047, n - 3, n - 2000], np.int64)
    deg = np.array([600, 1500, 5000, 900, 2600])
    hsrc = np.repeat(hubs, deg)
    hdst = np.concatenate([rng.choice(n, d, replace=False) for d in deg])
    back = rng.integers(0, 2048, size=(2, 8000))
    src = np.concatenate([core[0], hsrc, hdst[:8000]]).astype(np.int32)
    dst = np.concatenate([core[1], hdst, back[1]]).astype(np.int32)
    gg = tpa.Graph.from_edges(n, src, dst)
    og = oracle.Graph(n, src, dst)
    assert og.m == gg.m
    seeds_np = np.array([5, 100, n - 3, int(hdst[3])], np.int32)
    seeds = torch.from_numpy(seeds_np).cuda()
    W = ti.draw_loss_weights((4, n), 59)
    Wd = torch.from_numpy(W).cuda()
    out = {}
    for mode in (0, 1):
        gg.set_sliced_sweep(mode)
        gg.preprocess(c, T)
        out[mode] = gg.backward(Wd, c, S, T, seeds=seeds)
        if mode == 1:
            ck = gg.backward(Wd, c, S, T, seeds=seeds, checkpoint_every=7)
            for a, b in zip(out[1], ck):
                assert torch.equal(a, b)
    for a, b in zip(out[1], out[0]):
        assert nl1(a.double().cpu().numpy(), b.double().cpu().numpy()) <= 1e-6
    og.preprocess(c, T, EPS)
    odth, _, odq = og.backward(onehot(n, seeds_np), W.astype(np.float64), c, S, T, og.K)
    dth, dq = out[1]
    assert nl1(dth.cpu().numpy(), odth) <= TOL
    assert nl1(dq.cpu().numpy(), odq) <= TOL
    gg.close()
