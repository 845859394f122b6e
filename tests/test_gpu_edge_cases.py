"""Degenerate graphs and sizes on the GPU path, against closed forms and the
oracle.

* No input edges: every node is dangling and gets a self-loop, so A~ = I.
  Then x(i) = c (1-c)^i e_s, the family part is (1 - (1-c)^S) e_s, the
  neighbor part ((1-c)^S - (1-c)^T) e_s (Section 3.2's scale applied to
  it), and the stranger part is the PageRank tail
  ((1-c)^T - (1-c)^(K+1)) / n on every node (Algorithm 2, Lemma 2).
* One node: r_TPA = 1 - (1-c)^(K+1) exactly as exact RWR.
* k = 0 queries, S = 1 (combine only) on the single-vector path, and
  seed-tile widths that leave a ragged last tile.
"""
import numpy as np
import pytest

import oracle
import tpa_inputs as ti

pytestmark = pytest.mark.gpu

c, S, T, EPS = ti.C, ti.S, ti.T, ti.EPS
K = 116
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


def no_edge_graph(tpa, n):
    e = np.zeros(0, np.int32)
    return tpa.Graph.from_edges(n, e, e)


@pytest.mark.parametrize("kt", [1, 4, 64])
def test_graph_without_edges_closed_form(tpa, torch, kt):
    n = 300
    gg = no_edge_graph(tpa, n)
    assert gg.m == n  # one self-loop per node
    gg.preprocess(c, T)
    tail = ((1 - c) ** T - (1 - c) ** (K + 1)) / n
    st = gg.stranger().cpu().numpy()
    assert np.allclose(st, tail, rtol=1e-5, atol=0)
    seeds = np.array([0, 7, 299, 150, 8], np.int32)
    gg.set_tuning(seed_tile=kt)
    try:
        R = gg.query(torch.from_numpy(seeds), c, S, T).cpu().numpy()
    finally:
        gg.set_tuning(0, 0)
    for r, s in zip(R, seeds):
        expect = np.full(n, tail)
        expect[s] += 1 - (1 - c) ** T
        assert np.abs(r - expect).sum() <= TOL
    og = oracle.Graph(n, np.zeros(0, np.int32), np.zeros(0, np.int32))
    og.preprocess(c, T, EPS)
    for r, s in zip(R, seeds):
        assert np.abs(r - og.query(int(s), c, S, T)).sum() <= TOL


def test_single_node_graph(tpa, torch):
    gg = no_edge_graph(tpa, 1)
    gg.preprocess(c, T)
    exact = 1 - (1 - c) ** (K + 1)
    for kt in (1, 64):
        gg.set_tuning(seed_tile=kt)
        r = gg.query(torch.tensor([0], dtype=torch.int32), c, S, T).cpu().numpy()
        assert abs(float(r[0, 0]) - exact) < 1e-6
    gg.set_tuning(0, 0)
    x = gg.cpi(c, 0, -1, EPS, seed=0).cpu().numpy()
    assert abs(float(x[0]) - exact) < 1e-6


def test_adjoint_on_self_loop_graph(tpa, torch):
    """Every row of A~ is one self-loop, whose softmax weight is 1 for any
    logit: the logit gradient is exactly zero, and the restart gradient is
    (sum over the chains' weights) times the loss weights."""
    n = 50
    gg = no_edge_graph(tpa, n)
    gg.preprocess(c, T)
    W = ti.draw_loss_weights((3, n), 5)
    seeds = torch.tensor([1, 20, 49], dtype=torch.int32)
    dth, dq = gg.backward(torch.from_numpy(W), c, S, T, seeds=seeds)
    assert float(dth.abs().max()) == 0.0
    # dr_TPA[v]/dq[v] = alpha * (1 - (1-c)^S) (the stranger part does not depend on q)
    alpha = (1 - (1 - c) ** T) / (1 - (1 - c) ** S)
    expect = alpha * (1 - (1 - c) ** S) * W
    assert np.abs(dq.cpu().numpy() - expect).max() <= 1e-6


def test_empty_query_batch(tpa, torch):
    gg = tpa.Graph.rmat(8, 2000, 3)
    gg.preprocess(c, T)
    R = gg.query(torch.zeros(0, dtype=torch.int32), c, S, T)
    assert tuple(R.shape) == (0, gg.n)


@pytest.mark.parametrize("kt", [1, 64])
def test_S1_combine_only(tpa, torch, kt):
    og = oracle.Graph.rmat(9, 5000, 8)
    og.preprocess(c, T, EPS)
    gg = tpa.Graph.rmat(9, 5000, 8)
    gg.preprocess(c, T)
    seeds = ti.draw_seeds(og.export()["padded"] == 0, 3, 9)
    gg.set_tuning(seed_tile=kt)
    try:
        R = gg.query(torch.from_numpy(seeds), c, 1, T).cpu().numpy()
    finally:
        gg.set_tuning(0, 0)
    for r, s in zip(R, seeds):
        assert np.abs(r - og.query(int(s), c, 1, T)).sum() <= TOL


@pytest.mark.parametrize("k,kt", [(65, 64), (129, 64), (33, 32), (17, 16), (3, 2)])
def test_ragged_last_tile(tpa, torch, k, kt):
    og = oracle.Graph.rmat(10, 12000, 12)
    og.preprocess(c, T, EPS)
    gg = tpa.Graph.rmat(10, 12000, 12)
    gg.preprocess(c, T)
    seeds = ti.draw_seeds(og.export()["padded"] == 0, k, 13)
    gg.set_tuning(seed_tile=kt)
    try:
        R = gg.query(torch.from_numpy(seeds), c, S, T).cpu().numpy()
    finally:
        gg.set_tuning(0, 0)
    for j in (0, kt - 1, k - 1):
        assert np.abs(R[j] - og.query(int(seeds[j]), c, S, T)).sum() <= TOL
