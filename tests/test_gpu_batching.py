"""Batching machinery on the GPU: captured (HIP graph) queries replayed with
new seeds, and the autotuner's parity-checked choice."""
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


@pytest.mark.parametrize("k,kt", [(1, 1), (100, 64), (37, 8)])
def test_captured_query_replays(rmat13, torch, k, kt):
    og, gg = rmat13
    eligible = og.export()["padded"] == 0
    gg.set_tuning(seed_tile=kt)
    try:
        seeds_buf = torch.from_numpy(ti.draw_seeds(eligible, k, 100)).cuda()
        out = torch.empty((k, gg.n), dtype=torch.float32, device="cuda")
        qg = gg.capture_query(c, S, T, out, seeds=seeds_buf)
        for rep in range(3):
            new = torch.from_numpy(ti.draw_seeds(eligible, k, 200 + rep)).cuda()
            seeds_buf.copy_(new)
            qg.launch()
            torch.cuda.synchronize()
            scratch = torch.randn(1000, device="cuda").sum()  # eager work between replays
            torch.cuda.synchronize()
            eager = gg.query(new, c, S, T)
            torch.cuda.synchronize()
            assert torch.equal(out, eager), rep
            assert float(scratch) == float(scratch)
        qg.close()
    finally:
        gg.set_tuning(0, 0)


def test_captured_query_with_pushed_steps(rmat13, torch):
    """A captured single-seed query whose third step may be pushed (limit
    forced on this small graph) and a captured 16-seed tile whose second
    step may be pushed: replays with new seeds, eager work in between, equal
    bit for bit to eager queries, whichever direction the device takes."""
    og, gg = rmat13
    eligible = og.export()["padded"] == 0
    gg.set_push_limit(og.m)
    gg.set_third_push_limit(og.m)
    try:
        for k in (1, 16):
            seeds_buf = torch.from_numpy(ti.draw_seeds(eligible, k, 300 + k)).cuda()
            out = torch.empty((k, gg.n), dtype=torch.float32, device="cuda")
            qg = gg.capture_query(c, S, T, out, seeds=seeds_buf)
            for rep in range(3):
                new = torch.from_numpy(ti.draw_seeds(eligible, k, 400 + 10 * k + rep)).cuda()
                seeds_buf.copy_(new)
                qg.launch()
                torch.cuda.synchronize()
                scratch = torch.randn(1000, device="cuda").sum()
                torch.cuda.synchronize()
                eager = gg.query(new, c, S, T)
                torch.cuda.synchronize()
                assert torch.equal(out, eager), (k, rep)
                assert float(scratch) == float(scratch)
            qg.close()
    finally:
        gg.set_third_push_limit(-1)
        gg.set_push_limit(-1)


def test_captured_dense_and_packed(tpa, torch):
    params = [(9, 4000, 1, 400), (10, 9000, 2, 0)]
    ggs = []
    for scale, samples, seed, nn in params:
        ggs.append(tpa.Graph.rmat(scale, samples, seed, n_nodes=nn or (1 << scale)))
    pk = tpa.Graph.pack(ggs)
    pk.preprocess(c, T)
    off = pk.block_offsets()
    seeds = torch.tensor([[off[0] + 3, off[0] + 9], [off[1] + 1, off[1] + 500]], dtype=torch.int32).cuda()
    out = torch.empty((2, pk.n), dtype=torch.float32, device="cuda")
    qg = pk.capture_query(c, S, T, out, seeds=seeds, packed=True)
    for rep in range(2):
        qg.launch()
        torch.cuda.synchronize()
        assert torch.equal(out, pk.query_packed(seeds, c, S, T))
    q = torch.rand((3, pk.n), device="cuda")
    q /= q.sum(dim=1, keepdim=True)
    outq = torch.empty((3, pk.n), dtype=torch.float32, device="cuda")
    qd = pk.capture_query(c, S, T, outq, q=q)
    for rep in range(2):
        q.copy_(torch.rand((3, pk.n), device="cuda"))
        qd.launch()
        torch.cuda.synchronize()
        assert torch.equal(outq, pk.query_dense(q, c, S, T))


def test_autotune_choice_passes_parity(rmat13, torch):
    og, gg = rmat13
    seeds = ti.draw_seeds(og.export()["padded"] == 0, 200, 5)
    tile, ew, ms = gg.autotune(torch.from_numpy(seeds), c, S, T)
    assert tile in (8, 16, 32, 64) and ew in (128, 256, 512) and ms > 0
    assert gg.get_tuning() == (tile, ew)
    R = gg.query(torch.from_numpy(seeds).cuda(), c, S, T).cpu().numpy()
    gg.set_tuning(0, 0)
    for i in (0, 57, 199):
        assert l1_rows(R[i], og.query(int(seeds[i]), c, S, T)) <= TOL


def test_workspace_size_and_reserve(rmat13, torch):
    """tpa_query_workspace_size reports the bytes tpa_reserve holds; it grows
    with the batch (seed tiles of 1, 8 and 64) and covers dense restarts."""
    og, gg = rmat13
    gg.set_tuning(0, 0)  # automatic tiles (an earlier test may have autotuned the handle)
    sizes = [gg.workspace_size(k) for k in (1, 8, 100)]
    assert 0 < sizes[0] < sizes[1] < sizes[2]
    gg.reserve(100)
    seeds = torch.from_numpy(ti.draw_seeds(og.export()["padded"] == 0, 100, 5)).cuda()
    R = gg.query(seeds, c, S, T)
    assert bool(torch.isfinite(R).all())


def test_query_graph_keeps_group_order_copy(rmat13, torch):
    """A single-seed query graph captured under layout 2 reads the
    group-ordered column ids.  Switching to layout 1 afterwards keeps them
    allocated, so the replays still give the same bits, and switching back
    reuses the same copy (the handle's device bytes do not change)."""
    og, gg = rmat13
    seeds = torch.from_numpy(ti.draw_seeds(og.export()["padded"] == 0, 1, 48)).cuda()
    gg.set_gather_layout(2)
    ref = gg.query(seeds, c, S, T)
    held = gg.device_bytes()
    out = torch.empty_like(ref)
    qg = gg.capture_query(c, S, T, out, seeds=seeds)
    try:
        gg.set_gather_layout(1)
        assert gg.device_bytes() == held
        for _ in range(3):
            out.fill_(-1.0)
            qg.launch()
            torch.cuda.synchronize()
            assert torch.equal(out, ref)
            assert torch.equal(gg.query(seeds, c, S, T), ref)
        gg.set_gather_layout(2)
        assert gg.device_bytes() == held
        qg.launch()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        assert torch.equal(gg.query(seeds, c, S, T), ref)
    finally:
        qg.close()
        gg.set_gather_layout(2)
