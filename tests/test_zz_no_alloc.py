"""tpa_query_noalloc (the query whose workspace is the library's fixed device
array) against tpa_query and the oracle, through the C ABI.

Two calls in a row on different graphs, the second with a smaller input,
then a third back on the first graph: the fixed workspace keeps the previous
call's contents, so each result must still equal tpa_query's bit for bit
(the same kernels in the same order) and the oracle within L1 <= 1e-5 per
seed.  The error paths (no schedule for the seed tile yet, a workspace above
the array's size) leave the handle usable.
"""
import ctypes

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


def noalloc(tpa, torch, g, seeds, out):
    """The raw C entry point (argument marshalling only)."""
    lib = tpa.load_library()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib.tpa_query_noalloc(g._h, ctypes.c_void_p(seeds.data_ptr()), seeds.numel(), c, S, T,
                                 ctypes.c_void_p(out.data_ptr()), st)


def check(tpa, torch, og, g, seeds_h):
    seeds = torch.from_numpy(seeds_h).cuda()
    k = seeds.numel()
    out = torch.full((k, g.n), float("nan"), dtype=torch.float32, device="cuda")
    print(f"no-alloc: n={g.n} k={k}", flush=True)
    assert noalloc(tpa, torch, g, seeds, out) == 0, tpa.load_library().tpa_last_error_message()
    ref = g.query(seeds, c, S, T)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    got = out.cpu().numpy().astype(np.float64)
    for j, s in enumerate(seeds_h):
        assert np.abs(got[j] - og.query(int(s), c, S, T)).sum() <= TOL, (j, s)
    g.device_error()


def test_noalloc_matches_query_on_consecutive_calls(tpa, torch):
    scale, samples, gseed = ti.GRAPHS["rmat13"]
    ogA = oracle.Graph.rmat(scale, samples, gseed)
    ogA.preprocess(c, T, EPS)
    gA = tpa.Graph.rmat(scale, samples, gseed)
    gA.preprocess(c, T)
    ogB = oracle.Graph.rmat(10, 12000, 4711)
    ogB.preprocess(c, T, EPS)
    gB = tpa.Graph.rmat(10, 12000, 4711)
    gB.preprocess(c, T)
    seedsA = ti.draw_seeds(ogA.export()["padded"] == 0, 16, 61)
    seedsB = ti.draw_seeds(ogB.export()["padded"] == 0, 1, 62)
    gA.reserve(16)  # the 16-column schedule (building it allocates)
    check(tpa, torch, ogA, gA, seedsA)            # first call: 16 seeds on 8192 nodes
    check(tpa, torch, ogB, gB, seedsB)            # second, smaller: one seed on 1024 nodes
    check(tpa, torch, ogA, gA, seedsA[:1])        # back on the larger graph, one seed
    check(tpa, torch, ogA, gA, seedsA)


def test_noalloc_error_paths(tpa, torch):
    lib = tpa.load_library()
    g = tpa.Graph.rmat(10, 12000, 4711)
    g.preprocess(c, T)
    seeds = torch.from_numpy(ti.draw_seeds(np.ones(g.n, bool), 64, 63)).cuda()
    out = torch.empty((64, g.n), dtype=torch.float32, device="cuda")
    g.set_tuning(seed_tile=64)
    try:
        # no 64-column schedule yet: refused, nothing built
        assert noalloc(tpa, torch, g, seeds, out) == -1
        assert b"tpa_reserve" in lib.tpa_last_error_message()
        g.reserve(64)
        assert noalloc(tpa, torch, g, seeds, out) == 0
        assert torch.equal(out, g.query(seeds, c, S, T))
    finally:
        g.set_tuning(0, 0)
    # 5M isolated nodes (self-loops): one seed needs about 16 bytes per node
    big = tpa.Graph.from_edges(5_000_000, np.zeros(0, np.int32), np.zeros(0, np.int32))
    big.preprocess(c, T)
    one = torch.tensor([123], dtype=torch.int32, device="cuda")
    o1 = torch.empty((1, big.n), dtype=torch.float32, device="cuda")
    assert noalloc(tpa, torch, big, one, o1) == -1
    assert b"holds at most" in lib.tpa_last_error_message()
    # the handle stays usable
    r = big.query(one, c, S, T)[0]
    alpha = (1 - (1 - c) ** T) / (1 - (1 - c) ** S)
    assert abs(float(r[123]) - (alpha * (1 - (1 - c) ** S) + ((1 - c) ** T - (1 - c) ** 117) / big.n)) < 1e-6


def test_noalloc_with_pushed_steps(tpa, torch):
    """With the third step's push forced on a small graph (its frontier list
    lives in the fixed array too) and a seed tile whose second step may be
    pushed, tpa_query_noalloc still equals tpa_query bit for bit and the
    oracle within L1 <= 1e-5, on consecutive calls."""
    scale, samples, gseed = ti.GRAPHS["rmat13"]
    og = oracle.Graph.rmat(scale, samples, gseed)
    og.preprocess(c, T, EPS)
    g = tpa.Graph.rmat(scale, samples, gseed)
    g.preprocess(c, T)
    g.set_push_limit(og.m)
    g.set_third_push_limit(og.m)
    try:
        g.reserve(16)
        seeds = ti.draw_seeds(og.export()["padded"] == 0, 16, 64)
        for sd in (seeds[:1], seeds, seeds[3:4]):
            check(tpa, torch, og, g, sd)
    finally:
        g.set_third_push_limit(-1)
        g.set_push_limit(-1)
