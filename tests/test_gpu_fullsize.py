"""Full-size parity in the launch configurations bench.py times.

The oracle builds the same R-MAT graphs on the host and computes sampled
seeds one by one; every output is also checked against properties that hold
at any size (mass 1 - (1-c)^(K+1) per seed, non-negativity, plain vs
batched agreement).
"""
import numpy as np
import pytest

import oracle
import tpa_inputs as ti

pytestmark = pytest.mark.gpu

c, S, T, EPS = ti.C, ti.S, ti.T, ti.EPS
TOL = 1e-5
MASS = 1.0 - (1.0 - c) ** 117


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


def l1_rows(a, b):
    return np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)).sum(axis=-1)


def test_rmat20_bench_configuration(tpa, torch):
    """2^20 nodes, 2^24 samples: preprocess, single-seed queries (kt=1) and
    the 1000-seed batched query (kt=64) as bench.py runs them."""
    scale, samples, gseed = ti.GRAPHS["rmat20"]
    print("rmat20: GPU build + preprocess", flush=True)
    gg = tpa.Graph.rmat(scale, samples, gseed)
    gg.preprocess(c, T)
    eligible = (gg.padded() == 0).cpu().numpy()
    seeds = ti.draw_seeds(eligible, 1000, 1)
    sd = torch.from_numpy(seeds).cuda()
    gg.set_tuning(seed_tile=64)
    Rb = gg.query(sd, c, S, T)
    gg.set_tuning(seed_tile=0)
    sample = [0, 1, 2, 500, 999]
    Rp = torch.stack([gg.query(sd[i:i + 1], c, S, T)[0] for i in sample])
    st = gg.stranger().cpu().numpy()
    mass = Rb.sum(dim=1, dtype=torch.float64).cpu().numpy()
    assert np.all(np.abs(mass - MASS) < 1e-5)
    assert float(Rb.min()) >= 0.0
    assert float((Rb[sample] - Rp).abs().max()) < 1e-5
    print("rmat20: oracle build + preprocess", flush=True)
    og = oracle.Graph.rmat(scale, samples, gseed)
    assert og.m == gg.m
    assert np.array_equal(og.export()["padded"], gg.padded().cpu().numpy())
    og.preprocess(c, T, EPS)
    assert l1_rows(st, og.str) <= TOL
    Rp = Rp.cpu().numpy()
    Rbs = Rb[sample].cpu().numpy()
    for r, i in enumerate(sample):
        expect = og.query(int(seeds[i]), c, S, T)
        assert l1_rows(Rp[r], expect) <= TOL
        assert l1_rows(Rbs[r], expect) <= TOL


def test_rmat22_batched_sampled(tpa, torch):
    """2^22 nodes, 2^26 samples, 1024 seeds in one batched call (kt=64)."""
    scale, samples, gseed = ti.GRAPHS["rmat22"]
    print("rmat22: GPU build + preprocess + 1024-seed query", flush=True)
    gg = tpa.Graph.rmat(scale, samples, gseed)
    gg.preprocess(c, T)
    eligible = (gg.padded() == 0).cpu().numpy()
    seeds = ti.draw_seeds(eligible, 1024, 2)
    gg.set_tuning(seed_tile=64)
    R = gg.query(torch.from_numpy(seeds).cuda(), c, S, T)
    gg.set_tuning(seed_tile=0)
    mass = R.sum(dim=1, dtype=torch.float64).cpu().numpy()
    assert np.all(np.abs(mass - MASS) < 1e-5)
    assert float(R.min()) >= 0.0
    sample = [0, 517, 1023]
    Rs = R[sample].cpu().numpy()
    st = gg.stranger().cpu().numpy()
    del R
    print("rmat22: oracle build + preprocess", flush=True)
    og = oracle.Graph.rmat(scale, samples, gseed)
    assert og.m == gg.m
    og.preprocess(c, T, EPS)
    assert l1_rows(st, og.str) <= TOL
    for r, i in enumerate(sample):
        assert l1_rows(Rs[r], og.query(int(seeds[i]), c, S, T)) <= TOL
