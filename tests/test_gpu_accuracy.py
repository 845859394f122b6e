"""Exact RWR (CPI windows), top-k selection and the accuracy harness on the
GPU against the FP64 oracle.

* tpa_cpi vs oracle.Graph.cpi on every window the harness uses, seeds and
  dense restarts, uniform and logit weights: L1 <= 1e-5.
* tpa_topk vs oracle.topk on the same float32 rows: identical indices and
  values (the comparison is exact, so both sides decide in FP32).
* the harness's per-part errors vs the same errors from oracle vectors, and
  under the paper's bounds.
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


def l1(a, b):
    return float(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)).sum())


WINDOWS = [(0, -1), (0, S - 1), (S, T - 1), (T, -1), (0, 0), (3, 3), (7, 200)]


@pytest.mark.parametrize("layout", [2, 1, 0])
def test_cpi_windows_seed(rmat13, torch, layout):
    og, gg = rmat13
    gg.set_gather_layout(layout)
    try:
        for s in ti.draw_seeds(og.export()["padded"] == 0, 4, 61):
            q = np.zeros(og.n)
            q[s] = 1.0
            for si, tj in WINDOWS:
                r = gg.cpi(c, si, tj, EPS, seed=int(s)).cpu().numpy()
                expect, _ = og.cpi(q, c, EPS, si, tj)
                assert l1(r, expect) <= TOL, (s, si, tj)
    finally:
        gg.set_gather_layout(True)


def test_cpi_dense_restart_and_weights(tpa, torch):
    og = oracle.Graph.rmat(10, 12000, 41)
    gg = tpa.Graph.rmat(10, 12000, 41)
    theta = ti.draw_logits(og.m, 42)
    og.set_logits(theta.astype(np.float64))
    gg.set_logits(torch.from_numpy(theta).cuda())
    rng = np.random.default_rng(43)
    q = rng.random(og.n)
    q /= q.sum()
    for si, tj in WINDOWS:
        r = gg.cpi(c, si, tj, EPS, q=torch.from_numpy(q.astype(np.float32))).cpu().numpy()
        expect, _ = og.cpi(q, c, EPS, si, tj)
        assert l1(r, expect) <= TOL, (si, tj)
    # exact RWR of a restart vector with norm 1/2: the break comes earlier
    r = gg.cpi(c, 0, -1, EPS, q=torch.from_numpy((q / 2).astype(np.float32))).cpu().numpy()
    expect, _ = og.cpi(q / 2, c, EPS, 0, -1)
    assert l1(r, expect) <= TOL


def test_cpi_windows_add_up_to_exact_rwr(rmat13, torch):
    """The three exact parts add up to exact RWR: CPI(0, S-1) + CPI(S, T-1)
    + CPI(T, inf) = CPI(0, inf) (the split of Section 3), whose mass is
    1 - (1-c)^(K+1) (Lemma 2)."""
    og, gg = rmat13
    s = int(ti.draw_seeds(og.export()["padded"] == 0, 1, 62)[0])
    parts = [gg.cpi(c, a, b, EPS, seed=s) for a, b in ((0, S - 1), (S, T - 1), (T, -1))]
    whole = gg.cpi(c, 0, -1, EPS, seed=s)
    assert l1((parts[0] + parts[1] + parts[2]).cpu().numpy(), whole.cpu().numpy()) <= 1e-6
    mass = float(whole.double().sum())
    assert abs(mass - (1 - (1 - c) ** 117)) < 1e-6


def test_cpi_argument_errors(rmat13, tpa, torch):
    og, gg = rmat13
    for kw in ({"seed": og.n}, {"seed": 0, "s_iter": 3, "t_iter": 2}, {"seed": 0, "eps": 0.0},
               {"seed": 0, "s_iter": -1}):
        si = kw.pop("s_iter", 0)
        tj = kw.pop("t_iter", -1)
        eps = kw.pop("eps", EPS)
        with pytest.raises(tpa.TPAError):
            gg.cpi(c, si, tj, eps, **kw)
    with pytest.raises(ValueError):
        gg.cpi(c, 0, -1, EPS)


@pytest.mark.parametrize("k", [1, 5, 70])
def test_cpi_batch_seeds_vs_oracle(rmat13, torch, k):
    """Batched CPI windows (seed tiles of 1, 8 and 64 with a ragged last
    tile) against the oracle's CPI of each seed."""
    og, gg = rmat13
    seeds = ti.draw_seeds(og.export()["padded"] == 0, k, 67)
    sd = torch.from_numpy(seeds).cuda()
    rows = sorted({0, k // 2, k - 1})
    for si, tj in WINDOWS:
        R = gg.cpi_batch(c, si, tj, EPS, seeds=sd).cpu().numpy()
        for j in rows:
            q = np.zeros(og.n)
            q[seeds[j]] = 1.0
            expect, _ = og.cpi(q, c, EPS, si, tj)
            assert l1(R[j], expect) <= TOL, (k, j, si, tj)


def test_cpi_batch_dense_per_row_break(tpa, torch):
    """Dense restarts with different norms stop at their own last
    iteration (Lemma 2's c (1-c)^i ||q||_1 < eps per row), on node and hub
    layouts, matching the single-restart tpa_cpi and the oracle."""
    og = oracle.Graph.rmat(10, 12000, 71)
    gg = tpa.Graph.rmat(10, 12000, 71)
    rng = np.random.default_rng(72)
    q = rng.random((4, og.n))
    q /= q.sum(axis=1, keepdims=True)
    q[1] *= 0.5
    q[2] *= 3.0
    q[3] = 0.0
    q[3, 5] = 1e-3
    for layout in (2, 1, 0):
        gg.set_gather_layout(layout)
        for si, tj in ((0, -1), (2, 9), (10, -1)):
            R = gg.cpi_batch(c, si, tj, EPS, q=torch.from_numpy(q.astype(np.float32))).cpu().numpy()
            for j in range(4):
                expect, _ = og.cpi(q[j], c, EPS, si, tj)
                assert l1(R[j], expect) <= TOL * max(1.0, q[j].sum()), (layout, j, si, tj)
                single = gg.cpi(c, si, tj, EPS, q=torch.from_numpy(q[j].astype(np.float32))).cpu().numpy()
                assert l1(R[j], single) <= 1e-6 * max(1.0, q[j].sum()), (layout, j, si, tj)
    gg.set_gather_layout(True)


def test_cpi_batch_bad_seed_and_arguments(rmat13, tpa, torch):
    og, gg = rmat13
    gg.device_error()  # nothing pending
    seeds = torch.tensor([3, og.n, 7], dtype=torch.int32).cuda()
    R = gg.cpi_batch(c, 0, -1, EPS, seeds=seeds).cpu().numpy()
    assert np.isnan(R[1]).all() and np.isfinite(R[0]).all() and np.isfinite(R[2]).all()
    with pytest.raises(tpa.TPAError):
        gg.device_error()
    gg.device_error()  # cleared
    q = np.zeros(og.n)
    q[7] = 1.0
    assert l1(R[2], og.cpi(q, c, EPS, 0, -1)[0]) <= TOL
    empty = gg.cpi_batch(c, 0, -1, EPS, seeds=torch.zeros(0, dtype=torch.int32).cuda())
    assert tuple(empty.shape) == (0, og.n)
    with pytest.raises(tpa.TPAError):
        gg.cpi_batch(c, 3, 2, EPS, seeds=seeds[:1])
    with pytest.raises(tpa.TPAError):
        gg.cpi_batch(c, 0, -1, 0.0, seeds=seeds[:1])
    with pytest.raises(ValueError):
        gg.cpi_batch(c, 0, -1, EPS)


@pytest.mark.parametrize("rows,n,k", [(1, 1, 1), (3, 9, 4), (5, 300, 7), (2, 300, 300), (4, 5000, 64),
                                      (2, 70000, 1024), (3, 1024, 1024), (1, 100000, 1),
                                      (2, 49252, 1024), (1, 300000, 1024), (2, 300000, 10)])
def test_topk_vs_oracle(tpa, torch, rows, n, k):
    rng = np.random.default_rng(rows * 1000 + n + k)
    pool = np.array([0.5, 0.25, 0.0, -0.0, 1e-7, np.nan, 3.0, -2.0, np.inf], np.float32)
    vals = np.where(rng.random((rows, n)) < 0.5, rng.choice(pool, (rows, n)),
                    rng.standard_normal((rows, n)).astype(np.float32))
    idx, val = tpa.topk(torch.from_numpy(vals), k)
    oi, ov = oracle.topk(vals, k)
    assert np.array_equal(idx.cpu().numpy(), oi)
    assert np.array_equal(val.cpu().numpy(), ov, equal_nan=True)


@pytest.mark.parametrize("n,k", [(70000, 1000), (300000, 1024), (5000, 17)])
def test_topk_ties_keep_index_order_across_stages(tpa, torch, n, k):
    """Rows larger than one segment are reduced in stages; among equal
    values the smaller indices must survive every stage: a constant row
    gives indices 0..k-1, and a row of one value with a few larger ones
    gives those first, then the smallest remaining indices."""
    const = np.full((1, n), 0.5, np.float32)
    idx, val = tpa.topk(torch.from_numpy(const), k)
    assert np.array_equal(idx.cpu().numpy()[0], np.arange(k))
    assert np.all(val.cpu().numpy() == np.float32(0.5))
    x = np.full((1, n), 0.25, np.float32)
    big = np.array([n - 1, n // 2, 7], np.int64)
    x[0, big] = [3.0, 2.0, 1.0]
    idx, _ = tpa.topk(torch.from_numpy(x), k)
    bigset = set(big.tolist())
    rest = [i for i in range(k) if i not in bigset][:k - 3]
    assert np.array_equal(idx.cpu().numpy()[0], np.concatenate([big, rest]))


def test_topk_on_rwr_rows(rmat13, tpa, torch):
    og, gg = rmat13
    seeds = torch.from_numpy(ti.draw_seeds(og.export()["padded"] == 0, 16, 63)).cuda()
    R = gg.query(seeds, c, S, T)
    for k in (1, 10, 500, 1024):
        idx, val = tpa.topk(R, k)
        oi, ov = oracle.topk(R.cpu().numpy(), k)
        assert np.array_equal(idx.cpu().numpy(), oi), k
        assert np.array_equal(val.cpu().numpy(), ov), k


def test_topk_argument_errors(tpa, torch):
    x = torch.zeros((2, 10), device="cuda")
    for k in (0, 11, 1025):
        with pytest.raises(tpa.TPAError):
            tpa.topk(x, k)


def test_row_l1_vs_numpy(tpa, torch):
    rng = np.random.default_rng(64)
    x = rng.standard_normal((3, 4097)).astype(np.float32)
    y = rng.standard_normal((3, 4097)).astype(np.float32)
    got = tpa.row_l1(torch.from_numpy(x), torch.from_numpy(y), a=0.75).cpu().numpy()
    expect = np.abs(0.75 * x.astype(np.float64) - y.astype(np.float64)).sum(axis=1)
    assert np.allclose(got, expect, rtol=1e-12, atol=0)


def test_error_report_vs_oracle(rmat13, tpa, torch):
    """The harness on rmat13: per-part L1 errors agree with the same errors
    from oracle vectors and stay under the paper's bounds; recall values
    equal those computed by the oracle's top-k on the GPU vectors."""
    from paper_1708_02574_amd import accuracy
    og, gg = rmat13
    seeds = ti.draw_seeds(og.export()["padded"] == 0, 5, 65)
    rep = accuracy.error_report(gg, seeds, c, S, T, EPS, ks=(10, 100))
    exact_all = gg.cpi_batch(c, 0, -1, EPS, seeds=torch.from_numpy(seeds).cuda()).cpu().numpy()
    bounds = accuracy.error_bounds(c, S, T)
    assert abs(bounds["tpa"] - 2 * (1 - c) ** S) < 1e-15
    scale = oracle.neighbor_scale(c, S, T)
    for row, s in zip(rep, seeds):
        q = np.zeros(og.n)
        q[s] = 1.0
        exact, _ = og.cpi(q, c, EPS, 0, -1)
        fam, _ = og.cpi(q, c, EPS, 0, S - 1)
        nb, _ = og.cpi(q, c, EPS, S, T - 1)
        st, _ = og.cpi(q, c, EPS, T, -1)
        expect = {"neighbor": l1(scale * fam, nb), "stranger": l1(og.str, st),
                  "tpa": l1(og.query(int(s), c, S, T), exact)}
        for part in ("neighbor", "stranger", "tpa"):
            assert abs(row["l1"][part] - expect[part]) <= 3 * TOL, (s, part)
            assert row["l1"][part] <= bounds[part] + 1e-6, (s, part)
        for k, rec in row["recall"].items():
            assert 0.0 <= rec <= 1.0
        r = gg.query(torch.tensor([int(s)], dtype=torch.int32).cuda(), c, S, T)[0].cpu().numpy()
        ex = exact_all[list(seeds).index(s)]
        for k in (10, 100):
            a = set(oracle.topk(r, k)[0][0].tolist())
            b = set(oracle.topk(ex, k)[0][0].tolist())
            assert row["recall"][k] == len(a & b) / k


def test_st_sweep_agrees_with_error_report(tpa, torch):
    """The S/T sweep's per-(S, T) errors equal the harness's per-seed
    errors at the same parameters and respect the bound 2(1-c)^S."""
    from paper_1708_02574_amd import accuracy
    scale, samples, seed = ti.GRAPHS["rmat13"]
    gg = tpa.Graph.rmat(scale, samples, seed)
    seeds = ti.draw_seeds((gg.padded() == 0).cpu().numpy(), 3, 66)
    pairs = [(1, 10), (3, 10), (5, 10), (5, 5), (5, 20)]
    rows = accuracy.st_sweep(gg, seeds, c, pairs, EPS, reps=1)
    assert [(r["S"], r["T"]) for r in rows] == [(5, 5), (1, 10), (3, 10), (5, 10), (5, 20)]
    for r in rows:
        gg.preprocess(c, r["T"], EPS)
        rep = accuracy.error_report(gg, seeds, c, r["S"], r["T"], EPS, ks=(10,))
        assert abs(r["l1_mean"] - np.mean([x["l1"]["tpa"] for x in rep])) <= 1e-9
        assert abs(r["l1_stranger"] - np.mean([x["l1"]["stranger"] for x in rep])) <= 1e-9
        nb = np.mean([x["l1"]["neighbor"] for x in rep]) if r["S"] < r["T"] else 0.0
        assert abs(r["l1_neighbor"] - nb) <= 1e-9
        assert r["l1_max"] <= r["bound"] + 1e-6
        assert r["us_per_query"] > 0 and r["preprocess_ms"] > 0
