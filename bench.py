"""Benchmark of the TPA hot path on one MI355X.

One step = the plain-TPA job on an R-MAT graph of 2^20 nodes and 2^24
samples (the synthetic stand-in for the paper's social/web graphs):
tpa_preprocess (PageRank stranger part, T = 10, K = 116 CPI steps), then
1000 single-seed tpa_query calls (c = 0.15, S = 5), then the same 1000 seeds
as one batched tpa_query (seed tiles of 64 columns).  The graph, the seeds
and the output buffers are resident in HBM before timing starts.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.  `value` is whole-step throughput in GTEPS: every CPI
step traverses all m edges, so a step counts (K + 2 * 1000 * (S-1)) * m
edge traversals (work unit of the paper's complexity analysis, Section
3.4).  Seeds/s of the plain and batched forms are reported beside it, the
roofline of the dominant kernel from HIP events taken in the timed region,
and the FP64 oracle timed on host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

C_RESTART, S_FAM, T_STR = 0.15, 5, 10
N_SEEDS = 1000
HBM_PEAK_GBS = 8000.0
WORKLOAD = "rmat20"
PROFILE_PERIOD = 16
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_1_family_rmat20_traffic.json")
TRAFFIC_FILE_64 = os.path.join(ROOT, "profiles", "step_kernel_64_family_rmat20_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1708_02574_amd", "csrc", "cpi_kernels.hip")


def kernel_source_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def algorithmic_bytes_family_step(n: int, m: int) -> int:
    """Compulsory HBM bytes of one single-vector family CPI step with
    1/outdeg weights (the dominant kernel): column ids 4m, row offsets of
    the grouped rows 8(n+1), the gathered vector read once 4n, 1/outdeg 4n,
    the next vector written 4n."""
    return 4 * m + 8 * (n + 1) + 12 * n


def algorithmic_bytes_tile_step(n: int, m: int, kt: int = 64) -> int:
    """Compulsory HBM bytes of one family CPI step over a seed tile of kt
    columns (node-major): column ids 4m, row offsets 8(n+1), the gathered
    tile read once 4kt n, 1/outdeg 4n, the next tile written 4kt n."""
    return 4 * m + 8 * (n + 1) + (8 * kt + 4) * n


def traffic_from_profile(path: str = TRAFFIC_FILE):
    """HBM bytes per launch from the committed PMC summary, or None when it
    is missing or was taken on a different version of the kernel source."""
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(scale: int, samples: int, seed: int, seeds, n_queries: int):
    """The FP64 oracle, single-threaded, on a bounded sample of the same
    job: its preprocessing plus `n_queries` single-seed queries."""
    import oracle
    g = oracle.Graph.rmat(scale, samples, seed)
    t0 = time.perf_counter()
    g.preprocess(C_RESTART, T_STR, 1e-9)
    for s in seeds[:n_queries]:
        g.query(int(s), C_RESTART, S_FAM, T_STR)
    dt = time.perf_counter() - t0
    edges = (g.K + n_queries * (S_FAM - 1)) * g.m
    return {
        "value": round(edges / dt / 1e9, 4),
        "unit": "GTEPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{WORKLOAD}: oracle preprocess (K={g.K} steps) + {n_queries} single-seed queries, "
                  f"{dt:.1f} s on one host thread",
        "seconds": round(dt, 3),
    }


def extras(tpa, g, seeds, seeds_h, torch, np) -> dict:
    """Untimed context for the JSON line: TPA's accuracy against exact RWR
    on 4 seeds (the paper's error table and top-k recall, computed by the
    library's kernels), the adjoint's time for 64 seeds, and the times of
    the other device operations: exact RWR of one seed (CPI to eps), top-k
    of one row, and a batch of 64 dense restart vectors."""
    from paper_1708_02574_amd import accuracy
    print("bench: accuracy report and adjoint timing", file=sys.stderr, flush=True)
    rep = accuracy.error_report(g, seeds_h[:4], C_RESTART, S_FAM, T_STR, 1e-9, ks=(10, 100, 500))
    acc = {
        "seeds": len(rep),
        "l1_mean": {p: round(float(np.mean([r["l1"][p] for r in rep])), 5) for p in ("neighbor", "stranger", "tpa")},
        "l1_bound": {p: round(v, 5) for p, v in accuracy.error_bounds(C_RESTART, S_FAM, T_STR).items()},
        "recall_mean": {str(k): round(float(np.mean([r["recall"][k] for r in rep])), 4) for k in (10, 100, 500)},
    }
    ka = 64
    gv = torch.from_numpy(np.random.default_rng(7).standard_normal((ka, g.n)).astype(np.float32)).cuda()
    g.set_tuning(seed_tile=64)
    g.set_keep_iterates(True)  # as the autograd path does: preprocessing keeps the stranger chain
    g.preprocess(C_RESTART, T_STR)
    g.backward(gv, C_RESTART, S_FAM, T_STR, seeds=seeds[:ka])  # warm-up
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    g.backward(gv, C_RESTART, S_FAM, T_STR, seeds=seeds[:ka])
    b.record()
    torch.cuda.synchronize()
    # a second run times every launch of the single-vector adjoint step with
    # the edge gradient (the stranger chain's K steps) on its stream
    tpa.profile_enable(True, 4096, 1)
    tpa.profile_reset()
    g.backward(gv, C_RESTART, S_FAM, T_STR, seeds=seeds[:ka])
    torch.cuda.synchronize()
    adj_launches, adj_kms = tpa.profile_read(tpa.profile_code(1, 3, True, False))
    tpa.profile_enable(False)
    g.set_tuning(seed_tile=0)
    g.set_keep_iterates(False)
    adj_ms = a.elapsed_time(b)
    n, m = g.n, g.m
    # algorithmic bytes of one step: A~'s row offsets and columns, the edge
    # gradient read and written, lambda(i) gathered once, x(i-1), the loss
    # weights, 1/outdeg and lambda(i-1) written
    adj_bytes = 8 * (n + 1) + 4 * m + 8 * m + 4 * n * 5
    adj_us = adj_kms * 1e3 / adj_launches if adj_launches else None
    adj_roof = None
    if adj_us:
        achieved = adj_bytes / (adj_us * 1e-6) / 1e9
        adj_roof = {"kernel": "adj_kernel_1<1/outdeg, edge gradient> (stranger-chain adjoint step)", "bound": "hbm",
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": adj_bytes,
                    "avg_launch_us": round(adj_us, 2), "launches_timed": adj_launches}
    s0 = int(seeds_h[0])
    exact_ms = _time_ms(torch, lambda: g.cpi(C_RESTART, 0, -1, 1e-9, seed=s0))
    exact64_ms = _time_ms(torch, lambda: g.cpi_batch(C_RESTART, 0, -1, 1e-9, seeds=seeds[:64]), reps=2)
    row = g.cpi(C_RESTART, 0, -1, 1e-9, seed=s0)
    topk_ms = _time_ms(torch, lambda: tpa.topk(row, 100))
    qd = torch.from_numpy(np.random.default_rng(8).random((64, g.n)).astype(np.float32)).cuda()
    qd /= qd.sum(dim=1, keepdim=True)
    outd = torch.empty_like(qd)
    g.query_dense(qd, C_RESTART, S_FAM, T_STR, out=outd)  # warm-up
    dense_ms = _time_ms(torch, lambda: g.query_dense(qd, C_RESTART, S_FAM, T_STR, out=outd))
    return {"accuracy": acc,
            "adjoint": {"seeds": ka, "ms": round(adj_ms, 3),
                        "note": "gradients w.r.t. edge logits and restart vectors (both CPI chains, 64-seed tile; "
                                "the stranger chain's iterates kept by preprocessing)",
                        "roofline": adj_roof},
            "ops_ms": {"exact_rwr_one_seed": round(exact_ms, 3), "exact_rwr_64_seeds": round(exact64_ms, 3),
                       "topk_k100_one_row": round(topk_ms, 3),
                       "dense_restart_64": round(dense_ms, 3),
                       "note": "exact RWR = CPI from x(0) = c e_s until c(1-c)^i < 1e-9 (tpa_cpi, synchronous; "
                               "64 seeds at once: tpa_cpi_batch, one seed tile of 64); "
                               "top-k of one n-entry row (tpa_topk); TPA for 64 dense restart vectors "
                               "(tpa_query_dense, automatic seed tile: 64)"}}


def _time_ms(torch, fn, reps=3):
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def other_configs(tpa, torch, np) -> dict:
    """The other workloads on the same GPU (best of 3 after a warm-up, inputs
    resident): 1024 seeds on 2^22 nodes with the autotuner's choice replayed
    from a hipGraph; the uneven batch of 256 R-MAT graphs (4 seeds each,
    logit weights) forward and adjoint; the 2^27-node, 2^31-sample graph's
    preprocessing, 16-seed query and 4-seed adjoint."""
    import tpa_inputs as ti
    res = {}
    # 2^22 nodes, 1024 seeds, autotuned, captured
    print("bench: rmat22 batched (autotune + capture)", file=sys.stderr, flush=True)
    scale, samples, gseed = ti.GRAPHS["rmat22"]
    g = tpa.Graph.rmat(scale, samples, gseed)
    g.preprocess(C_RESTART, T_STR)
    sd = torch.from_numpy(ti.draw_seeds((g.padded() == 0).cpu().numpy(), 1024, 2)).cuda()
    out = torch.empty((1024, g.n), dtype=torch.float32, device="cuda")
    tile, ew, _ = g.autotune(sd, C_RESTART, S_FAM, T_STR, scratch_out=out)
    g.reserve(1024)
    qg = g.capture_query(C_RESTART, S_FAM, T_STR, out, seeds=sd)
    qg.launch()
    torch.cuda.synchronize()
    ms = _time_ms(torch, qg.launch)
    qg.close()
    res["rmat22_batched"] = {"n": g.n, "m": g.m, "seeds": 1024, "seed_tile": tile, "edges_per_item": ew,
                             "captured_ms": round(ms, 3), "seeds_per_s": round(1024 / (ms * 1e-3), 1),
                             "gteps": round(1024 * (S_FAM - 1) * g.m / (ms * 1e-3) / 1e9, 1)}
    del g, out, qg
    torch.cuda.empty_cache()
    # uneven 256-graph batch with logits: forward and adjoint
    print("bench: uneven 256-graph batch", file=sys.stderr, flush=True)
    sizes = ti.block_sizes(256, 2024)
    gs = [tpa.Graph.rmat(sc, smp, s_, n_nodes=ng) for sc, ng, smp, s_ in ti.block_rmat_params(sizes, 2024)]
    pk = tpa.Graph.pack(gs)
    del gs
    off = pk.block_offsets()
    pk.set_logits(torch.from_numpy(ti.draw_logits(pk.m, 2025)).cuda())
    pk.preprocess(C_RESTART, T_STR)  # builds the gather layout once
    t_pre = _time_ms(torch, lambda: pk.preprocess(C_RESTART, T_STR), reps=1)
    padded = pk.padded().cpu().numpy()
    seeds = np.stack([off[b] + ti.draw_seeds(padded[off[b]:off[b + 1]] == 0, 4, 3000 + b)
                      for b in range(256)]).astype(np.int32)
    sdp = torch.from_numpy(seeds).cuda()
    W = torch.from_numpy(ti.draw_loss_weights((4, pk.n), 2026)).cuda()
    pk.query_packed(sdp, C_RESTART, S_FAM, T_STR)
    fwd = _time_ms(torch, lambda: pk.query_packed(sdp, C_RESTART, S_FAM, T_STR))
    pk.backward(W, C_RESTART, S_FAM, T_STR, seeds=sdp, packed=True)
    bwd_re = _time_ms(torch, lambda: pk.backward(W, C_RESTART, S_FAM, T_STR, seeds=sdp, packed=True), reps=2)
    pk.set_keep_iterates(True)  # as the autograd path does
    pk.preprocess(C_RESTART, T_STR)
    bwd = _time_ms(torch, lambda: pk.backward(W, C_RESTART, S_FAM, T_STR, seeds=sdp, packed=True), reps=2)
    pk.set_keep_iterates(False)
    res["uneven_batch"] = {"graphs": 256, "N": pk.n, "m": pk.m, "seeds_per_graph": 4,
                           "preprocess_ms": round(t_pre, 3), "query_ms": round(fwd, 3),
                           "backward_ms": round(bwd, 3), "backward_recomputing_ms": round(bwd_re, 3)}
    del pk, W, sdp
    torch.cuda.empty_cache()
    # billion-edge graph
    print("bench: rmat27 (2^31 samples)", file=sys.stderr, flush=True)
    scale, samples, gseed = ti.GRAPHS["rmat27"]
    g = tpa.Graph.rmat(scale, samples, gseed)
    g.preprocess(C_RESTART, T_STR)
    t_pre = _time_ms(torch, lambda: g.preprocess(C_RESTART, T_STR), reps=1)
    sd = torch.from_numpy(ti.draw_seeds((g.padded() == 0).cpu().numpy(), 16, 27)).cuda()
    g.set_tuning(seed_tile=16)
    out = torch.empty((16, g.n), dtype=torch.float32, device="cuda")
    g.query(sd, C_RESTART, S_FAM, T_STR, out=out)
    q16 = _time_ms(torch, lambda: g.query(sd, C_RESTART, S_FAM, T_STR, out=out), reps=2)
    g.set_tuning(0, 0)
    W = torch.from_numpy(ti.draw_loss_weights((4, g.n), 28)).cuda()
    bwd = _time_ms(torch, lambda: g.backward(W, C_RESTART, S_FAM, T_STR, seeds=sd[:4]), reps=1)
    res["rmat27"] = {"n": g.n, "m": g.m, "preprocess_ms": round(t_pre, 1),
                     "preprocess_gteps": round(116 * g.m / (t_pre * 1e-3) / 1e9, 1),
                     "query16_ms": round(q16, 2), "backward4_ms": round(bwd, 1)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seeds", type=int, default=N_SEEDS)
    ap.add_argument("--cpu-queries", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the untimed accuracy report and adjoint timing")
    ap.add_argument("--all-configs", action="store_true",
                    help="also time the other workloads (untimed in the step): 2^22-node batched query with "
                         "autotune and hipGraph capture, the uneven 256-graph batch with its adjoint, and the "
                         "billion-edge graph")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="after timing, run one device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the seed and block axes would shard with no communication; see DESIGN.md).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1708_02574_amd as tpa
    import tpa_inputs as ti

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    scale, samples, gseed = ti.GRAPHS[WORKLOAD]
    print(f"bench: building {WORKLOAD} (scale {scale}, {samples} samples)", file=sys.stderr, flush=True)
    g = tpa.Graph.rmat(scale, samples, gseed)
    n, m = g.n, g.m
    eligible = (g.padded() == 0).cpu().numpy()
    seeds_h = ti.draw_seeds(eligible, args.seeds, 1)
    seeds = torch.from_numpy(seeds_h).cuda()
    k = seeds.numel()
    out_plain = torch.empty((k, n), dtype=torch.float32, device="cuda")
    out_batch = torch.empty((k, n), dtype=torch.float32, device="cuda")
    g.preprocess(C_RESTART, T_STR)
    g.set_tuning(seed_tile=64)
    g.reserve(k)
    g.set_tuning(seed_tile=0)
    torch.cuda.synchronize()

    def step():
        g.set_tuning(seed_tile=0)
        g.preprocess(C_RESTART, T_STR)
        e1.record()
        for i in range(k):
            g.query(seeds[i:i + 1], C_RESTART, S_FAM, T_STR, out=out_plain[i:i + 1])
        e2.record()
        g.set_tuning(seed_tile=64)
        g.query(seeds, C_RESTART, S_FAM, T_STR, out=out_batch)
        g.set_tuning(seed_tile=0)

    ev = lambda: torch.cuda.Event(enable_timing=True)
    e0, e1, e2, e3 = ev(), ev(), ev(), ev()
    for _ in range(args.warmup):
        e0.record()
        step()
        e3.record()
    torch.cuda.synchronize()

    # HIP events bracket one in PERIOD launches of each step-kernel variant
    # in the timed region (the dominant kernel's average launch duration)
    tpa.profile_enable(True, 65536, PROFILE_PERIOD)
    tpa.profile_reset()
    t_pre = t_plain = t_batch = 0.0
    torch.cuda.synchronize()
    start, stop = ev(), ev()
    start.record()
    for _ in range(args.steps):
        e0.record()
        step()
        e3.record()
        torch.cuda.synchronize()
        t_pre += e0.elapsed_time(e1)
        t_plain += e1.elapsed_time(e2)
        t_batch += e2.elapsed_time(e3)
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    ms_step = total_ms / args.steps
    code = tpa.profile_code(1, 0, False, False)
    launches, kms = tpa.profile_read(code)
    launches64, kms64 = tpa.profile_read(tpa.profile_code(64, 0, False, False))
    tpa.profile_enable(False)

    # sanity: every r_TPA has mass 1 - (1-c)^(K+1) (Lemma 2 + closed-form K)
    mass = out_plain.double().sum(dim=1)
    mass_b = out_batch.double().sum(dim=1)
    expect = 1.0 - (1.0 - C_RESTART) ** 117
    mass_err = float(max((mass - expect).abs().max().item(), (mass_b - expect).abs().max().item()))
    max_diff = float((out_plain - out_batch).abs().max().item())

    K = 116
    edges_step = (K + 2 * k * (S_FAM - 1)) * m
    t_pre /= args.steps
    t_plain /= args.steps
    t_batch /= args.steps
    avg_launch_ms = kms / max(launches, 1)
    alg = algorithmic_bytes_family_step(n, m)
    achieved = alg / (avg_launch_ms * 1e-3) / 1e9
    traffic = traffic_from_profile(TRAFFIC_FILE)
    avg64_ms = kms64 / max(launches64, 1)
    alg64 = algorithmic_bytes_tile_step(n, m)
    achieved64 = alg64 / (avg64_ms * 1e-3) / 1e9 if launches64 else 0.0
    traffic64 = traffic_from_profile(TRAFFIC_FILE_64)

    rec = {
        "metric": "TPA query GTEPS & seeds/s, batched vs 1-seed, at L1 <=1e-5 vs FP64 oracle",
        "value": round(edges_step / (ms_step * 1e-3) / 1e9, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{WORKLOAD}: R-MAT (0.57,0.19,0.19,0.05) 2^{scale} nodes, 2^{int(np.log2(samples))} samples, "
                        f"deduped + dangling self-loops; tpa_preprocess + {k} single-seed tpa_query + "
                        f"{k}-seed batched tpa_query (kt=64)",
            "n": n, "m": m, "seeds": k, "c": C_RESTART, "S": S_FAM, "T": T_STR, "K": K,
            "parallelism": "single GPU",
        },
        "seeds_per_s": {"plain": round(k / (t_plain * 1e-3), 1), "batched": round(k / (t_batch * 1e-3), 1)},
        "gteps": {
            "plain": round(k * (S_FAM - 1) * m / (t_plain * 1e-3) / 1e9, 2),
            "batched": round(k * (S_FAM - 1) * m / (t_batch * 1e-3) / 1e9, 2),
            "preprocess": round(K * m / (t_pre * 1e-3) / 1e9, 2),
        },
        "ms": {"preprocess": round(t_pre, 3), "plain_1000": round(t_plain, 3), "batched_1000": round(t_batch, 3)},
        "roofline": {
            "kernel": "step_kernel_1<family, non-first, 1/outdeg> (single-seed CPI step)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg,
            "avg_launch_us": round(avg_launch_ms * 1e3, 2),
            "launches_timed": launches,
        },
        "roofline_batched": {
            "kernel": "step_kernel_64<family, non-first, 1/outdeg> (64-seed tile CPI step)",
            "bound": "hbm",
            "achieved": round(achieved64, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved64 / HBM_PEAK_GBS, 4),
            "traffic": traffic64,
            "traffic_GBps": round(traffic64 / (avg64_ms * 1e-3) / 1e9, 1) if traffic64 and launches64 else None,
            "algorithmic_bytes_per_launch": alg64,
            "avg_launch_us": round(avg64_ms * 1e3, 2),
            "launches_timed": launches64,
        },
        "checks": {"mass_max_err": mass_err, "plain_vs_batched_max_abs": max_diff},
    }
    if not args.no_extras:
        rec.update(extras(tpa, g, seeds, seeds_h, torch, np))
    if args.all_configs:
        del out_plain, out_batch, g
        torch.cuda.empty_cache()
        rec["configs"] = other_configs(tpa, torch, np)
    if args.calibration_copy_mib > 0:
        src = torch.empty(args.calibration_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(scale, samples, gseed, seeds_h, args.cpu_queries)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
