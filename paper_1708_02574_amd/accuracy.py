"""Accuracy of TPA against exact RWR on the GPU (Section 4's error table and
top-k recall).

For a seed s, the exact parts come from CPI windows (Algorithm 1 with
x(0) = c e_s):

    r_exact     = CPI(0, unbounded)      exact RWR up to the truncation eps
    r_family    = CPI(0, S-1)
    r_neighbor  = CPI(S, T-1)
    r_stranger  = CPI(T, unbounded)

and TPA's approximations are r~_neighbor = scale * r_family (Section 3.2)
and r~_stranger = the preprocessed PageRank tail (Section 3.1).  The L1
errors are compared with the bounds the paper states: 2(1-c)^S - 2(1-c)^T
for the neighbor part (Lemma 3), 2(1-c)^T for the stranger part (Lemma 1)
and 2(1-c)^S for r_TPA (Theorem 2).  Recall@k is |top-k(r_TPA) and
top-k(r_exact)| / k with ties broken by node id.

Every vector and every L1 distance is computed by the library's kernels
(tpa_cpi_batch, tpa_query, tpa_row_l1, tpa_topk); only the set
intersection of the two top-k lists is taken on the host.
"""
from __future__ import annotations

from . import Graph, neighbor_scale, row_l1, topk


def error_bounds(c: float, S: int, T: int) -> dict:
    """The paper's L1 error bounds of the neighbor and stranger
    approximations and of r_TPA."""
    pS, pT = (1.0 - c) ** S, (1.0 - c) ** T
    return {"neighbor": 2 * pS - 2 * pT, "stranger": 2 * pT, "tpa": 2 * pS}


def error_report(g: Graph, seeds, c: float, S: int, T: int, eps: float = 1e-9, ks=(10, 100, 500)) -> list[dict]:
    """Per seed: L1 errors of r~_neighbor, r~_stranger and r_TPA against the
    exact parts, and recall of r_TPA's top-k for each k in ks.  The graph
    must be preprocessed with (c, T).  The exact parts of all seeds are
    computed together (tpa_cpi_batch); r_TPA by one single-seed query each."""
    import torch

    seeds = [int(x) for x in seeds]
    sd = torch.tensor(seeds, dtype=torch.int32, device="cuda")
    scale = neighbor_scale(c, S, T)
    stranger = g.stranger()
    exact = g.cpi_batch(c, 0, -1, eps, seeds=sd)
    st = g.cpi_batch(c, T, -1, eps, seeds=sd)
    r = torch.stack([g.query(sd[i:i + 1], c, S, T)[0] for i in range(len(seeds))])
    nb_err = [0.0] * len(seeds)  # S == T: the neighbor part is empty
    if S < T:
        fam = g.cpi_batch(c, 0, S - 1, eps, seeds=sd)
        nb = g.cpi_batch(c, S, T - 1, eps, seeds=sd)
        nb_err = row_l1(fam, nb, a=scale).cpu().tolist()
    st_err = row_l1(stranger.expand(len(seeds), -1).contiguous(), st).cpu().tolist()
    tpa_err = row_l1(r, exact).cpu().tolist()
    tops = {}
    for k in ks:
        k = min(int(k), g.n)
        ia, _ = topk(r, k)
        ib, _ = topk(exact, k)
        tops[k] = (ia.cpu().tolist(), ib.cpu().tolist())
    out = []
    for i, s in enumerate(seeds):
        rec = {k: len(set(a[i]) & set(b[i])) / k for k, (a, b) in tops.items()}
        out.append({"seed": s, "l1": {"neighbor": float(nb_err[i]), "stranger": float(st_err[i]),
                                      "tpa": float(tpa_err[i])}, "recall": rec})
    return out


def st_sweep(g: Graph, seeds, c: float, pairs, eps: float = 1e-9, reps: int = 3) -> list[dict]:
    """Errors against exact RWR and single-seed query time for each (S, T)
    in pairs: the trade-off the paper discusses when selecting S and T and
    measures in its study of the effects of the parameters (online time and
    L1 error of r_TPA over S at T = 10; L1 errors of the neighbor part, the
    stranger part and r_TPA over T at S = 5).  For each T the graph is
    preprocessed again (the stranger part depends on T).  Each row holds
    the mean and largest L1 error of r_TPA over the seeds, the mean L1
    errors of r~_neighbor and r~_stranger against their exact parts, the
    bound 2(1-c)^S, the best of `reps` timings of one single-seed query per
    seed (microseconds per query) and the preprocessing time.  The graph is
    left preprocessed with the last T of the sweep."""
    import torch

    seeds = [int(x) for x in seeds]
    sd = torch.tensor(seeds, dtype=torch.int32, device="cuda")
    exact = g.cpi_batch(c, 0, -1, eps, seeds=sd)
    out = torch.empty_like(exact)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    rows = []
    for T in sorted({int(t) for _, t in pairs}):
        a, b = ev(), ev()
        a.record()
        g.preprocess(c, T, eps)
        b.record()
        torch.cuda.synchronize()
        pre_ms = a.elapsed_time(b)
        stranger = g.stranger().expand(len(seeds), -1).contiguous()
        st_err = row_l1(stranger, g.cpi_batch(c, T, -1, eps, seeds=sd)).cpu().tolist()
        for S in sorted({int(s) for s, t in pairs if int(t) == T}):
            best = float("inf")
            for _ in range(reps):
                a.record()
                for i in range(len(seeds)):
                    g.query(sd[i:i + 1], c, S, T, out=out[i:i + 1])
                b.record()
                torch.cuda.synchronize()
                best = min(best, a.elapsed_time(b))
            err = row_l1(out, exact).cpu().tolist()
            scale = neighbor_scale(c, S, T)
            nb_err = [0.0] * len(seeds)
            if S < T:
                nb_err = row_l1(g.cpi_batch(c, 0, S - 1, eps, seeds=sd), g.cpi_batch(c, S, T - 1, eps, seeds=sd),
                                a=scale).cpu().tolist()
            rows.append({"S": S, "T": T, "l1_mean": sum(err) / len(err), "l1_max": max(err),
                         "l1_neighbor": sum(nb_err) / len(nb_err), "l1_stranger": sum(st_err) / len(st_err),
                         "bound": 2 * (1.0 - c) ** S, "us_per_query": best * 1e3 / len(seeds),
                         "preprocess_ms": pre_ms})
    return rows


def _main():
    import argparse
    import os
    import sys

    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import tpa_inputs as ti

    ap = argparse.ArgumentParser(description="TPA accuracy vs exact RWR on a synthetic R-MAT graph")
    ap.add_argument("--graph", default="rmat20", choices=sorted(ti.GRAPHS))
    ap.add_argument("--seeds", type=int, default=16)
    args = ap.parse_args()
    scale, samples, gseed = ti.GRAPHS[args.graph]
    g = Graph.rmat(scale, samples, gseed)
    seeds = ti.draw_seeds((g.padded() == 0).cpu().numpy(), args.seeds, 1)
    pairs = [(S, ti.T) for S in range(1, 11)] + [(ti.S, T) for T in (5, 6, 8, 12, 15, 20, 25, 30)]
    print(f"{args.graph}: n={g.n} m={g.m}, {len(seeds)} seeds, c={ti.C}")
    print(f"{'S':>3} {'T':>3} {'L1 TPA':>8} {'max':>8} {'bound':>7} {'L1 nbr':>8} {'L1 str':>8} "
          f"{'us/query':>9} {'prep ms':>8}")
    for r in st_sweep(g, seeds, ti.C, pairs, ti.EPS):
        print(f"{r['S']:3d} {r['T']:3d} {r['l1_mean']:8.4f} {r['l1_max']:8.4f} {r['bound']:7.4f} "
              f"{r['l1_neighbor']:8.4f} {r['l1_stranger']:8.4f} {r['us_per_query']:9.1f} "
              f"{r['preprocess_ms']:8.2f}", flush=True)
    torch.cuda.synchronize()


if __name__ == "__main__":
    _main()
