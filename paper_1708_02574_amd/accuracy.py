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
(tpa_cpi, tpa_query, tpa_row_l1, tpa_topk); only the set intersection of
the two top-k lists is taken on the host.
"""
from __future__ import annotations

from . import Graph, row_l1, topk


def error_bounds(c: float, S: int, T: int) -> dict:
    """The paper's L1 error bounds of the neighbor and stranger
    approximations and of r_TPA."""
    pS, pT = (1.0 - c) ** S, (1.0 - c) ** T
    return {"neighbor": 2 * pS - 2 * pT, "stranger": 2 * pT, "tpa": 2 * pS}


def error_report(g: Graph, seeds, c: float, S: int, T: int, eps: float = 1e-9, ks=(10, 100, 500)) -> list[dict]:
    """Per seed: L1 errors of r~_neighbor, r~_stranger and r_TPA against the
    exact parts, and recall of r_TPA's top-k for each k in ks.  The graph
    must be preprocessed with (c, T)."""
    import torch

    scale = ((1.0 - c) ** S - (1.0 - c) ** T) / (1.0 - (1.0 - c) ** S)
    stranger = g.stranger()
    out = []
    for s in [int(x) for x in seeds]:
        exact = g.cpi(c, 0, -1, eps, seed=s)
        fam = g.cpi(c, 0, S - 1, eps, seed=s)
        nb = g.cpi(c, S, T - 1, eps, seed=s)
        st = g.cpi(c, T, -1, eps, seed=s)
        r = g.query(torch.tensor([s], dtype=torch.int32, device="cuda"), c, S, T)[0]
        err = {
            "neighbor": float(row_l1(fam, nb, a=scale)[0]),
            "stranger": float(row_l1(stranger, st)[0]),
            "tpa": float(row_l1(r, exact)[0]),
        }
        rec = {}
        for k in ks:
            k = min(int(k), g.n)
            ia, _ = topk(r, k)
            ib, _ = topk(exact, k)
            a = set(ia[0].cpu().tolist())
            b = set(ib[0].cpu().tolist())
            rec[k] = len(a & b) / k
        out.append({"seed": s, "l1": err, "recall": rec})
    return out
