"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the method: it only fixes workload shapes
and draws random inputs (seed nodes, loss weights, edge logits, block sizes)
from numpy's PCG64 with fixed seeds.  Graph edges themselves are drawn by
each side's own counter-based R-MAT generator from the same (scale, samples,
seed) triple, listed here.

The workloads stand in for the paper's evaluation graphs (Table 2: social
and hyperlink graphs with power-law degrees, 0.5M..2.6B edges), which are
not available: R-MAT with (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), directed,
duplicate edges merged, a self-loop on every node without out-edges.
Method constants follow the paper's setup (Section 4.1): c = 0.15,
eps = 1e-9; S = 5, T = 10 as for its Pokec / LiveJournal runs (Table 2).
"""
from __future__ import annotations

import numpy as np

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)
C = 0.15
EPS = 1e-9
S = 5
T = 10

# name -> (scale, samples, rmat seed)
GRAPHS = {
    "rmat13": (13, 1 << 17, 0x5EED0013),   # 2^13 nodes, 2^17 samples (small case)
    "rmat20": (20, 1 << 24, 0x5EED0020),   # 2^20 nodes, 2^24 samples (plain TPA)
    "rmat22": (22, 1 << 26, 0x5EED0022),   # 2^22 nodes, 2^26 samples (batched seeds)
    "rmat27": (27, 1 << 31, 0x5EED0027),   # 2^27 nodes, 2^31 samples (billion edge)
}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def draw_seeds(eligible: np.ndarray, k: int, seed: int) -> np.ndarray:
    """k seed nodes drawn uniformly (with replacement) from the node ids where
    `eligible` is true; int32."""
    ids = np.flatnonzero(np.asarray(eligible))
    if ids.size == 0:
        raise ValueError("no eligible seed node")
    pick = rng(seed).integers(0, ids.size, size=k)
    return ids[pick].astype(np.int32)


def draw_loss_weights(shape, seed: int) -> np.ndarray:
    """w ~ N(0, 1), float32 (the loss L = sum_v w_v r_TPA[v])."""
    return rng(seed).standard_normal(shape).astype(np.float32)


def draw_logits(m: int, seed: int, sigma: float = 0.1) -> np.ndarray:
    """Per-edge logits theta ~ N(0, sigma), float32."""
    return (sigma * rng(seed).standard_normal(m)).astype(np.float32)


def block_sizes(count: int, seed: int, lo_log2: int = 12, hi_log2: int = 18) -> np.ndarray:
    """Node counts log-uniform in [2^lo, 2^hi]: floor(2^(lo + (hi-lo) U))."""
    u = rng(seed).random(count)
    return np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def block_rmat_params(sizes: np.ndarray, seed: int, avg_deg: int = 16):
    """Per-block R-MAT parameters: (scale = ceil(log2 n_g), n_g, accepted
    samples = avg_deg * n_g, rmat seed)."""
    out = []
    for g, ng in enumerate(np.asarray(sizes).tolist()):
        scale = max(1, int(np.ceil(np.log2(ng))))
        out.append((scale, int(ng), int(avg_deg * ng), (seed * 1000003 + g) & 0xFFFFFFFFFFFF))
    return out
