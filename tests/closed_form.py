"""Exact TPA values on a structured graph whose A~ has a closed form.

The graph is the union of three parts on consecutive node ids:

* a complete digraph with self-loops on nc nodes (A~ = J / nc on its block:
  every in-row of A~^T averages the block);
* a circulant on L nodes where node i points to i+1 and i+2 (mod L), so
  each node's two in-edges come from i-1 and i-2 with weight 1/2;
* D isolated nodes, which the builder gives self-loops (A~ = I there).

Every node has its out-edges inside its part, so A~ is row-stochastic and
column-stochastic.  Applying A~^T or A~ to a vector costs O(n): a block mean,
two shifts and the identity.  That gives the exact CPI iterates (Section 2.3),
r_family, the PageRank stranger tail (Section 3.1) and the adjoint recursion
in FP64 without any sparse-matrix code, for sizes where no dense matrix (and
no host oracle) fits: with nc = 46341 the block alone has nc^2 =
2,147,488,281 > 2^31 edges.

Edges of A~ in CSR order (rows ascending, columns ascending within a row):
the block row u holds (u, 0..nc-1) at offsets u*nc + v; the circulant row
of node nc+i holds its two successors in ascending node order; each isolated
node holds its self-loop.
"""
from __future__ import annotations

import numpy as np


class Structured:
    def __init__(self, nc: int, L: int, D: int):
        assert nc >= 1 and L >= 3 and D >= 0
        self.nc, self.L, self.D = nc, L, D
        self.n = nc + L + D
        self.m = nc * nc + 2 * L + D
        self.c0, self.i0 = nc, nc + L  # first node of the circulant / isolated part

    # -- edge lists ----------------------------------------------------------
    def circ_succ(self):
        """(src, dst) of the circulant's edges, as node ids (int64)."""
        i = np.arange(self.L)
        src = np.concatenate([i, i]) + self.c0
        dst = np.concatenate([(i + 1) % self.L, (i + 2) % self.L]) + self.c0
        return src, dst

    def a_rowptr(self) -> np.ndarray:
        deg = np.concatenate([np.full(self.nc, self.nc), np.full(self.L, 2), np.ones(self.D, np.int64)])
        return np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)

    def circ_rows_cols(self):
        """CSR columns of the circulant rows (L x 2, ascending per row)."""
        i = np.arange(self.L)
        a, b = (i + 1) % self.L, (i + 2) % self.L
        return np.stack([np.minimum(a, b), np.maximum(a, b)], axis=1) + self.c0

    def edge_index(self, u: np.ndarray, v: np.ndarray) -> np.ndarray:
        """A~ offsets of edges (u, v) of the block or the circulant."""
        u = np.asarray(u, np.int64)
        v = np.asarray(v, np.int64)
        out = np.empty(u.shape, np.int64)
        blk = u < self.nc
        out[blk] = u[blk] * self.nc + v[blk]
        cu = u[~blk] - self.c0
        cols = self.circ_rows_cols()[cu]
        out[~blk] = self.nc * self.nc + 2 * cu + (cols[:, 1] == v[~blk])
        return out

    # -- operators -----------------------------------------------------------
    def At(self, x: np.ndarray) -> np.ndarray:
        """A~^T x (x: [..., n])."""
        y = np.empty_like(x)
        nc, c0, i0 = self.nc, self.c0, self.i0
        y[..., :nc] = x[..., :nc].mean(axis=-1, keepdims=True)
        xc = x[..., c0:i0]
        y[..., c0:i0] = 0.5 * (np.roll(xc, 1, axis=-1) + np.roll(xc, 2, axis=-1))
        y[..., i0:] = x[..., i0:]
        return y

    def A(self, lam: np.ndarray) -> np.ndarray:
        """A~ lam (lam: [..., n])."""
        y = np.empty_like(lam)
        nc, c0, i0 = self.nc, self.c0, self.i0
        y[..., :nc] = lam[..., :nc].mean(axis=-1, keepdims=True)
        lc = lam[..., c0:i0]
        y[..., c0:i0] = 0.5 * (np.roll(lc, -1, axis=-1) + np.roll(lc, -2, axis=-1))
        y[..., i0:] = lam[..., i0:]
        return y

    # -- TPA -----------------------------------------------------------------
    def iterates(self, q: np.ndarray, c: float, count: int) -> list:
        """x(0) = c q, x(i) = (1-c) A~^T x(i-1) for i < count."""
        xs = [c * np.asarray(q, np.float64)]
        for _ in range(1, count):
            xs.append((1 - c) * self.At(xs[-1]))
        return xs

    def family(self, q: np.ndarray, c: float, S: int) -> np.ndarray:
        return sum(self.iterates(q, c, S))

    def stranger(self, c: float, T: int, K: int) -> np.ndarray:
        """sum of x'(i), T <= i <= K, x'(0) = (c/n) 1: A~^T keeps a uniform
        vector uniform, so every entry is ((1-c)^T - (1-c)^(K+1)) / n."""
        return np.full(self.n, ((1 - c) ** T - (1 - c) ** (K + 1)) / self.n)

    def tpa(self, q: np.ndarray, c: float, S: int, T: int, K: int) -> np.ndarray:
        alpha = (1 - (1 - c) ** T) / (1 - (1 - c) ** S)
        return alpha * self.family(q, c, S) + self.stranger(c, T, K)

    # -- adjoint -------------------------------------------------------------
    def backward(self, Q: np.ndarray, W: np.ndarray, c: float, S: int, T: int, K: int):
        """Gradients of L = sum_j <W_j, r_TPA(Q_j)> with weights A~ = softmax
        of zero logits: the restart gradient dQ [k, n] and a function giving
        dL/dtheta at A~ offsets of block and circulant edges.

        Family chain of restart j: lam(S-1) = alpha W_j, lam(i) = alpha W_j +
        (1-c) A~ lam(i+1); dQ_j = c lam(0).  Stranger chain (shared by all
        restarts): mu(K) = sum_j W_j, mu(i) = [i >= T] sum_j W_j + (1-c) A~
        mu(i+1).  Edge term g_uv = (1-c) sum over both chains of
        x(i-1)[u] lam(i)[v]; softmax backward dtheta_uv = A~_uv (g_uv -
        sum_w A~_uw g_uw)."""
        Q = np.atleast_2d(np.asarray(Q, np.float64))
        W = np.atleast_2d(np.asarray(W, np.float64))
        alpha = (1 - (1 - c) ** T) / (1 - (1 - c) ** S)
        X, LAM = [], []  # pairs (x(i-1), lam(i)), i >= 1
        dQ = np.empty_like(Q)
        for j in range(Q.shape[0]):
            xs = self.iterates(Q[j], c, S)
            lam = [None] * S
            lam[S - 1] = alpha * W[j]
            for i in range(S - 2, -1, -1):
                lam[i] = alpha * W[j] + (1 - c) * self.A(lam[i + 1])
            dQ[j] = c * lam[0]
            for i in range(1, S):
                X.append(xs[i - 1])
                LAM.append(lam[i])
        wsum = W.sum(axis=0)
        xs = self.iterates(np.full(self.n, 1.0 / self.n), c, K + 1)
        mu = [None] * (K + 1)
        mu[K] = wsum.copy()
        for i in range(K - 1, -1, -1):
            mu[i] = (wsum if i >= T else 0.0) + (1 - c) * self.A(mu[i + 1])
        for i in range(1, K + 1):
            X.append(xs[i - 1])
            LAM.append(mu[i])
        X = np.stack(X)
        LAM = np.stack(LAM)
        ALAM = self.A(LAM)  # row means sum_w A~_uw lam[w], per pair
        nc, c0 = self.nc, self.c0

        def g(u, v):
            return (1 - c) * np.einsum("pk,pk->k", X[:, u], LAM[:, v])

        def rowmean(u):
            return (1 - c) * np.einsum("pk,pk->k", X[:, u], ALAM[:, u])

        def dtheta(u, v):
            u = np.asarray(u, np.int64)
            v = np.asarray(v, np.int64)
            w = np.where(u < nc, 1.0 / nc, 0.5)
            out = w * (g(u, v) - rowmean(u))
            iso = u >= c0 + self.L
            out[iso] = 0.0
            return out

        return dQ, dtheta

    def edge_list(self, order_seed: int | None = None):
        """(src, dst) of every edge except the isolated nodes' (the builder
        adds those), block edges last; int64 numpy, for small instances."""
        cs, cd = self.circ_succ()
        u = np.repeat(np.arange(self.nc), self.nc)
        v = np.tile(np.arange(self.nc), self.nc)
        src = np.concatenate([cs, u])
        dst = np.concatenate([cd, v])
        if order_seed is not None:
            p = np.random.default_rng(order_seed).permutation(src.size)
            src, dst = src[p], dst[p]
        return src, dst
