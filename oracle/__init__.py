"""FP64 CPU oracle of the TPA hot path -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import this package.  The product library never loads it and shares no code
with it.

Everything here is a thin ctypes wrapper around tpa_oracle.c (plain,
single-threaded C in double precision).  What each function follows and
what pins it (tests/test_oracle.py):

* ``rmat``            R-MAT sampling with a SplitMix64 counter hash (input
                      generator, not paper arithmetic).  Pinned by quadrant
                      statistics and bit decomposition; the hash constants are
                      those of the published SplitMix64.
* ``Graph``           dedupe + dangling self-loops + CSR of A~ and A~^T.
                      Pinned by brute force (Python sets) on small graphs and
                      structural invariants (row sums of A~ are 1).
* ``cpi``             Algorithm 1 (Section 2.3).  Pinned by a dense linear
                      solve (Theorem 1), closed-form graphs, the per-iterate
                      norms of Lemma 2 and brute-force dense matrix powers.
* ``preprocess``      Algorithm 2 (Section 3.1).  Pinned by dense PageRank
                      minus its first T terms, and K = 116 at (c, eps) =
                      (0.15, 1e-9) from the L1 break.
* ``query``           Algorithm 3 + the neighbor scale (Section 3.2, Lemma 2).
                      Pinned by dense brute force, closed-form graphs, the
                      Table 3 bound values, and Lemma 1 / Lemma 3 / Theorem 2
                      against exact CPI.
* ``topk``            the k largest entries per row, ties by smaller index
                      (the ranking whose recall Section 4 reports).  Pinned
                      by the properties that define it uniquely: order,
                      domination of every unselected entry, smallest indices
                      among ties at the cut.
* ``backward``        reverse-mode derivative of the online + preprocessing
                      chains w.r.t. edge logits and the restart vector (an
                      extension, not in the paper).  Pinned by central finite
                      differences of the oracle forward pass.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None

_i64 = C.c_int64
_u64 = C.c_uint64
_dbl = C.c_double
_vp = C.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "tpa_oracle.c"))
    ):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    lib.orc_splitmix64.restype = _u64
    lib.orc_splitmix64.argtypes = [_u64, _u64]
    lib.orc_rmat.restype = _i64
    lib.orc_rmat.argtypes = [C.c_int, _i64, _i64, _u64, _dbl, _dbl, _dbl, _i64, _vp, _vp, _vp]
    lib.orc_graph_build.restype = _vp
    lib.orc_graph_build.argtypes = [_i64, _i64, _vp, _vp]
    lib.orc_graph_free.restype = None
    lib.orc_graph_free.argtypes = [_vp]
    lib.orc_graph_n.restype = _i64
    lib.orc_graph_n.argtypes = [_vp]
    lib.orc_graph_m.restype = _i64
    lib.orc_graph_m.argtypes = [_vp]
    lib.orc_graph_export.restype = None
    lib.orc_graph_export.argtypes = [_vp] * 8
    lib.orc_graph_set_logits.restype = None
    lib.orc_graph_set_logits.argtypes = [_vp, _vp]
    lib.orc_cpi.restype = _i64
    lib.orc_cpi.argtypes = [_vp, _vp, _dbl, _dbl, _i64, _i64, _vp]
    lib.orc_preprocess.restype = _i64
    lib.orc_preprocess.argtypes = [_vp, _dbl, _i64, _dbl, _vp]
    lib.orc_neighbor_scale.restype = _dbl
    lib.orc_neighbor_scale.argtypes = [_dbl, _i64, _i64]
    lib.orc_query_q.restype = C.c_int
    lib.orc_query_q.argtypes = [_vp, _vp, _dbl, _i64, _i64, _dbl, _vp, _vp, _vp]
    lib.orc_query.restype = C.c_int
    lib.orc_query.argtypes = [_vp, _i64, _dbl, _i64, _i64, _dbl, _vp, _vp]
    lib.orc_chain_adjoint.restype = C.c_int
    lib.orc_chain_adjoint.argtypes = [_vp, _vp, _i64, _dbl, _vp, _vp, _vp, _vp]
    lib.orc_backward_q.restype = C.c_int
    lib.orc_backward_q.argtypes = [_vp, _vp, _dbl, _i64, _i64, _i64, _vp, C.c_int, C.c_int, _vp, _vp]
    lib.orc_softmax_backward.restype = None
    lib.orc_softmax_backward.argtypes = [_vp, _vp, _vp]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_vp)


def splitmix64(seed: int, j: int) -> int:
    return int(_load().orc_splitmix64(seed & 0xFFFFFFFFFFFFFFFF, j))


def rmat(scale: int, samples: int, seed: int, n_nodes: int | None = None,
         abcd=(0.57, 0.19, 0.19, 0.05), max_raw: int | None = None):
    """Accepted R-MAT samples (src, dst) as int32 arrays, and the raw count."""
    lib = _load()
    n_nodes = (1 << scale) if n_nodes is None else int(n_nodes)
    max_raw = (samples if n_nodes == (1 << scale) else 64 * samples + 1024) if max_raw is None else max_raw
    src = np.empty(samples, np.int32)
    dst = np.empty(samples, np.int32)
    raw = np.zeros(1, np.int64)
    got = lib.orc_rmat(scale, n_nodes, samples, seed & 0xFFFFFFFFFFFFFFFF,
                       abcd[0], abcd[1], abcd[2], max_raw, _p(src), _p(dst), _p(raw))
    return src[:got].copy(), dst[:got].copy(), int(raw[0])


def topk(vals, k: int):
    """Indices and values of the k largest entries of each row of vals
    ([rows, n] or [n]), ordered by value descending then index ascending;
    NaN ranks below every number, -0 equals +0.  Values are compared in the
    dtype given (float32 results stay float32)."""
    v = np.atleast_2d(np.asarray(vals))
    rows, n = v.shape
    idx = np.arange(n)
    out_i = np.empty((rows, k), np.int64)
    for r in range(rows):
        row = v[r]
        nan = np.isnan(row)
        key = np.where(nan, 0, -row.astype(np.float64))  # -x: ascending sort = descending value
        order = np.lexsort((idx, key, nan))
        out_i[r] = order[:k]
    return out_i, np.take_along_axis(v, out_i, axis=1)


def neighbor_scale(c: float, S: int, T: int) -> float:
    return float(_load().orc_neighbor_scale(c, S, T))


class Graph:
    """Oracle graph: A~ by rows (out-edges) and A~^T by rows (in-edges)."""

    def __init__(self, n: int, src, dst):
        lib = _load()
        src = np.ascontiguousarray(src, np.int32)
        dst = np.ascontiguousarray(dst, np.int32)
        if src.shape != dst.shape:
            raise ValueError("src/dst length mismatch")
        h = lib.orc_graph_build(int(n), int(src.size), _p(src), _p(dst))
        if not h:
            raise ValueError("oracle graph build failed (bad node id or out of memory)")
        self._h = h
        self.n = int(lib.orc_graph_n(h))
        self.m = int(lib.orc_graph_m(h))
        self.K = None

    @classmethod
    def rmat(cls, scale: int, samples: int, seed: int, n_nodes: int | None = None):
        n = (1 << scale) if n_nodes is None else n_nodes
        s, d, _ = rmat(scale, samples, seed, n_nodes=n)
        return cls(n, s, d)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_graph_free(h)
            self._h = None

    def export(self) -> dict:
        n, m = self.n, self.m
        out = dict(
            a_rowptr=np.empty(n + 1, np.int64), a_col=np.empty(m, np.int32),
            a_w=np.empty(m, np.float64), t_rowptr=np.empty(n + 1, np.int64),
            t_col=np.empty(m, np.int32), t2a=np.empty(m, np.int64),
            padded=np.empty(n, np.uint8))
        _lib.orc_graph_export(self._h, *[_p(out[k]) for k in (
            "a_rowptr", "a_col", "a_w", "t_rowptr", "t_col", "t2a", "padded")])
        return out

    def set_logits(self, theta):
        if theta is None:
            _lib.orc_graph_set_logits(self._h, None)
        else:
            th = np.ascontiguousarray(theta, np.float64)
            if th.size != self.m:
                raise ValueError("theta must have one entry per edge")
            _lib.orc_graph_set_logits(self._h, _p(th))

    def dense_At(self) -> np.ndarray:
        """Dense A~^T (n x n) for small graphs (pins only)."""
        e = self.export()
        A = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(e["a_rowptr"]))
        A[rows, e["a_col"]] = e["a_w"]
        return A.T.copy()

    # -- Algorithm 1 -------------------------------------------------------
    def cpi(self, q, c: float, eps: float, s_iter: int, t_iter: int):
        q = np.ascontiguousarray(q, np.float64)
        r = np.empty(self.n, np.float64)
        last = _lib.orc_cpi(self._h, _p(q), c, eps, s_iter, t_iter, _p(r))
        if last < 0:
            raise MemoryError("oracle cpi")
        return r, int(last)

    # -- Algorithm 2 -------------------------------------------------------
    def preprocess(self, c: float, T: int, eps: float = 1e-9) -> np.ndarray:
        s = np.empty(self.n, np.float64)
        K = _lib.orc_preprocess(self._h, c, T, eps, _p(s))
        if K < 0:
            raise MemoryError("oracle preprocess")
        self.K = int(K)
        self.c, self.T, self.str = c, T, s
        return s

    # -- Algorithm 3 -------------------------------------------------------
    def query(self, seed: int, c: float, S: int, T: int, str_vec=None, eps: float = 1e-9):
        str_vec = self.str if str_vec is None else np.ascontiguousarray(str_vec, np.float64)
        out = np.empty(self.n, np.float64)
        rc = _lib.orc_query(self._h, int(seed), c, S, T, eps, _p(str_vec), _p(out))
        if rc:
            raise ValueError(f"oracle query failed ({rc})")
        return out

    def query_q(self, q, c: float, S: int, T: int, str_vec=None, eps: float = 1e-9,
                return_family: bool = False):
        str_vec = self.str if str_vec is None else np.ascontiguousarray(str_vec, np.float64)
        q = np.ascontiguousarray(q, np.float64)
        out = np.empty(self.n, np.float64)
        fam = np.empty(self.n, np.float64)
        rc = _lib.orc_query_q(self._h, _p(q), c, S, T, eps, _p(str_vec), _p(out), _p(fam))
        if rc:
            raise ValueError(f"oracle query failed ({rc})")
        return (out, fam) if return_family else out

    # -- adjoint -------------------------------------------------------------
    def backward(self, qs, gvs, c: float, S: int, T: int, K: int):
        """Gradients of L = sum_j <gvs[j], r_TPA(qs[j])> w.r.t. the edge logits
        (A~ order) and each restart vector.  Returns (dtheta, dA, dq)."""
        qs = np.atleast_2d(np.asarray(qs, np.float64))
        gvs = np.atleast_2d(np.asarray(gvs, np.float64))
        dA = np.zeros(self.m, np.float64)
        dq = np.zeros_like(qs)
        for j in range(qs.shape[0]):
            q = np.ascontiguousarray(qs[j])
            g = np.ascontiguousarray(gvs[j])
            row = np.empty(self.n, np.float64)
            rc = _lib.orc_backward_q(self._h, _p(q), c, S, T, K, _p(g), 1, 0, _p(dA), _p(row))
            if rc:
                raise MemoryError("oracle backward")
            dq[j] = row
        gsum = np.ascontiguousarray(gvs.sum(axis=0))
        zero = np.zeros(self.n, np.float64)
        rc = _lib.orc_backward_q(self._h, _p(zero), c, S, T, K, _p(gsum), 0, 1, _p(dA), None)
        if rc:
            raise MemoryError("oracle backward")
        dtheta = np.empty(self.m, np.float64)
        _lib.orc_softmax_backward(self._h, _p(dA), _p(dtheta))
        return dtheta, dA, dq

    def tpa_forward(self, qs, c: float, S: int, T: int, eps: float = 1e-9):
        """r_TPA for each restart vector in qs with the stranger recomputed
        from the current weights (used by finite differences)."""
        s = np.empty(self.n, np.float64)
        K = _lib.orc_preprocess(self._h, c, T, eps, _p(s))
        qs = np.atleast_2d(np.asarray(qs, np.float64))
        return np.stack([self.query_q(q, c, S, T, str_vec=s, eps=eps) for q in qs]), int(K)
