"""Python binding of libtpa (include/tpa.h): TPA's hot path on MI355X.

Argument marshalling only.  Every step of graph construction, preprocessing
and querying runs in the HIP kernels of libtpa.so; torch provides device
memory (tensors) and the current HIP stream.  There is no CPU fallback: if
the library is missing or no HIP device is present, calls raise.

The raw C entry points are exposed under their C names (``tpa_query`` ...)
taking plain integers / pointers; ``Graph`` wraps them for torch tensors.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtpa.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "tpa.h")

TPA_OK = 0
STATUS = {
    0: "TPA_OK", -1: "TPA_ERR_INVALID_ARG", -2: "TPA_ERR_NOT_PREPROCESSED",
    -3: "TPA_ERR_PARAM_MISMATCH", -4: "TPA_ERR_OUT_OF_MEMORY", -5: "TPA_ERR_HIP",
    -6: "TPA_ERR_INDEX_OVERFLOW", -7: "TPA_ERR_CAPTURE",
}

_i = C.c_int
_i64 = C.c_int64
_u64 = C.c_uint64
_d = C.c_double
_vp = C.c_void_p

# name -> (restype, argtypes); mirrors include/tpa.h
_SIGS = {
    "tpa_graph_rmat": (_i, [_i, _i64, _i64, _u64, _d, _d, _d, _vp, _vp]),
    "tpa_graph_from_edges": (_i, [_i64, _i64, _vp, _vp, _i, _vp, _vp]),
    "tpa_graph_pack": (_i, [_vp, _i, _vp, _vp]),
    "tpa_graph_destroy": (_i, [_vp]),
    "tpa_graph_info": (_i, [_vp, _vp, _vp, _vp]),
    "tpa_graph_blocks": (_i, [_vp, _vp]),
    "tpa_graph_version": (_i, [_vp, _vp]),
    "tpa_neighbor_scale": (_i, [_d, _i, _i, _vp]),
    "tpa_graph_device_bytes": (_i, [_vp, _vp]),
    "tpa_graph_export": (_i, [_vp, _i, _vp, _vp, _vp, _vp]),
    "tpa_graph_padded": (_i, [_vp, _vp, _vp]),
    "tpa_graph_set_logits": (_i, [_vp, _vp, _vp]),
    "tpa_preprocess": (_i, [_vp, _d, _i, _vp]),
    "tpa_preprocess_ex": (_i, [_vp, _d, _i, _d, _vp]),
    "tpa_stranger": (_i, [_vp, _vp, _vp]),
    "tpa_preprocess_info": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "tpa_query": (_i, [_vp, _vp, _i64, _d, _i, _i, _vp, _vp]),
    "tpa_query_noalloc": (_i, [_vp, _vp, _i64, _d, _i, _i, _vp, _vp]),
    "tpa_query_packed": (_i, [_vp, _vp, _i, _d, _i, _i, _vp, _vp]),
    "tpa_query_dense": (_i, [_vp, _vp, _i64, _d, _i, _i, _vp, _vp]),
    "tpa_backward": (_i, [_vp, _vp, _vp, _i64, _i, _d, _i, _i, _vp, _vp, _vp, _i, _vp]),
    "tpa_query_graph_create": (_i, [_vp, _vp, _vp, _i64, _i, _d, _i, _i, _vp, _vp, _vp]),
    "tpa_query_graph_launch": (_i, [_vp, _vp]),
    "tpa_query_graph_destroy": (_i, [_vp]),
    "tpa_autotune": (_i, [_vp, _vp, _i64, _d, _i, _i, _vp, _vp, _vp, _vp, _vp]),
    "tpa_reserve": (_i, [_vp, _i64]),
    "tpa_query_workspace_size": (_i, [_vp, _i64, _vp]),
    "tpa_set_tuning": (_i, [_vp, _i, _i]),
    "tpa_get_tuning": (_i, [_vp, _vp, _vp]),
    "tpa_set_push_limit": (_i, [_vp, _i64]),
    "tpa_set_keep_iterates": (_i, [_vp, _i]),
    "tpa_set_gather_layout": (_i, [_vp, _i]),
    "tpa_get_gather_layout": (_i, [_vp, _vp]),
    "tpa_set_sliced_sweep": (_i, [_vp, _i]),
    "tpa_get_sliced_sweep": (_i, [_vp, _vp, _vp]),
    "tpa_get_push_limit": (_i, [_vp, _vp]),
    "tpa_set_tile_push_limit": (_i, [_vp, _i64]),
    "tpa_get_tile_push_limit": (_i, [_vp, _vp]),
    "tpa_set_third_push_limit": (_i, [_vp, _i64]),
    "tpa_get_third_push_limit": (_i, [_vp, _vp]),
    "tpa_get_device_error": (_i, [_vp, _vp]),
    "tpa_cpi": (_i, [_vp, C.c_int32, _vp, _d, _i, _i, _d, _vp, _vp]),
    "tpa_cpi_batch": (_i, [_vp, _vp, _vp, _i64, _d, _i, _i, _d, _vp, _vp]),
    "tpa_topk": (_i, [_vp, _i64, _i64, _i, _vp, _vp, _vp]),
    "tpa_row_l1": (_i, [_vp, _vp, _i64, _i64, _d, _vp, _vp]),
    "tpa_profile_enable": (_i, [_i, _i, _i]),
    "tpa_profile_read": (_i, [_i, _vp, _vp]),
    "tpa_profile_reset": (_i, []),
    "tpa_status_string": (C.c_char_p, [_i]),
    "tpa_last_error_message": (C.c_char_p, []),
}

_lib = None


class TPAError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


def load_library():
    """Load libtpa.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1708_02574_amd.build")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def header_symbols() -> list[str]:
    """Names of the functions declared in include/tpa.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tpa_[a-z_]+)\s*\(", txt)))


def _check(status: int, where: str):
    if status != TPA_OK:
        msg = _lib.tpa_last_error_message().decode(errors="replace")
        raise TPAError(status, where, msg)


def _call(name: str, *args):
    lib = load_library()
    _check(getattr(lib, name)(*args), name)


# raw entry points under their C names -------------------------------------
def __getattr__(name):
    if name in _SIGS:
        return getattr(load_library(), name)
    raise AttributeError(name)


# --------------------------------------------------------------- torch glue
def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libtpa needs a HIP device (torch.cuda.is_available() is False)")
    return torch


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return _vp(s.cuda_stream)


def _ptr(t):
    return _vp(t.data_ptr())


def neighbor_scale(c: float, S: int, T: int) -> float:
    """The closed-form neighbor scale of Section 3.2 (tpa_neighbor_scale)."""
    v = C.c_double()
    _call("tpa_neighbor_scale", c, S, T, C.byref(v))
    return v.value


def profile_code(kt: int, mode: int, first: bool, weighted: bool, last: bool = False) -> int:
    """Variant code of a CPI step kernel for tpa_profile_read (the last
    family step of a single seed and of tiles of 16 and 64 has its own)."""
    if last and mode == 0 and kt in (1, 16, 64):
        return 112 + 2 * {1: 0, 16: 1, 64: 2}[kt] + int(weighted)
    return 16 * (int(kt).bit_length() - 1) + 4 * mode + 2 * int(first) + int(weighted)


def profile_enable(enable: bool = True, capacity: int = 65536, sample_period: int = 1):
    _call("tpa_profile_enable", int(enable), capacity, sample_period)


def profile_reset():
    _call("tpa_profile_reset")


def profile_read(code: int):
    """(launches, total milliseconds) recorded for a kernel variant."""
    n, ms = C.c_int64(), C.c_double()
    _call("tpa_profile_read", code, C.byref(n), C.byref(ms))
    return n.value, ms.value


class Graph:
    """Owning wrapper of a tpa_graph_t (device CSR of A~ and A~^T)."""

    def __init__(self, handle: int, _keep=()):
        self._h = _vp(handle)
        self._keep = _keep
        n, m, nb = C.c_int64(), C.c_int64(), C.c_int64()
        _call("tpa_graph_info", self._h, C.byref(n), C.byref(m), C.byref(nb))
        self.n, self.m, self.nblocks = n.value, m.value, nb.value

    # -- constructors ------------------------------------------------------
    @classmethod
    def rmat(cls, scale: int, samples: int, seed: int, n_nodes: int = 0,
             abcd=(0.57, 0.19, 0.19, 0.05), stream=None) -> "Graph":
        _torch()
        h = _vp()
        _call("tpa_graph_rmat", scale, n_nodes, samples, seed & 0xFFFFFFFFFFFFFFFF,
              abcd[0], abcd[1], abcd[2], _stream(stream), C.byref(h))
        return cls(h.value)

    @classmethod
    def from_edges(cls, n: int, src, dst, stream=None) -> "Graph":
        torch = _torch()
        if isinstance(src, torch.Tensor) and src.is_cuda:
            s = src.to(torch.int32).contiguous()
            d = dst.to(torch.int32).contiguous()
            dev = 1
            ps, pd = _ptr(s), _ptr(d)
            m = s.numel()
        else:
            s = np.ascontiguousarray(np.asarray(src), np.int32)
            d = np.ascontiguousarray(np.asarray(dst), np.int32)
            dev = 0
            ps, pd = s.ctypes.data_as(_vp), d.ctypes.data_as(_vp)
            m = s.size
        if (d.numel() if dev else d.size) != m:
            raise ValueError("src and dst differ in length")
        h = _vp()
        _call("tpa_graph_from_edges", n, m, ps, pd, dev, _stream(stream), C.byref(h))
        return cls(h.value)

    @classmethod
    def pack(cls, graphs, stream=None) -> "Graph":
        _torch()
        arr = (_vp * len(graphs))(*[g._h.value for g in graphs])
        h = _vp()
        _call("tpa_graph_pack", arr, len(graphs), _stream(stream), C.byref(h))
        return cls(h.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().tpa_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- accessors ---------------------------------------------------------
    def block_offsets(self) -> np.ndarray:
        out = np.empty(self.nblocks + 1, np.int64)
        _call("tpa_graph_blocks", self._h, out.ctypes.data_as(_vp))
        return out

    def version(self) -> int:
        """Counter of the weights / preprocessed state (tpa_graph_version)."""
        v = C.c_uint64()
        _call("tpa_graph_version", self._h, C.byref(v))
        return v.value

    def export(self, transpose: bool = False, col: bool = True, weights: bool = True, stream=None):
        """(row_ptr, col, w) of A~ (or A~^T); col / w are None when not asked for."""
        torch = _torch()
        rp = torch.empty(self.n + 1, dtype=torch.int64, device="cuda")
        cl = torch.empty(self.m, dtype=torch.int32, device="cuda") if col else None
        w = torch.empty(self.m, dtype=torch.float32, device="cuda") if weights else None
        _call("tpa_graph_export", self._h, int(transpose), _ptr(rp), _ptr(cl) if cl is not None else None,
              _ptr(w) if w is not None else None, _stream(stream))
        return rp, cl, w

    def padded(self, stream=None):
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.uint8, device="cuda")
        _call("tpa_graph_padded", self._h, _ptr(out), _stream(stream))
        return out

    def set_logits(self, theta=None, stream=None):
        if theta is None:
            _call("tpa_graph_set_logits", self._h, None, _stream(stream))
            return
        th = theta.to(dtype=_torch().float32).contiguous()
        if th.numel() != self.m or not th.is_cuda:
            raise ValueError("theta must be a device tensor with one entry per edge")
        _call("tpa_graph_set_logits", self._h, _ptr(th), _stream(stream))

    # -- TPA ---------------------------------------------------------------
    def preprocess(self, c: float, T: int, eps: float | None = None, stream=None):
        if eps is None:
            _call("tpa_preprocess", self._h, c, T, _stream(stream))
        else:
            _call("tpa_preprocess_ex", self._h, c, T, eps, _stream(stream))

    def preprocess_info(self) -> dict:
        """c, T, eps and K (the stranger chain's last iteration) of the last
        preprocessing (tpa_preprocess_info)."""
        cc, tt, ee, kk = C.c_double(), C.c_int(), C.c_double(), C.c_int64()
        _call("tpa_preprocess_info", self._h, C.byref(cc), C.byref(tt), C.byref(ee), C.byref(kk))
        return {"c": cc.value, "T": tt.value, "eps": ee.value, "K": kk.value}

    def stranger(self, stream=None):
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.float32, device="cuda")
        _call("tpa_stranger", self._h, _ptr(out), _stream(stream))
        return out

    def query(self, seeds, c: float, S: int, T: int, out=None, stream=None):
        """r_TPA for each seed: float32 [k, n] on the device."""
        torch = _torch()
        sd = seeds.to(device="cuda", dtype=torch.int32).contiguous()
        k = sd.numel()
        if out is None:
            out = torch.empty((k, self.n), dtype=torch.float32, device="cuda")
        elif out.shape != (k, self.n) or out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 [k, n] device tensor")
        _call("tpa_query", self._h, _ptr(sd), k, c, S, T, _ptr(out), _stream(stream))
        return out

    def query_noalloc(self, seeds, c: float, S: int, T: int, out, stream=None):
        """tpa_query_noalloc: r_TPA for each seed into out [k, n] with the
        library's fixed workspace (no device allocation in the call)."""
        torch = _torch()
        if seeds.dtype != torch.int32 or not seeds.is_cuda or not seeds.is_contiguous():
            raise ValueError("seeds must be a contiguous int32 device tensor")
        k = seeds.numel()
        if out.shape != (k, self.n) or out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 [k, n] device tensor")
        _call("tpa_query_noalloc", self._h, _ptr(seeds), k, c, S, T, _ptr(out), _stream(stream))
        return out

    def query_packed(self, seeds, c: float, S: int, T: int, out=None, stream=None):
        """seeds: int [nblocks, P] (node ids of each block); returns [P, n]."""
        torch = _torch()
        sd = seeds.to(device="cuda", dtype=torch.int32).contiguous()
        if sd.dim() != 2 or sd.shape[0] != self.nblocks:
            raise ValueError("seeds must be [nblocks, per_block]")
        P = sd.shape[1]
        if out is None:
            out = torch.empty((P, self.n), dtype=torch.float32, device="cuda")
        _call("tpa_query_packed", self._h, _ptr(sd), P, c, S, T, _ptr(out), _stream(stream))
        return out

    def cpi(self, c: float, s_iter: int, t_iter: int = -1, eps: float = 1e-9, seed: int | None = None,
            q=None, out=None, stream=None):
        """Algorithm 1 for one restart (a seed, or a dense q [n]): the sum of
        x(i) over s_iter <= i <= t_iter (t_iter = -1: until ||x(i)||_1 < eps).
        cpi(c, 0) is exact RWR up to the truncation.  Returns float32 [n]."""
        torch = _torch()
        if (seed is None) == (q is None):
            raise ValueError("pass exactly one of seed and q")
        qd = None
        if q is not None:
            qd = q.to(device="cuda", dtype=torch.float32).contiguous()
            if qd.shape != (self.n,):
                raise ValueError("q must be [n]")
        if out is None:
            out = torch.empty(self.n, dtype=torch.float32, device="cuda")
        _call("tpa_cpi", self._h, -1 if seed is None else int(seed), None if qd is None else _ptr(qd), c, s_iter,
              t_iter, eps, _ptr(out), _stream(stream))
        return out

    def cpi_batch(self, c: float, s_iter: int, t_iter: int = -1, eps: float = 1e-9, seeds=None, q=None, out=None,
                  stream=None):
        """Algorithm 1 for k restarts at once (seeds [k], or dense q [k, n]),
        on seed tiles: row j is the sum of x(i) over s_iter <= i <= t_iter
        for restart j, each with its own eps break.  Returns float32 [k, n]."""
        torch = _torch()
        if (seeds is None) == (q is None):
            raise ValueError("pass exactly one of seeds and q")
        sd = qd = None
        if seeds is not None:
            sd = seeds.to(device="cuda", dtype=torch.int32).contiguous().reshape(-1)
            k = sd.numel()
        else:
            qd = q.to(device="cuda", dtype=torch.float32).contiguous()
            if qd.dim() != 2 or qd.shape[1] != self.n:
                raise ValueError("q must be [k, n]")
            k = qd.shape[0]
        if out is None:
            out = torch.empty((k, self.n), dtype=torch.float32, device="cuda")
        _call("tpa_cpi_batch", self._h, None if sd is None else _ptr(sd), None if qd is None else _ptr(qd), k, c,
              s_iter, t_iter, eps, _ptr(out), _stream(stream))
        return out

    def query_dense(self, q, c: float, S: int, T: int, out=None, stream=None):
        """r_TPA for dense restart vectors q [k, n] (float32): returns [k, n]."""
        torch = _torch()
        qd = q.to(device="cuda", dtype=torch.float32).contiguous()
        if qd.dim() != 2 or qd.shape[1] != self.n:
            raise ValueError("q must be [k, n]")
        k = qd.shape[0]
        if out is None:
            out = torch.empty((k, self.n), dtype=torch.float32, device="cuda")
        _call("tpa_query_dense", self._h, _ptr(qd), k, c, S, T, _ptr(out), _stream(stream))
        return out

    def backward(self, grad_out, c: float, S: int, T: int, seeds=None, q=None, packed: bool = False,
                 want_logits: bool = True, want_q: bool = True, checkpoint_every: int = 0, stream=None):
        """Gradients of L = sum(grad_out * r_TPA) w.r.t. the edge logits (A~
        order, [m]) and the restart vectors ([k, n]); returns (dtheta, dq)."""
        torch = _torch()
        go = grad_out.to(device="cuda", dtype=torch.float32).contiguous()
        k = go.shape[0]
        if go.dim() != 2 or go.shape[1] != self.n:
            raise ValueError("grad_out must be [k, n]")
        sp = qp = None
        if seeds is not None:
            sd = seeds.to(device="cuda", dtype=torch.int32).contiguous()
            sp = _ptr(sd)
        if q is not None:
            qd = q.to(device="cuda", dtype=torch.float32).contiguous()
            if qd.shape != go.shape:
                raise ValueError("q must match grad_out's shape")
            qp = _ptr(qd)
        dth = torch.empty(self.m, dtype=torch.float32, device="cuda") if want_logits else None
        dq = torch.empty((k, self.n), dtype=torch.float32, device="cuda") if want_q else None
        _call("tpa_backward", self._h, sp, qp, k, int(packed), c, S, T, _ptr(go),
              _ptr(dth) if dth is not None else None, _ptr(dq) if dq is not None else None,
              checkpoint_every, _stream(stream))
        return dth, dq

    def capture_query(self, c: float, S: int, T: int, out, seeds=None, q=None, packed: bool = False,
                      stream=None) -> "QueryGraph":
        """Record a query into a HIP graph; seeds / q / out must stay alive and
        keep their addresses (their contents may change between replays)."""
        torch = _torch()
        sp = qp = None
        if seeds is not None:
            if seeds.dtype != torch.int32 or not seeds.is_cuda or not seeds.is_contiguous():
                raise ValueError("seeds must be a contiguous int32 device tensor")
            sp, keep, k = _ptr(seeds), seeds, (seeds.shape[1] if packed else seeds.numel())
        elif q is not None:
            if q.dtype != torch.float32 or not q.is_cuda or not q.is_contiguous():
                raise ValueError("q must be a contiguous float32 device tensor")
            qp, keep, k = _ptr(q), q, q.shape[0]
        else:
            raise ValueError("pass seeds or q")
        h = _vp()
        _call("tpa_query_graph_create", self._h, sp, qp, k, int(packed), c, S, T, _ptr(out),
              _stream(stream), C.byref(h))
        return QueryGraph(h.value, (self, keep, out))

    def autotune(self, seeds, c: float, S: int, T: int, scratch_out=None, stream=None):
        """Pick the fastest parity-checked (seed tile, edge budget) for these
        seeds; returns (seed_tile, edges_per_item, ms)."""
        torch = _torch()
        sd = seeds.to(device="cuda", dtype=torch.int32).contiguous()
        k = sd.numel()
        if scratch_out is None:
            scratch_out = torch.empty((k, self.n), dtype=torch.float32, device="cuda")
        t, e, ms = C.c_int(), C.c_int(), C.c_double()
        _call("tpa_autotune", self._h, _ptr(sd), k, c, S, T, _ptr(scratch_out), C.byref(t), C.byref(e),
              C.byref(ms), _stream(stream))
        return t.value, e.value, ms.value

    def reserve(self, k: int):
        _call("tpa_reserve", self._h, k)

    def workspace_size(self, k: int) -> int:
        """Bytes of query workspace for k columns (tpa_query_workspace_size)."""
        b = C.c_size_t(0)
        _call("tpa_query_workspace_size", self._h, k, C.byref(b))
        return int(b.value)

    def set_tuning(self, seed_tile: int = 0, edges_per_item: int = 0):
        _call("tpa_set_tuning", self._h, seed_tile, edges_per_item)

    def set_push_limit(self, max_edges: int = -1):
        """Single-seed queries push their second family step when the
        seed's frontier has at most max_edges out-edges (-1: default m/8,
        0: always pull)."""
        _call("tpa_set_push_limit", self._h, max_edges)

    def set_gather_layout(self, layout=2):
        """Order of the gathered work vectors and of each row's edge sum:
        2 (default, also for True) hub-first with the single-vector step's
        group items in rank order (bitwise the sums of 1), 1 hub-first,
        0 (also for False) node order; 0 and 1 agree up to FP32 rounding."""
        if isinstance(layout, bool):
            layout = 2 if layout else 0
        _call("tpa_set_gather_layout", self._h, int(layout))

    def device_bytes(self) -> int:
        """Device memory the handle holds (tpa_graph_device_bytes)."""
        v = C.c_size_t()
        _call("tpa_graph_device_bytes", self._h, C.byref(v))
        return v.value

    def get_gather_layout(self) -> int:
        v = C.c_int()
        _call("tpa_get_gather_layout", self._h, C.byref(v))
        return v.value

    def set_sliced_sweep(self, mode: int = 1):
        """XCD-sliced sweep of the stranger chain: 0 off, 1 (default) from
        2^23 nodes, 2 always (graphs with 1/outdeg weights in the hub-first
        layout)."""
        _call("tpa_set_sliced_sweep", self._h, int(mode))

    def get_sliced_sweep(self):
        """(mode, active): the mode and whether the sliced schedule is built
        and in use."""
        v, a = C.c_int(), C.c_int()
        _call("tpa_get_sliced_sweep", self._h, C.byref(v), C.byref(a))
        return v.value, bool(a.value)

    def get_push_limit(self) -> int:
        v = C.c_int64()
        _call("tpa_get_push_limit", self._h, C.byref(v))
        return v.value

    def set_tile_push_limit(self, max_edges: int = -1):
        """Seed tiles (2..64 seeds) push their second family step when the
        tile's frontier edges, summed over its columns, number at most
        max_edges (-1: default m/4, 0: always pull)."""
        _call("tpa_set_tile_push_limit", self._h, max_edges)

    def get_tile_push_limit(self) -> int:
        v = C.c_int64()
        _call("tpa_get_tile_push_limit", self._h, C.byref(v))
        return v.value

    def set_third_push_limit(self, max_edges: int = -1):
        """Single-seed queries whose second step was pushed push their third
        step too when y2's support has at most max_edges out-edges (-1:
        default m/20 on graphs of at least 2^28 edges, else pull; 0: always
        pull)."""
        _call("tpa_set_third_push_limit", self._h, max_edges)

    def get_third_push_limit(self) -> int:
        v = C.c_int64()
        _call("tpa_get_third_push_limit", self._h, C.byref(v))
        return v.value

    def get_tuning(self):
        a, b = C.c_int(), C.c_int()
        _call("tpa_get_tuning", self._h, C.byref(a), C.byref(b))
        return a.value, b.value

    def set_keep_iterates(self, keep: bool = True):
        """Keep the stranger chain's iterates at the next preprocess, for the
        adjoint (tpa_set_keep_iterates)."""
        _call("tpa_set_keep_iterates", self._h, int(bool(keep)))

    def device_error(self, stream=None):
        """Raise TPAError if a query since the last check saw a bad seed."""
        _call("tpa_get_device_error", self._h, _stream(stream))


def topk(vals, k: int, stream=None):
    """The k largest entries of each row of vals [rows, n] (value
    descending, ties by smaller index, NaN last): (int32 idx, float32 val),
    both [rows, k]."""
    torch = _torch()
    v = vals.to(device="cuda", dtype=torch.float32).contiguous()
    if v.dim() == 1:
        v = v.unsqueeze(0)
    rows, n = v.shape
    idx = torch.empty((rows, k), dtype=torch.int32, device="cuda")
    val = torch.empty((rows, k), dtype=torch.float32, device="cuda")
    _call("tpa_topk", _ptr(v), rows, n, k, _ptr(idx), _ptr(val), _stream(stream))
    return idx, val


def row_l1(x, y, a: float = 1.0, stream=None):
    """Per-row sum |a x - y| in FP64 (x, y: [rows, n] or [n])."""
    torch = _torch()
    xd = x.to(device="cuda", dtype=torch.float32).contiguous()
    yd = y.to(device="cuda", dtype=torch.float32).contiguous()
    if xd.shape != yd.shape:
        raise ValueError("x and y differ in shape")
    if xd.dim() == 1:
        xd, yd = xd.unsqueeze(0), yd.unsqueeze(0)
    out = torch.empty(xd.shape[0], dtype=torch.float64, device="cuda")
    _call("tpa_row_l1", _ptr(xd), _ptr(yd), xd.shape[0], xd.shape[1], a, _ptr(out), _stream(stream))
    return out


class QueryGraph:
    """A captured query (tpa_query_graph_t); launch() replays it."""

    def __init__(self, handle: int, keep):
        self._h = _vp(handle)
        self._keep = keep

    def launch(self, stream=None):
        _call("tpa_query_graph_launch", self._h, _stream(stream))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().tpa_query_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _set_state(graph, theta, c, T, keep_iterates):
    """Weights from theta, then preprocessing (the stranger part depends
    on the weights), keeping the stranger chain's iterates for the adjoint
    when asked."""
    graph.set_logits(theta.detach())
    if keep_iterates:
        graph.set_keep_iterates(True)
    graph.preprocess(c, T)


def _autograd_function():
    import torch

    class TPAFunction(torch.autograd.Function):
        """r_TPA = TPAFunction.apply(theta, Q, graph, c, S, T[, checkpoint_every]).

        theta: per-edge logits [m] in A~ order (row-softmax weights), Q: dense
        restart vectors [k, n].  The forward sets the graph's weights from
        theta and re-runs preprocessing (the stranger part depends on the
        weights), keeping the stranger chain's iterates when theta needs a
        gradient and checkpoint_every is 0 (tpa_set_keep_iterates); the
        backward differentiates both CPI chains on the device.
        """

        @staticmethod
        def forward(ctx, theta, Q, graph, c, S, T, checkpoint_every=0):
            keep = ctx.needs_input_grad[0] and checkpoint_every == 0
            _set_state(graph, theta, c, T, keep)
            R = graph.query_dense(Q.detach(), c, S, T)
            ctx.graph, ctx.args = graph, (c, S, T, checkpoint_every, keep)
            # the handle's state this output was computed from
            ctx.version = graph.version()
            ctx.save_for_backward(theta, Q)
            return R

        @staticmethod
        def backward(ctx, gR):
            theta, Q = ctx.saved_tensors
            c, S, T, ck, keep = ctx.args
            g = ctx.graph
            if g.version() != ctx.version:
                # the graph was given other logits (or preprocessed again)
                # since this forward: restore the forward's weights and
                # stranger part, so the derivative is that of this output
                _set_state(g, theta, c, T, keep)
            dth, dq = g.backward(gR, c, S, T, q=Q, want_logits=ctx.needs_input_grad[0],
                                 want_q=ctx.needs_input_grad[1], checkpoint_every=ck)
            return dth, dq, None, None, None, None, None

    return TPAFunction


class _LazyFunction:
    _f = None

    def __getattr__(self, name):
        if _LazyFunction._f is None:
            _LazyFunction._f = _autograd_function()
        return getattr(_LazyFunction._f, name)


TPAFunction = _LazyFunction()

