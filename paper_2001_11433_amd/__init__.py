"""Python binding of the MI355X maximal clique enumeration library (libmce.so).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides device memory and streams.  If ``libmce.so`` is not
built, importing the binding's entry points raises; there is no CPU fallback.

Entry points mirror ``include/mce.h``: :func:`mce_static`,
:func:`mce_rank_metric`, :func:`mce_features`, and :class:`ImceState`
(``imce_create`` / ``imce_add_edges`` / ``imce_destroy``).
"""

from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmce.so")

MCE_OK, MCE_EINVAL, MCE_ENOMEM, MCE_ENOSPC, MCE_EDEVICE, MCE_ENOTSUP, MCE_ECANCELED = 0, -1, -2, -3, -4, -5, -6
RANKS = {"degree": 0, "degeneracy": 1, "triangle": 2, "ttt_root": 3, "peel": 4}
SCHEDS = {"degree": 0, "triangle": 1, "cost": 2, "id": 3, "mlp": 4}


class MceError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_strerror(code), code, msg))
        self.code = code


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("on_device", ctypes.c_int)]


class _Opts(ctypes.Structure):
    _fields_ = [("sched", ctypes.c_int), ("validate", ctypes.c_int), ("hip_stream", ctypes.c_void_p),
                ("sched_cost", ctypes.c_void_p), ("waves_per_cu", ctypes.c_uint32),
                ("donate_interval", ctypes.c_uint32), ("frame_cap", ctypes.c_uint32), ("split", ctypes.c_uint32),
                ("compact_waves_per_cu", ctypes.c_uint32), ("inline_compact", ctypes.c_uint32),
                ("compact_order", ctypes.c_uint32), ("lds_row_words", ctypes.c_uint32), ("hand_mb", ctypes.c_uint32),
                ("sched_model", ctypes.c_void_p), ("sched_model_bf16", ctypes.c_void_p)]


class _Result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("set_hash", ctypes.c_uint64), ("nodes_total", ctypes.c_uint64),
                ("donated", ctypes.c_uint64), ("subproblems", ctypes.c_uint64), ("max_cand", ctypes.c_uint64),
                ("alg_ops", ctypes.c_uint64), ("rank_ms", ctypes.c_double), ("build_ms", ctypes.c_double), ("enum_ms", ctypes.c_double),
                ("retries", ctypes.c_uint32), ("pad", ctypes.c_uint32), ("diag", ctypes.c_uint64 * 8),
                ("compact_ms", ctypes.c_double), ("handed", ctypes.c_uint64), ("exec_ops", ctypes.c_uint64),
                ("lds_bytes", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64)]


class _CliqueBuf(ctypes.Structure):
    _fields_ = [("cap_cliques", ctypes.c_uint64), ("cap_verts", ctypes.c_uint64), ("off", ctypes.c_void_p),
                ("vert", ctypes.c_void_p), ("on_device", ctypes.c_int), ("n_cliques", ctypes.c_uint64),
                ("n_verts", ctypes.c_uint64)]


class _PerVertex(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_void_p), ("count", ctypes.c_void_p), ("hash", ctypes.c_void_p),
                ("size_hist", ctypes.c_void_p), ("hist_len", ctypes.c_uint64), ("sched_cost", ctypes.c_void_p)]


class _ImceResult(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in
                ("n_applied", "n_skipped", "n_new", "n_del", "hash_new", "hash_del", "count", "set_hash")] + \
               [("new_ms", ctypes.c_double), ("sub_ms", ctypes.c_double), ("ms", ctypes.c_double),
                ("nodes", ctypes.c_uint64), ("handed", ctypes.c_uint64), ("compact_ms", ctypes.c_double)]


EXPORTS = ("mce_static", "mce_static_noalloc", "mce_rank_metric", "mce_features", "imce_create", "imce_add_edges", "imce_remove_edges",
           "imce_submit", "imce_collect", "imce_device_bytes", "imce_batch_bytes",
           "imce_info",
           "imce_destroy", "mce_strerror", "mce_last_error", "mce_mlp_param_count", "mce_mlp_forward",
           "mce_mlp_forward_bf16", "mce_mlp_grad", "mce_mlp_adam", "mce_mlp_fit_norm", "mce_mlp_to_bf16",
           "mce_mlp_labels")

_lib = None


def lib():
    """Loads libmce.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmce.so is not built; run `python -m paper_2001_11433_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.mce_strerror.restype = ctypes.c_char_p
        L.mce_strerror.argtypes = [ctypes.c_int]
        L.mce_last_error.restype = ctypes.c_char_p
        L.mce_static.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int, ctypes.POINTER(_Opts), ctypes.POINTER(_Result),
                                 ctypes.POINTER(_CliqueBuf), ctypes.POINTER(_PerVertex)]
        L.mce_static_noalloc.argtypes = L.mce_static.argtypes
        L.mce_rank_metric.argtypes = [ctypes.POINTER(_Csr), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        L.mce_features.argtypes = [ctypes.POINTER(_Csr), ctypes.c_void_p, ctypes.c_void_p]
        L.imce_create.argtypes = [ctypes.POINTER(_Csr), ctypes.POINTER(_Opts), ctypes.POINTER(ctypes.c_void_p),
                                  ctypes.POINTER(_Result)]
        L.imce_add_edges.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                     ctypes.c_int, ctypes.POINTER(_ImceResult), ctypes.POINTER(_CliqueBuf),
                                     ctypes.POINTER(_CliqueBuf)]
        L.imce_remove_edges.argtypes = L.imce_add_edges.argtypes
        L.imce_submit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                  ctypes.c_int]
        L.imce_collect.argtypes = [ctypes.c_void_p, ctypes.POINTER(_ImceResult), ctypes.POINTER(_CliqueBuf),
                                   ctypes.POINTER(_CliqueBuf)]
        L.imce_device_bytes.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]
        L.imce_batch_bytes.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
        L.imce_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]
        L.imce_destroy.argtypes = [ctypes.c_void_p]
        L.mce_mlp_param_count.restype = ctypes.c_uint32
        vp, u64 = ctypes.c_void_p, ctypes.c_uint64
        L.mce_mlp_forward.argtypes = [vp, vp, u64, vp, vp]
        L.mce_mlp_forward_bf16.argtypes = [vp, vp, vp, u64, vp, vp]
        L.mce_mlp_grad.argtypes = [vp, vp, vp, u64, vp, vp, vp]
        L.mce_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_float, ctypes.c_uint32, vp]
        L.mce_mlp_fit_norm.argtypes = [vp, vp, u64, vp]
        L.mce_mlp_to_bf16.argtypes = [vp, vp, vp]
        L.mce_mlp_labels.argtypes = [vp, u64, vp, vp]
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().mce_strerror(code).decode()
    except Exception:
        return "error"


def _check(code: int):
    if code != MCE_OK:
        raise MceError(code, lib().mce_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a HIP device is required")
    return torch


class DeviceGraph:
    """A CSR resident in device memory (torch tensors; uint64/uint32 bits
    stored in int64/int32 tensors)."""

    def __init__(self, n: int, row_ptr, col):
        self.n = int(n)
        self.row_ptr = row_ptr
        self.col = col

    @classmethod
    def from_numpy(cls, n: int, row_ptr: np.ndarray, col: np.ndarray, device: str = "cuda"):
        torch = _torch()
        rp = torch.from_numpy(np.ascontiguousarray(row_ptr, dtype=np.uint64).view(np.int64)).to(device)
        c = np.ascontiguousarray(col, dtype=np.uint32)
        if c.size == 0:
            c = np.zeros(1, np.uint32)
        cc = torch.from_numpy(c.view(np.int32)).to(device)
        return cls(n, rp, cc)

    @classmethod
    def from_graph(cls, g, device: str = "cuda"):
        return cls.from_numpy(g.n, g.row_ptr, g.col, device)

    def csr(self) -> _Csr:
        return _Csr(self.n, self.row_ptr.data_ptr(), self.col.data_ptr(), 1)


def _as_device_graph(g) -> DeviceGraph:
    return g if isinstance(g, DeviceGraph) else DeviceGraph.from_graph(g)


def _stream_ptr(stream) -> Optional[int]:
    torch = _torch()
    st = stream if stream is not None else torch.cuda.current_stream()
    return int(st.cuda_stream) or None


def _opts(sched="degree", validate=False, stream=None, cost=None, waves_per_cu=0, donate_interval=0,
          frame_cap=0, split=0, compact_waves_per_cu=0, inline_compact=False, compact_order=0,
          lds_row_words=0, model=None, hand_mb=0) -> _Opts:
    o = _Opts()
    o.sched = SCHEDS[sched]
    o.validate = int(bool(validate))
    o.hip_stream = _stream_ptr(stream)
    o.sched_cost = cost.data_ptr() if cost is not None else None
    o.waves_per_cu = int(waves_per_cu)
    o.donate_interval = int(donate_interval)
    o.frame_cap = int(frame_cap)
    o.split = int(split)
    o.compact_waves_per_cu = int(compact_waves_per_cu)
    o.inline_compact = int(bool(inline_compact))
    o.compact_order = int(compact_order)
    o.lds_row_words = int(lds_row_words)
    o.hand_mb = int(hand_mb)
    if sched == "mlp":
        if model is None:
            raise ValueError("sched='mlp' needs model= (a costmodel.CostModel)")
        o.sched_model = model.params.data_ptr()
        o.sched_model_bf16 = model.bf16().data_ptr()
    return o


def _decode_cliques(off: np.ndarray, vert: np.ndarray, nc: int) -> List[Tuple[int, ...]]:
    return [tuple(int(x) for x in vert[int(off[i]):int(off[i + 1])]) for i in range(nc)]


def mce_static(g, rank: str = "degree", sched: str = "degree", cliques: bool = False, per_vertex: bool = False,
               validate: bool = False, stream=None, cost=None, waves_per_cu: int = 0, donate_interval: int = 0,
               frame_cap: int = 0, cap_cliques: int = 1 << 16, cap_verts: int = 1 << 20,
               split: int = 0, compact_waves_per_cu: int = 0, inline_compact: bool = False,
               compact_order: int = 0, size_hist: int = 0, noalloc: bool = False,
               lds_row_words: int = 0, model=None, sched_cost_out: bool = False,
               hand_mb: int = 0) -> Dict[str, object]:
    """All maximal cliques of `g` (a graphgen.Graph or DeviceGraph).

    Returns a dict with count, set_hash, nodes_total, donated, subproblems,
    max_cand, rank_ms, build_ms, enum_ms, retries; with cliques=True also
    'cliques' (sorted list of sorted tuples); with per_vertex=True the device
    tensors 'nodes_v', 'count_v', 'hash_v' (int64 views of uint64); with
    noalloc=True the call goes to mce_static_noalloc (no device allocation
    inside the library; the outputs are allocated here, by torch); with
    size_hist=L > 1 also 'size_hist', a numpy uint64 array of L entries (entry
    k = maximal cliques with k vertices, the last entry L-1 or more).
    sched='mlp' evaluates the cost model `model` (costmodel.CostModel) inside
    the call to order the queue; sched_cost_out=True returns its predictions
    as 'sched_cost' (float32 device tensor)."""
    torch = _torch()
    dg = _as_device_graph(g)
    csr = dg.csr()
    o = _opts(sched, validate, stream, cost, waves_per_cu, donate_interval, frame_cap, split, compact_waves_per_cu,
              inline_compact, compact_order, lds_row_words, model, hand_mb)
    entry = lib().mce_static_noalloc if noalloc else lib().mce_static
    res = _Result()
    pv = None
    tensors = {}
    hist = None
    if per_vertex:
        for k in ("nodes_v", "count_v", "hash_v"):
            tensors[k] = torch.zeros(max(dg.n, 1), dtype=torch.int64, device=dg.row_ptr.device)
    if size_hist:
        hist = torch.zeros(int(size_hist), dtype=torch.int64, device=dg.row_ptr.device)
    costs = None
    if sched_cost_out:
        costs = torch.zeros(max(dg.n, 1), dtype=torch.float32, device=dg.row_ptr.device)
    if per_vertex or size_hist or sched_cost_out:
        pv = _PerVertex(tensors["nodes_v"].data_ptr() if per_vertex else None,
                        tensors["count_v"].data_ptr() if per_vertex else None,
                        tensors["hash_v"].data_ptr() if per_vertex else None,
                        hist.data_ptr() if hist is not None else None, int(size_hist),
                        costs.data_ptr() if costs is not None else None)
    out = {}
    if cliques:
        cc, cv = cap_cliques, cap_verts
        for _ in range(3):
            off = torch.zeros(cc + 1, dtype=torch.int64, device=dg.row_ptr.device)
            vert = torch.zeros(max(cv, 1), dtype=torch.int32, device=dg.row_ptr.device)
            buf = _CliqueBuf(cc, cv, off.data_ptr(), vert.data_ptr(), 1, 0, 0)
            rc = entry(ctypes.byref(csr), RANKS[rank], ctypes.byref(o), ctypes.byref(res),
                       ctypes.byref(buf), ctypes.byref(pv) if pv else None)
            if rc == MCE_ENOSPC:
                cc, cv = int(buf.n_cliques), int(buf.n_verts)
                continue
            _check(rc)
            nc = int(buf.n_cliques)
            offn = off[:nc + 1].cpu().numpy().view(np.uint64)
            vn = vert[:int(buf.n_verts)].cpu().numpy().view(np.uint32)
            out["cliques"] = sorted(_decode_cliques(offn, vn, nc))
            break
        else:
            raise MceError(MCE_ENOSPC, "clique buffer sizing did not converge")
    else:
        _check(entry(ctypes.byref(csr), RANKS[rank], ctypes.byref(o), ctypes.byref(res), None,
                     ctypes.byref(pv) if pv else None))
    out.update({k: getattr(res, k) for k, _ in _Result._fields_ if k not in ("pad", "diag")})
    out["diag"] = list(res.diag)
    if per_vertex:
        for k, t in tensors.items():
            out[k] = t[:dg.n]
    if hist is not None:
        out["size_hist"] = hist.cpu().numpy().view(np.uint64)
    if costs is not None:
        out["sched_cost"] = costs[:dg.n]
    return out


def mce_rank_metric(g, rank: str = "degree", stream=None):
    """Per-vertex rank metric (degree, core number or triangle count), int64 device tensor."""
    torch = _torch()
    dg = _as_device_graph(g)
    out = torch.zeros(max(dg.n, 1), dtype=torch.int64, device=dg.row_ptr.device)
    csr = dg.csr()
    _check(lib().mce_rank_metric(ctypes.byref(csr), RANKS[rank], out.data_ptr(), _stream_ptr(stream)))
    return out[:dg.n]


def mce_features(g, stream=None):
    """Cost-model features [n, 4] float32 on the device: log1p of degree, core
    number, triangles, length-2 walks."""
    torch = _torch()
    dg = _as_device_graph(g)
    out = torch.zeros((max(dg.n, 1), 4), dtype=torch.float32, device=dg.row_ptr.device)
    csr = dg.csr()
    _check(lib().mce_features(ctypes.byref(csr), out.data_ptr(), _stream_ptr(stream)))
    return out[:dg.n]


def to_u64(t) -> np.ndarray:
    """Device int64 tensor holding uint64 bits -> numpy uint64."""
    return t.detach().cpu().numpy().view(np.uint64)


class ImceState:
    """Device-resident incremental state (imce_create / imce_add_edges /
    imce_destroy).  `add` returns a dict with the batch result and, on
    request, the new and subsumed cliques as sorted lists of sorted tuples."""

    def __init__(self, g, stream=None, waves_per_cu: int = 0, donate_interval: int = 0, compact_waves_per_cu: int = 0,
                 inline_compact: bool = False, compact_order: int = 0, lds_row_words: int = 0, frame_cap: int = 0):
        torch = _torch()
        self._torch = torch
        dg = _as_device_graph(g)
        self.n = dg.n
        self.stream = stream
        self._opts = _opts("degree", False, stream, None, waves_per_cu, donate_interval, frame_cap, 0,
                           compact_waves_per_cu, inline_compact, compact_order, lds_row_words)
        h = ctypes.c_void_p()
        res = _Result()
        csr = dg.csr()
        _check(lib().imce_create(ctypes.byref(csr), ctypes.byref(self._opts), ctypes.byref(h), ctypes.byref(res)))
        self._h = h
        self.initial = {"count": res.count, "set_hash": res.set_hash, "nodes_total": res.nodes_total,
                        "enum_ms": res.enum_ms}

    def close(self):
        if getattr(self, "_h", None):
            lib().imce_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        n, nnz, c, h = (ctypes.c_uint64() for _ in range(4))
        _check(lib().imce_info(self._h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(c), ctypes.byref(h)))
        return {"n": n.value, "nnz": nnz.value, "count": c.value, "set_hash": h.value}

    def add(self, src, dst, cliques: bool = False, cap_cliques: int = 1 << 14, cap_verts: int = 1 << 18):
        """imce_add_edges: 'new' / 'del' are the cliques that become / stop
        being maximal."""
        return self._update(lib().imce_add_edges, src, dst, cliques, cap_cliques, cap_verts)

    def remove(self, src, dst, cliques: bool = False, cap_cliques: int = 1 << 14, cap_verts: int = 1 << 18):
        """imce_remove_edges (deletions by reduction to additions): same result
        layout as add."""
        return self._update(lib().imce_remove_edges, src, dst, cliques, cap_cliques, cap_verts)

    def device_bytes(self) -> int:
        """imce_device_bytes: device memory the state holds now."""
        b = ctypes.c_uint64()
        _check(lib().imce_device_bytes(self._h, ctypes.byref(b)))
        return b.value

    def batch_bytes(self, rho: int) -> int:
        """imce_batch_bytes: device memory a batch of rho edges may add."""
        b = ctypes.c_uint64()
        _check(lib().imce_batch_bytes(self._h, int(rho), ctypes.byref(b)))
        return b.value

    def submit(self, src, dst, remove: bool = False):
        """imce_submit: the batch's search now, its subsumed pass on the
        state's second stream; collect() returns the result."""
        torch = self._torch
        s = torch.as_tensor(np.ascontiguousarray(np.asarray(src, dtype=np.uint32)).view(np.int32)).cuda()
        d = torch.as_tensor(np.ascontiguousarray(np.asarray(dst, dtype=np.uint32)).view(np.int32)).cuda()
        rho = int(s.numel())
        _check(lib().imce_submit(self._h, s.data_ptr() if rho else None, d.data_ptr() if rho else None, rho, 1,
                                 1 if remove else 0))

    def collect(self, cliques: bool = False, cap_cliques: int = 1 << 14, cap_verts: int = 1 << 18):
        """imce_collect: the oldest submitted batch's result (same layout as add)."""
        torch = self._torch
        res = _ImceResult()
        if not cliques:
            _check(lib().imce_collect(self._h, ctypes.byref(res), None, None))
            return {k: getattr(res, k) for k, _ in _ImceResult._fields_}
        cc, cv = cap_cliques, cap_verts
        for _ in range(3):
            bufs, cbs = [], []
            for _k in range(2):
                off = torch.zeros(cc + 1, dtype=torch.int64, device="cuda")
                vert = torch.zeros(max(cv, 1), dtype=torch.int32, device="cuda")
                bufs.append((off, vert))
                cbs.append(_CliqueBuf(cc, cv, off.data_ptr(), vert.data_ptr(), 1, 0, 0))
            rc = lib().imce_collect(self._h, ctypes.byref(res), ctypes.byref(cbs[0]), ctypes.byref(cbs[1]))
            if rc == MCE_ENOSPC:  # the batch stays to be collected: grow and ask again
                cc = max(cc, int(cbs[0].n_cliques), int(cbs[1].n_cliques))
                cv = max(cv, int(cbs[0].n_verts), int(cbs[1].n_verts))
                continue
            _check(rc)
            out = {k: getattr(res, k) for k, _ in _ImceResult._fields_}
            for name, cb, (off, vert) in zip(("new", "del"), cbs, bufs):
                nc = int(cb.n_cliques)
                offn = off[:nc + 1].cpu().numpy().view(np.uint64)
                vn = vert[:int(cb.n_verts)].cpu().numpy().view(np.uint32)
                out[name] = sorted(_decode_cliques(offn, vn, nc))
            return out
        raise MceError(MCE_ENOSPC, "clique buffer sizing did not converge")

    def _update(self, fn, src, dst, cliques, cap_cliques, cap_verts):
        torch = self._torch
        s = torch.as_tensor(np.ascontiguousarray(np.asarray(src, dtype=np.uint32)).view(np.int32)).cuda()
        d = torch.as_tensor(np.ascontiguousarray(np.asarray(dst, dtype=np.uint32)).view(np.int32)).cuda()
        rho = int(s.numel())
        res = _ImceResult()
        if not cliques:
            _check(fn(self._h, s.data_ptr() if rho else None, d.data_ptr() if rho else None, rho, 1,
                      ctypes.byref(res), None, None))
            out = {k: getattr(res, k) for k, _ in _ImceResult._fields_}
            return out
        cc, cv = cap_cliques, cap_verts
        for _ in range(3):
            bufs = []
            cbs = []
            for _k in range(2):
                off = torch.zeros(cc + 1, dtype=torch.int64, device="cuda")
                vert = torch.zeros(max(cv, 1), dtype=torch.int32, device="cuda")
                bufs.append((off, vert))
                cbs.append(_CliqueBuf(cc, cv, off.data_ptr(), vert.data_ptr(), 1, 0, 0))
            rc = fn(self._h, s.data_ptr() if rho else None, d.data_ptr() if rho else None, rho, 1,
                    ctypes.byref(res), ctypes.byref(cbs[0]), ctypes.byref(cbs[1]))
            if rc == MCE_ENOSPC:
                cc = max(cc, int(cbs[0].n_cliques), int(cbs[1].n_cliques))
                cv = max(cv, int(cbs[0].n_verts), int(cbs[1].n_verts))
                continue
            _check(rc)
            out = {k: getattr(res, k) for k, _ in _ImceResult._fields_}
            for name, cb, (off, vert) in zip(("new", "del"), cbs, bufs):
                nc = int(cb.n_cliques)
                offn = off[:nc + 1].cpu().numpy().view(np.uint64)
                vn = vert[:int(cb.n_verts)].cpu().numpy().view(np.uint32)
                out[name] = sorted(_decode_cliques(offn, vn, nc))
            return out
        raise MceError(MCE_ENOSPC, "clique buffer sizing did not converge")
