"""Python binding of the CPU oracle (``mce_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this
package and this package never imports the GPU library; the two share nothing
but the seeded input generators in ``graphgen``.

Functions return plain Python values / numpy arrays.  Clique lists come back
as sorted lists of sorted tuples.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mce_oracle.cpp")
_LIB = os.path.join(_HERE, "libmce_oracle.so")

RANK_DEGREE = 0
RANK_DEGENERACY = 1
RANK_TRIANGLE = 2
RANK_PEEL = 3
HIST_LEN = 4097  # clique-size histogram entries: sizes 0..4095, then >= 4096

RANKS = {"degree": RANK_DEGREE, "degeneracy": RANK_DEGENERACY, "triangle": RANK_TRIANGLE, "peel": RANK_PEEL}


class _Result(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("set_hash", ctypes.c_uint64), ("nodes", ctypes.c_uint64)]


class _ImceResult(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in
                ("n_applied", "n_skipped", "n_new", "n_del", "hash_new", "hash_del", "count", "set_hash")]


class _Cliques(ctypes.Structure):
    _fields_ = [("cap_cliques", ctypes.c_uint64), ("cap_verts", ctypes.c_uint64),
                ("off", ctypes.POINTER(ctypes.c_uint64)), ("vert", ctypes.POINTER(ctypes.c_uint32)),
                ("n_cliques", ctypes.c_uint64), ("n_verts", ctypes.c_uint64)]


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (host only, no GPU code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P64 = ctypes.POINTER(ctypes.c_uint64)
        P32 = ctypes.POINTER(ctypes.c_uint32)
        L.orc_mix64.restype = ctypes.c_uint64
        L.orc_mix64.argtypes = [ctypes.c_uint64]
        L.orc_clique_hash.restype = ctypes.c_uint64
        L.orc_clique_hash.argtypes = [P32, ctypes.c_uint64]
        L.orc_csr_valid.argtypes = [ctypes.c_uint64, P64, P32]
        L.orc_rank_metric.argtypes = [ctypes.c_uint64, P64, P32, ctypes.c_int, P64]
        L.orc_mce_ttt_root.argtypes = [ctypes.c_uint64, P64, P32, ctypes.POINTER(_Result), ctypes.POINTER(_Cliques)]
        L.orc_mce_brute.argtypes = [ctypes.c_uint64, P64, P32, ctypes.POINTER(_Result), ctypes.POINTER(_Cliques)]
        L.orc_mce_parmce.argtypes = [ctypes.c_uint64, P64, P32, ctypes.c_int, P32, ctypes.c_uint64, ctypes.c_int,
                                     ctypes.POINTER(_Result), P64, P64, P64, ctypes.POINTER(_Cliques), P64,
                                     ctypes.c_uint64]
        L.orc_imce_create.restype = ctypes.c_void_p
        L.orc_imce_create.argtypes = [ctypes.c_uint64, P64, P32, ctypes.c_int]
        L.orc_imce_destroy.argtypes = [ctypes.c_void_p]
        L.orc_imce_snapshot.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Result), ctypes.POINTER(_Cliques)]
        L.orc_imce_add.argtypes = [ctypes.c_void_p, P32, P32, ctypes.c_uint64, ctypes.POINTER(_ImceResult),
                                   ctypes.POINTER(_Cliques), ctypes.POINTER(_Cliques), ctypes.c_int]
        L.orc_imce_remove.argtypes = [ctypes.c_void_p, P32, P32, ctypes.c_uint64, ctypes.POINTER(_ImceResult),
                                      ctypes.POINTER(_Cliques), ctypes.POINTER(_Cliques)]
        _lib = L
    return _lib


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)) if a is not None else None


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)) if a is not None else None


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(g.col, dtype=np.uint32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.uint32)
    return rp, col


def _collect(call) -> List[Tuple[int, ...]]:
    """Runs `call(cliques_struct)` twice: once to size, once to fill."""
    c = _Cliques(0, 0, None, None, 0, 0)
    call(c)
    off = np.zeros(c.n_cliques + 1, dtype=np.uint64)
    vert = np.zeros(max(c.n_verts, 1), dtype=np.uint32)
    c2 = _Cliques(c.n_cliques, c.n_verts, _p64(off), _p32(vert), 0, 0)
    call(c2)
    return [tuple(int(x) for x in vert[off[i]:off[i + 1]]) for i in range(int(c2.n_cliques))]


def mix64(x: int) -> int:
    return int(lib().orc_mix64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def clique_hash(c: Sequence[int]) -> int:
    a = np.ascontiguousarray(sorted(c), dtype=np.uint32)
    return int(lib().orc_clique_hash(_p32(a) if a.size else None, len(a)))


def csr_valid(g) -> bool:
    rp, col = _csr(g)
    return bool(lib().orc_csr_valid(g.n, _p64(rp), _p32(col)))


def rank_metric(g, kind: str = "degree") -> np.ndarray:
    rp, col = _csr(g)
    out = np.zeros(max(g.n, 1), dtype=np.uint64)
    lib().orc_rank_metric(g.n, _p64(rp), _p32(col), RANKS[kind], _p64(out))
    return out[:g.n]


def mce_root(g, cliques: bool = False):
    """Algorithm 1 from the root.  Returns (count, hash, nodes[, cliques])."""
    rp, col = _csr(g)
    r = _Result()
    if cliques:
        cl = _collect(lambda c: lib().orc_mce_ttt_root(g.n, _p64(rp), _p32(col), ctypes.byref(r), ctypes.byref(c)))
        return r.count, r.set_hash, r.nodes, sorted(cl)
    lib().orc_mce_ttt_root(g.n, _p64(rp), _p32(col), ctypes.byref(r), None)
    return r.count, r.set_hash, r.nodes


def mce_brute(g, cliques: bool = False):
    """Definition by exhaustive subsets (n <= 24).  Returns (count, hash[, cliques])."""
    rp, col = _csr(g)
    r = _Result()
    if cliques:
        cl = _collect(lambda c: lib().orc_mce_brute(g.n, _p64(rp), _p32(col), ctypes.byref(r), ctypes.byref(c)))
        return r.count, r.set_hash, sorted(cl)
    rc = lib().orc_mce_brute(g.n, _p64(rp), _p32(col), ctypes.byref(r), None)
    if rc != 0:
        raise ValueError("brute force needs n <= 24")
    return r.count, r.set_hash


class ParMCE:
    """Result of the per-vertex decomposition (Algorithm 4)."""

    def __init__(self, count, set_hash, nodes, nodes_v, count_v, hash_v, cliques, verts, sizes):
        self.count, self.set_hash, self.nodes = count, set_hash, nodes
        self.sizes = sizes  # sizes[k] = maximal cliques with k vertices (last entry: k >= len-1)
        self.nodes_v, self.count_v, self.hash_v = nodes_v, count_v, hash_v
        self.cliques = cliques
        self.verts = verts


def mce_parmce(g, rank: str = "degree", verts: Optional[np.ndarray] = None, threads: int = 1,
               cliques: bool = False) -> ParMCE:
    rp, col = _csr(g)
    r = _Result()
    vs = None if verts is None else np.ascontiguousarray(verts, dtype=np.uint32)
    k = g.n if vs is None else vs.size
    nodes_v = np.zeros(max(k, 1), dtype=np.uint64)
    count_v = np.zeros(max(k, 1), dtype=np.uint64)
    hash_v = np.zeros(max(k, 1), dtype=np.uint64)
    sizes = np.zeros(HIST_LEN, dtype=np.uint64)

    def call(c):
        return lib().orc_mce_parmce(g.n, _p64(rp), _p32(col), RANKS[rank], _p32(vs), k, threads, ctypes.byref(r),
                                    _p64(nodes_v), _p64(count_v), _p64(hash_v), c, _p64(sizes), HIST_LEN)

    cl = None
    if cliques:
        cl = sorted(_collect(lambda c: call(ctypes.byref(c))))
    else:
        call(None)
    return ParMCE(r.count, r.set_hash, r.nodes, nodes_v[:k], count_v[:k], hash_v[:k], cl, vs, sizes)


class Imce:
    """Sequential IMCE: new cliques by Algorithms 5 + 8, subsumed cliques by
    Algorithm 7 run serially against the stored clique set C."""

    def __init__(self, g, threads: int = 1):
        rp, col = _csr(g)
        self.n = g.n
        self._h = lib().orc_imce_create(g.n, _p64(rp), _p32(col), threads)

    def close(self):
        if self._h:
            lib().orc_imce_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def snapshot(self, cliques: bool = False):
        r = _Result()
        if cliques:
            cl = _collect(lambda c: lib().orc_imce_snapshot(self._h, ctypes.byref(r), ctypes.byref(c)))
            return r.count, r.set_hash, sorted(cl)
        lib().orc_imce_snapshot(self._h, ctypes.byref(r), None)
        return r.count, r.set_hash

    def add(self, src, dst, cliques: bool = False, check_form: bool = False):
        """Returns a dict of the batch result (and 'new'/'del' clique lists)."""
        return self._update(lambda s, d, rho, r, cn, cd: lib().orc_imce_add(self._h, s, d, rho, r, cn, cd,
                                                                           int(check_form)), src, dst, cliques)

    def remove(self, src, dst, cliques: bool = False):
        """Edge deletions by the reduction of Section 5.3.  Same dict as add:
        'new' are the cliques that become maximal, 'del' those that stop
        being maximal."""
        return self._update(lambda s, d, rho, r, cn, cd: lib().orc_imce_remove(self._h, s, d, rho, r, cn, cd),
                            src, dst, cliques)

    def _update(self, call, src, dst, cliques):
        s = np.ascontiguousarray(src, dtype=np.uint32)
        d = np.ascontiguousarray(dst, dtype=np.uint32)
        if s.size == 0:
            s = np.zeros(1, np.uint32)
            d = np.zeros(1, np.uint32)
            rho = 0
        else:
            rho = s.size
        r = _ImceResult()
        if cliques:
            # a state-changing call cannot be repeated to size its output, so
            # the lists get a fixed, generous capacity
            cap_c, cap_v = 1 << 16, 1 << 20
            while True:
                off_n = np.zeros(cap_c + 1, np.uint64)
                vert_n = np.zeros(cap_v, np.uint32)
                off_d = np.zeros(cap_c + 1, np.uint64)
                vert_d = np.zeros(cap_v, np.uint32)
                cn = _Cliques(cap_c, cap_v, _p64(off_n), _p32(vert_n), 0, 0)
                cd = _Cliques(cap_c, cap_v, _p64(off_d), _p32(vert_d), 0, 0)
                rc = call(_p32(s), _p32(d), rho, ctypes.byref(r), ctypes.byref(cn), ctypes.byref(cd))
                if rc != 0:
                    raise ValueError("oracle incremental update failed: %d" % rc)
                if cn.n_cliques <= cap_c and cn.n_verts <= cap_v and cd.n_cliques <= cap_c and cd.n_verts <= cap_v:
                    break
                raise RuntimeError("clique lists exceed the oracle's list capacity")
            new = [tuple(int(x) for x in vert_n[off_n[i]:off_n[i + 1]]) for i in range(int(cn.n_cliques))]
            dele = [tuple(int(x) for x in vert_d[off_d[i]:off_d[i + 1]]) for i in range(int(cd.n_cliques))]
        else:
            rc = call(_p32(s), _p32(d), rho, ctypes.byref(r), None, None)
            if rc != 0:
                raise ValueError("oracle incremental update failed: %d" % rc)
            new = dele = None
        out = {k: int(getattr(r, k)) for k, _ in _ImceResult._fields_}
        if cliques:
            out["new"] = sorted(new)
            out["del"] = sorted(dele)
        return out
