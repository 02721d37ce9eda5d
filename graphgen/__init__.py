"""Seeded synthetic graph and edge-batch generators.

This module only produces inputs: simple undirected graphs in CSR form
(``row_ptr`` uint64[n+1], ``col`` uint32[2m], each row sorted ascending,
symmetric, no self-loops, no duplicate edges) and edge-addition batches.  It
holds none of the clique-enumeration arithmetic, so both the CPU oracle and the
GPU library can consume its output without sharing any method code.

Every generator draws from ``numpy.random.Generator(PCG64(seed))`` and is a pure
function of its arguments.  The paper evaluates on real networks turned into
simple undirected graphs (self-loops, weights, parallel edges and directions
removed, Section 6.1); these synthetic families stand in for them.
"""

from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Graph", "csr_from_edges", "edges_of", "er", "rmat", "chung_lu",
    "plant_communities", "complete", "edgeless", "cycle", "complete_multipartite",
    "moon_moser", "disjoint_union", "from_edge_list", "edge_stream", "add_edges", "remove_edges", "deletion_stream",
    "relabel", "star", "path",
]


@dataclasses.dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # uint64[n+1]
    col: np.ndarray      # uint32[row_ptr[n]]
    meta: Dict[str, object] = dataclasses.field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1]) // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def neighbors(self, v: int) -> np.ndarray:
        return self.col[int(self.row_ptr[v]):int(self.row_ptr[v + 1])]

    def describe(self) -> Dict[str, object]:
        d = self.degrees()
        out = dict(self.meta)
        out.update(n=self.n, m=self.m,
                   max_degree=int(d.max()) if self.n else 0,
                   isolated=int((d == 0).sum()) if self.n else 0)
        return out


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray, meta: Optional[dict] = None) -> Graph:
    """Symmetrise, drop self-loops and duplicates, sort rows: a simple graph."""
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    if u.size:
        if u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n:
            raise ValueError("edge endpoint out of range")
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = np.unique(a * np.int64(n) + b)
    a = key // n
    b = key % n
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    counts = np.bincount(src, minlength=n) if n else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    if n:
        row_ptr[1:] = np.cumsum(counts, dtype=np.uint64)
    return Graph(n=n, row_ptr=row_ptr, col=dst.astype(np.uint32), meta=dict(meta or {}))


def edges_of(g: Graph) -> Tuple[np.ndarray, np.ndarray]:
    """Each undirected edge once, as (u, v) with u < v, sorted."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr).astype(np.int64))
    dst = g.col.astype(np.int64)
    keep = src < dst
    return src[keep], dst[keep]


def from_edge_list(n: int, edges: Sequence[Tuple[int, int]], name: str = "edges") -> Graph:
    if len(edges) == 0:
        return csr_from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64), {"family": name})
    e = np.asarray(edges, dtype=np.int64)
    return csr_from_edges(n, e[:, 0], e[:, 1], {"family": name})


# ----------------------------------------------------------------------------
# random families

def er(n: int, p: float, seed: int = 0) -> Graph:
    """Erdos-Renyi G(n, p): one Bernoulli(p) draw per pair i<j, in row-major order."""
    rng = _rng(seed)
    iu, ju = np.triu_indices(n, 1)
    r = rng.random(iu.size)
    keep = r < p
    return csr_from_edges(n, iu[keep], ju[keep], {"family": "er", "p": p, "seed": seed})


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 0) -> Graph:
    """R-MAT (Graph500 style): edge_factor*2^scale samples, one quadrant choice
    per level, most significant bit first, no noise and no vertex permutation;
    then symmetrised and deduplicated."""
    n = 1 << scale
    ns = edge_factor * n
    rng = _rng(seed)
    src = np.zeros(ns, dtype=np.int64)
    dst = np.zeros(ns, dtype=np.int64)
    ab = a + b
    abc = a + b + c
    for level in range(scale):
        r = rng.random(ns)
        sb = r >= ab
        db = ((r >= a) & (r < ab)) | (r >= abc)
        bit = np.int64(1) << (scale - 1 - level)
        src |= sb.astype(np.int64) * bit
        dst |= db.astype(np.int64) * bit
    return csr_from_edges(n, src, dst, {"family": "rmat", "scale": scale, "edge_factor": edge_factor,
                                        "abcd": (a, b, c, 1 - abc), "seed": seed})


def _chung_lu_weights(n: int, gamma: float, dbar: float) -> np.ndarray:
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    target = n * dbar
    for _ in range(50):
        w *= target / w.sum()
        cap = np.sqrt(w.sum())
        if w.max() <= cap * (1 + 1e-12):
            break
        w = np.minimum(w, cap)
    return w


def chung_lu(n: int, gamma: float, dbar: float, seed: int = 0) -> Graph:
    """Chung-Lu power-law graph.  Weights w_i ~ (i+1)^(-1/(gamma-1)), capped at
    sqrt(sum w), rescaled to sum n*dbar.  Endpoint pairs are drawn
    proportionally to w until n*dbar/2 distinct non-loop edges exist (first
    occurrences in draw order are kept)."""
    rng = _rng(seed)
    w = _chung_lu_weights(n, gamma, dbar)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m_target = int(round(n * dbar / 2))
    keys = np.zeros(0, dtype=np.int64)
    have = 0
    rounds = 0
    while have < m_target and rounds < 64:
        k = int((m_target - have) * 1.15) + 1024
        u = np.searchsorted(cdf, rng.random(k), side="right")
        v = np.searchsorted(cdf, rng.random(k), side="right")
        u = np.minimum(u, n - 1)
        v = np.minimum(v, n - 1)
        keep = u != v
        a = np.minimum(u[keep], v[keep]).astype(np.int64)
        b = np.maximum(u[keep], v[keep]).astype(np.int64)
        keys = np.concatenate([keys, a * n + b])
        uniq, first = np.unique(keys, return_index=True)
        keys = keys[np.sort(first)]
        have = keys.size
        rounds += 1
    keys = keys[:m_target]
    return csr_from_edges(n, keys // n, keys % n, {"family": "chung_lu", "gamma": gamma, "dbar": dbar,
                                                   "seed": seed})


def plant_communities(g: Graph, count: int = 500, smin: int = 30, smax: int = 80, p: float = 0.9,
                      seed: int = 1) -> Graph:
    """Adds `count` dense communities on disjoint, uniformly sampled vertex sets
    of size ~U{smin..smax}; each intra-community pair is an edge with
    probability p."""
    rng = _rng(seed)
    sizes = rng.integers(smin, smax + 1, size=count)
    if sizes.sum() > g.n:
        raise ValueError("communities do not fit")
    perm = rng.permutation(g.n)
    us: List[np.ndarray] = []
    vs: List[np.ndarray] = []
    off = 0
    for s in sizes:
        members = perm[off:off + s]
        off += s
        iu, ju = np.triu_indices(int(s), 1)
        keep = rng.random(iu.size) < p
        us.append(members[iu[keep]])
        vs.append(members[ju[keep]])
    bu, bv = edges_of(g)
    meta = dict(g.meta)
    meta.update(communities=count, community_size=(smin, smax), community_p=p, community_seed=seed)
    return csr_from_edges(g.n, np.concatenate([bu] + us), np.concatenate([bv] + vs), meta)


# ----------------------------------------------------------------------------
# structured families (closed forms are known for these)

def complete(n: int) -> Graph:
    iu, ju = np.triu_indices(n, 1)
    return csr_from_edges(n, iu, ju, {"family": "complete"})


def edgeless(n: int) -> Graph:
    return csr_from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64), {"family": "edgeless"})


def cycle(n: int) -> Graph:
    i = np.arange(n, dtype=np.int64)
    return csr_from_edges(n, i, (i + 1) % n, {"family": "cycle"})


def path(n: int) -> Graph:
    i = np.arange(max(n - 1, 0), dtype=np.int64)
    return csr_from_edges(n, i, i + 1, {"family": "path"})


def star(n: int) -> Graph:
    i = np.arange(1, n, dtype=np.int64)
    return csr_from_edges(n, np.zeros_like(i), i, {"family": "star"})


def complete_multipartite(sizes: Sequence[int]) -> Graph:
    """Vertices are numbered part by part; two vertices are adjacent iff they
    lie in different parts."""
    sizes = [int(s) for s in sizes]
    n = int(sum(sizes))
    part = np.repeat(np.arange(len(sizes)), sizes)
    iu, ju = np.triu_indices(n, 1)
    keep = part[iu] != part[ju]
    return csr_from_edges(n, iu[keep], ju[keep], {"family": "complete_multipartite", "parts": sizes})


def moon_moser_parts(n: int) -> List[int]:
    """Part sizes of the Moon-Moser extremal graph on n vertices: threes, with
    one part of 4 (or two parts of 2) when n = 1 (mod 3), one part of 2 when
    n = 2 (mod 3)."""
    if n <= 0:
        return []
    if n % 3 == 0:
        return [3] * (n // 3)
    if n % 3 == 1:
        return ([3] * ((n - 4) // 3) + [4]) if n >= 4 else [1]
    return [3] * ((n - 2) // 3) + [2]


def moon_moser(n: int) -> Graph:
    g = complete_multipartite(moon_moser_parts(n))
    g.meta["family"] = "moon_moser"
    return g


def disjoint_union(a: Graph, b: Graph) -> Graph:
    au, av = edges_of(a)
    bu, bv = edges_of(b)
    return csr_from_edges(a.n + b.n, np.concatenate([au, bu + a.n]), np.concatenate([av, bv + a.n]),
                          {"family": "union"})


def relabel(g: Graph, perm: np.ndarray) -> Graph:
    """Vertex v becomes perm[v]."""
    u, v = edges_of(g)
    perm = np.asarray(perm, dtype=np.int64)
    return csr_from_edges(g.n, perm[u], perm[v], dict(g.meta, relabelled=True))


def add_edges(g: Graph, src: np.ndarray, dst: np.ndarray) -> Graph:
    u, v = edges_of(g)
    return csr_from_edges(g.n, np.concatenate([u, np.asarray(src, np.int64)]),
                          np.concatenate([v, np.asarray(dst, np.int64)]), dict(g.meta))


def remove_edges(g: Graph, src: np.ndarray, dst: np.ndarray) -> Graph:
    """g without the listed pairs (in either orientation); pairs that are not
    edges are ignored."""
    u, v = edges_of(g)
    a = np.minimum(np.asarray(src, np.int64), np.asarray(dst, np.int64))
    b = np.maximum(np.asarray(src, np.int64), np.asarray(dst, np.int64))
    gone = np.isin(u * np.int64(g.n) + v, a * np.int64(g.n) + b)
    return csr_from_edges(g.n, u[~gone], v[~gone], dict(g.meta))


def deletion_stream(g: Graph, batches: int, rho_min: int, rho_max: int, seed: int = 3,
                    junk_fraction: float = 0.0) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Pre-generates batches of edge deletions from `g`: each batch draws
    U{rho_min..rho_max} distinct edges of the current graph uniformly (the
    graph shrinks batch by batch); a `junk_fraction` share of extra pairs are
    repeats or non-edges, which a deletion step must skip.  Returns
    [(src uint32[rho], dst uint32[rho])]."""
    rng = _rng(seed)
    u, v = edges_of(g)
    alive = np.ones(u.size, bool)
    out: List[Tuple[np.ndarray, np.ndarray]] = []
    for _ in range(batches):
        idx = np.flatnonzero(alive)
        rho = min(int(rng.integers(rho_min, rho_max + 1)), idx.size)
        pick = rng.choice(idx, rho, replace=False) if rho else np.zeros(0, np.int64)
        alive[pick] = False
        s, d = u[pick].copy(), v[pick].copy()
        flip = rng.random(rho) < 0.5
        s[flip], d[flip] = d[flip].copy(), s[flip].copy()
        nj = int(round(rho * junk_fraction))
        if nj and g.n > 1:
            js = rng.integers(0, g.n, nj)
            jd = (js + rng.integers(1, g.n, nj)) % g.n
            rep = rng.integers(0, max(rho, 1), nj)
            use_rep = (rng.random(nj) < 0.5) & (rho > 0)
            js = np.where(use_rep, s[rep % max(rho, 1)] if rho else js, js)
            jd = np.where(use_rep, d[rep % max(rho, 1)] if rho else jd, jd)
            s = np.concatenate([s, js])
            d = np.concatenate([d, jd])
            perm = rng.permutation(s.size)
            s, d = s[perm], d[perm]
        out.append((s.astype(np.uint32), d.astype(np.uint32)))
    return out


# ----------------------------------------------------------------------------
# edge-addition stream

def edge_stream(g: Graph, batches: int, rho_min: int, rho_max: int, seed: int = 2,
                triadic_fraction: float = 0.5) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Pre-generates a stream of edge-addition batches on top of `g`.

    Batch sizes ~U{rho_min..rho_max}.  A `triadic_fraction` share of each batch
    closes a wedge u-w-v of the *current* stream graph with (u, v) not an edge
    (w drawn proportionally to d(w)(d(w)-1), then u, v two distinct uniform
    neighbours of w); the rest are uniform vertex pairs u != v that are not
    edges.  Collisions (existing edge or repeat within the batch) are
    resampled.  Returns [(src uint32[rho], dst uint32[rho])].
    """
    rng = _rng(seed)
    n = g.n
    deg = g.degrees().astype(np.int64)
    base_keys = None  # sorted keys u*n+v (u<v) of the base graph
    bu, bv = edges_of(g)
    base_keys = np.sort(bu * n + bv)
    added_adj: Dict[int, List[int]] = {}
    added_keys = set()
    out: List[Tuple[np.ndarray, np.ndarray]] = []

    def is_edge(a: int, b: int) -> bool:
        if a > b:
            a, b = b, a
        k = a * n + b
        if k in added_keys:
            return True
        i = np.searchsorted(base_keys, k)
        return bool(i < base_keys.size and base_keys[i] == k)

    def nbr(w: int, idx: int) -> int:
        d0 = int(g.row_ptr[w + 1] - g.row_ptr[w])
        if idx < d0:
            return int(g.col[int(g.row_ptr[w]) + idx])
        return added_adj[w][idx - d0]

    for _ in range(batches):
        rho = int(rng.integers(rho_min, rho_max + 1))
        n_tri = int(round(rho * triadic_fraction))
        n_uni = rho - n_tri
        batch_keys = set()
        src: List[int] = []
        dst: List[int] = []
        wedge_w = deg * (deg - 1)
        cdf = np.cumsum(wedge_w.astype(np.float64))
        total = cdf[-1] if cdf.size else 0.0
        made = 0
        tries = 0
        while made < n_tri and total > 0 and tries < 50 * rho:
            tries += 1
            w = int(np.searchsorted(cdf, rng.random() * total, side="right"))
            w = min(w, n - 1)
            d = int(deg[w])
            if d < 2:
                continue
            i = int(rng.integers(0, d))
            j = int(rng.integers(0, d - 1))
            if j >= i:
                j += 1
            a, b = nbr(w, i), nbr(w, j)
            if a == b:
                continue
            a, b = min(a, b), max(a, b)
            k = a * n + b
            if k in batch_keys or is_edge(a, b):
                continue
            batch_keys.add(k)
            src.append(a)
            dst.append(b)
            made += 1
        want = n_uni + (n_tri - len(src))
        made = 0
        tries = 0
        while made < want and tries < 50 * rho:
            tries += 1
            a = int(rng.integers(0, n))
            b = int(rng.integers(0, n))
            if a == b:
                continue
            a, b = min(a, b), max(a, b)
            k = a * n + b
            if k in batch_keys or is_edge(a, b):
                continue
            batch_keys.add(k)
            src.append(a)
            dst.append(b)
            made += 1
        perm = rng.permutation(len(src))
        s = np.asarray(src, dtype=np.uint32)[perm]
        t = np.asarray(dst, dtype=np.uint32)[perm]
        # flip a random half so batches are not all (min, max) ordered
        flip = rng.random(len(src)) < 0.5
        s2 = np.where(flip, t, s)
        t2 = np.where(flip, s, t)
        out.append((s2.astype(np.uint32), t2.astype(np.uint32)))
        for a, b in zip(s.tolist(), t.tolist()):
            added_keys.add(a * n + b)
            added_adj.setdefault(a, []).append(b)
            added_adj.setdefault(b, []).append(a)
            deg[a] += 1
            deg[b] += 1
    return out
