"""Work-distribution diagnostics of a static run (host side, numpy only).

The paper motivates its recursive splitting by how unevenly the maximal
cliques, and so the search work, fall on the per-vertex subproblems (Section 4,
Figure 2), and it reports the clique-size distribution of every input graph
(Section 6.1, Figure 5).  These helpers turn the library's per-subproblem
outputs (``mce_static(..., per_vertex=True)``) and its size histogram
(``size_hist=L``) into those two views.  They read results only; nothing here
takes part in the enumeration.
"""

from __future__ import annotations

from typing import Dict

import numpy as np


def smallest_share_holding(x, fraction: float = 0.9) -> float:
    """Smallest share of the entries of `x` (non-negative work per subproblem)
    whose sum reaches `fraction` of the total: the heaviest entries first.
    0 when the total is 0."""
    x = np.sort(np.asarray(x, dtype=np.float64))[::-1]
    if x.size == 0:
        return 0.0
    tot = x.sum()
    if tot == 0:
        return 0.0
    k = int(np.searchsorted(np.cumsum(x), fraction * tot - 1e-9 * tot)) + 1
    return min(k, x.size) / float(x.size)


def imbalance(nodes_v, count_v, fraction: float = 0.9) -> Dict[str, float]:
    """Figure 2 analog: shares of subproblems that hold `fraction` of the search
    nodes and of the cliques, and the heaviest subproblem's share of the nodes."""
    nodes = np.asarray(nodes_v, dtype=np.float64)
    count = np.asarray(count_v, dtype=np.float64)
    tot = nodes.sum()
    pct = int(round(fraction * 100))
    return {"subproblems": int(nodes.size),
            "share_of_subproblems_for_%dpct_nodes" % pct: smallest_share_holding(nodes, fraction),
            "share_of_subproblems_for_%dpct_cliques" % pct: smallest_share_holding(count, fraction),
            "largest_subproblem_share_of_nodes": float(nodes.max() / tot) if tot else 0.0}


def size_distribution(size_hist) -> Dict[str, object]:
    """Figure 5 analog from a clique-size histogram (entry k = cliques with k
    vertices): the non-zero bins, the largest and the mean clique size."""
    h = np.asarray(size_hist, dtype=np.uint64)
    nz = np.flatnonzero(h)
    total = int(h.sum())
    mean = float((np.arange(h.size, dtype=np.float64) * h.astype(np.float64)).sum() / total) if total else 0.0
    return {"bins": {int(k): int(h[k]) for k in nz}, "cliques": total,
            "largest": int(nz[-1]) if nz.size else 0, "mean": mean}
