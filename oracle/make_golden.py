"""Writes the stored expected values of the full-size parity tests.

TEST INFRASTRUCTURE ONLY.  Every value this script writes comes from the CPU
oracle (``oracle``) run on inputs from the seeded generators (``graphgen``);
it imports nothing else of this repository, and in particular nothing of the
GPU library.

    python oracle/make_golden.py c3 [--threads T]    # tests/golden/c3_totals.json
    python oracle/make_golden.py c5 [--threads T]    # tests/golden/c5_stream.json
    python oracle/make_golden.py rmat --scale S      # tests/golden/rmat<S>_totals.json

* c3: the 1M-vertex Chung-Lu graph (gamma 2.1, mean degree 20, seed 0) with 500
  planted communities (U{30..80}, p 0.9, seed 1) under degree ownership:
  ParMCE (Algorithm 4 over Algorithm 1) on every vertex.  Stores the totals
  (cliques, set hash, search nodes), the per-subproblem triples of the
  heaviest subproblems, a SHA-256 digest of the three per-subproblem arrays
  (uint64 little-endian, nodes then cliques then hashes) and the clique-size
  histogram.
* c5: the 500k-vertex Chung-Lu graph (gamma 2.2, mean degree 16, seed 0) and
  its 200-batch edge stream (U{1000..5000}, seed 2, half triadic closures):
  the sequential IMCE of Section 5 (Algorithms 5, 8 and 7) batch by batch,
  with the stored-set test of Algorithm 7 cross-checked against the maximality
  form on the first batches.  Stores all eight result fields of every batch.
* rmat: R-MAT (edge factor 16, a/b/c/d .57/.19/.19/.05, seed 0) at the given
  scale under degeneracy ownership, same fields as c3.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, _ROOT)

import graphgen as gg  # noqa: E402
import oracle as O  # noqa: E402

GOLDEN = os.path.join(_ROOT, "tests", "golden")


def _digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype="<u8").tobytes())
    return h.hexdigest()


def _static(g, rank: str, threads: int, desc: str, out_name: str, heavy: int = 64):
    t0 = time.time()
    r = O.mce_parmce(g, rank, threads=threads)
    el = time.time() - t0
    order = np.argsort(r.nodes_v, kind="stable")[::-1][:heavy]
    res = {
        "workload": desc,
        "rank": rank,
        "n": int(g.n),
        "m": int(g.m),
        "count": int(r.count),
        "set_hash": "%016x" % int(r.set_hash),
        "nodes_total": int(r.nodes),
        "per_vertex_sha256": _digest(r.nodes_v, r.count_v, r.hash_v),
        "heaviest": [[int(v), int(r.nodes_v[v]), int(r.count_v[v]), "%016x" % int(r.hash_v[v])] for v in order],
        "size_hist": {str(k): int(c) for k, c in enumerate(r.sizes) if c},
        "source": "oracle.mce_parmce (Algorithm 4 over Algorithm 1, sequential TTT per subproblem, %d threads "
                  "over a shared vertex counter), %.0f s" % (threads, el),
        "command": "python oracle/make_golden.py " + " ".join(sys.argv[1:]),
    }
    path = os.path.join(GOLDEN, out_name)
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")
    print("wrote", path, res["count"], res["set_hash"], res["nodes_total"], "%.0f s" % el, flush=True)


def c3(threads: int):
    g = gg.plant_communities(gg.chung_lu(1_000_000, 2.1, 20, seed=0), count=500, smin=30, smax=80, p=0.9, seed=1)
    _static(g, "degree", threads,
            "chung_lu(n=1000000, gamma=2.1, mean_degree=20, seed=0) + 500 planted communities U{30..80} p=0.9 "
            "seed=1; degree rank", "c3_totals.json")


def rmat(scale: int, threads: int):
    g = gg.rmat(scale, 16, 0.57, 0.19, 0.19, seed=0)
    _static(g, "degeneracy", threads,
            "rmat(scale=%d, edge_factor=16, abcd=.57/.19/.19/.05, seed=0); degeneracy rank" % scale,
            "rmat%d_totals.json" % scale)


def c5(threads: int, checked: int = 3):
    g = gg.chung_lu(500_000, 2.2, 16, seed=0)
    stream = gg.edge_stream(g, 200, 1000, 5000, seed=2, triadic_fraction=0.5)
    t0 = time.time()
    st = O.Imce(g, threads=threads)
    count0, hash0 = st.snapshot()
    print("initial", count0, "%016x" % hash0, "%.0f s" % (time.time() - t0), flush=True)
    keys = ("n_applied", "n_skipped", "n_new", "n_del", "hash_new", "hash_del", "count", "set_hash")
    batches = []
    for i, (s, d) in enumerate(stream):
        r = st.add(s, d, check_form=i < checked)
        batches.append([r[k] if not k.startswith("hash") and k != "set_hash" else "%016x" % r[k] for k in keys])
        if i % 10 == 0:
            print("batch", i, r["n_new"], r["n_del"], "%.0f s" % (time.time() - t0), flush=True)
    res = {
        "workload": "chung_lu(n=500000, gamma=2.2, mean_degree=16, seed=0); edge_stream(200 batches, "
                    "rho U{1000..5000}, seed=2, triadic_fraction=0.5)",
        "initial": {"count": int(count0), "set_hash": "%016x" % int(hash0)},
        "fields": list(keys),
        "batches": batches,
        "check_form_batches": checked,
        "source": "oracle.Imce (Section 5: Algorithm 5 with the exclusion of Algorithm 8 for new cliques, "
                  "Algorithm 7 against the stored clique set for subsumed ones), %.0f s" % (time.time() - t0),
        "command": "python oracle/make_golden.py " + " ".join(sys.argv[1:]),
    }
    path = os.path.join(GOLDEN, "c5_stream.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")
    print("wrote", path, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["c3", "c5", "rmat"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--scale", type=int, default=15)
    a = ap.parse_args()
    if a.which == "c3":
        c3(a.threads)
    elif a.which == "c5":
        c5(a.threads)
    else:
        rmat(a.scale, a.threads)


if __name__ == "__main__":
    main()
