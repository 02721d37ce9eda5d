"""Benchmark: maximal cliques per second of the static ParMCE path on one GPU.

A step is one full pass of the hot path over the resident graph: rank metric,
subproblem build and queue, persistent enumeration (mce_static).  The default
workload is the 1M-vertex Chung-Lu graph (exponent 2.1, mean degree 20) plus
500 planted communities of 30..80 vertices with intra-edge probability 0.9,
degree ranking: the largest of the configured inputs that one GPU finishes
(the R-MAT scale-18 graph has an estimated ~1e13+ maximal cliques).

Prints one JSON line.  `roofline` covers the persistent enumeration kernel:
achieved = algorithmic 32-bit integer operations counted by the kernel per
launch / the kernel's average duration (HIP events on its stream), against the
integer VALU peak of MI355X (256 CUs x 64 lanes x 2.4 GHz).  `cpu_baseline`
times the CPU oracle on a bounded random sample of the same subproblems.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "maximal cliques/s (bit-exact set hash), learned vs plain sched; p99 update ms"
INT32_VALU_PEAK = 256 * 64 * 2.4e9  # lane-ops/s
LDS_PEAK = 256 * 128 * 2.4e9  # bytes/s: 128 bytes per clock per CU


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str, scale: int):
    import graphgen as gg
    if name == "cl-communities":
        g = gg.plant_communities(gg.chung_lu(1_000_000, 2.1, 20, seed=0), count=500, smin=30, smax=80, p=0.9,
                                 seed=1)
        desc = ("chung_lu(n=1000000, gamma=2.1, mean_degree=20, seed=0) + 500 planted communities "
                "U{30..80} p=0.9 seed=1; degree rank")
        return g, "degree", desc
    if name == "rmat":
        g = gg.rmat(scale, 16, 0.57, 0.19, 0.19, seed=0)
        return g, "degeneracy", "rmat(scale=%d, edge_factor=16, abcd=.57/.19/.19/.05, seed=0); degeneracy rank" % scale
    if name == "er":
        g = gg.er(2000, 0.01, seed=0)
        return g, "degree", "er(n=2000, p=0.01, seed=0); degree rank"
    if name == "cl":
        g = gg.chung_lu(500_000, 2.2, 16, seed=0)
        return g, "degree", "chung_lu(n=500000, gamma=2.2, mean_degree=16, seed=0); degree rank"
    raise SystemExit("unknown workload " + name)


def cpu_baseline(g, rank: str, seconds: float, seed: int = 7):
    """The oracle (sequential per-vertex TTT, all host threads) on a random
    sample of subproblems, grown in chunks until `seconds` have passed."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    order = np.random.default_rng(seed).permutation(g.n).astype(np.uint32)
    done = 0
    cliques = 0
    t0 = time.perf_counter()
    chunk = 4096
    while done < g.n and time.perf_counter() - t0 < seconds:
        sel = order[done:done + chunk]
        r = oracle.mce_parmce(g, rank, verts=sel, threads=threads)
        cliques += r.count
        done += sel.size
        chunk = min(chunk * 2, 1 << 17)
    el = time.perf_counter() - t0
    return {"value": cliques / el if el > 0 else 0.0, "unit": "maximal cliques/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d of %d subproblems in uniform random order (seed %d), %d cliques in %.1f s; the oracle's "
                      "rank metric and G_v construction are inside the timed region" % (done, g.n, seed, cliques, el)}


def cpu_baseline_legs(g, rank: str, seconds: float, seed: int = 7):
    """The other oracle legs: the per-vertex decomposition on one thread over
    the same kind of random sample, and Algorithm 1 from the root (the paper's
    sequential baseline) on the 2000-vertex ER graph, where it finishes."""
    import graphgen as gg
    import oracle
    order = np.random.default_rng(seed).permutation(g.n).astype(np.uint32)
    done = cliques = 0
    t0 = time.perf_counter()
    chunk = 1024
    while done < g.n and time.perf_counter() - t0 < seconds:
        sel = order[done:done + chunk]
        cliques += oracle.mce_parmce(g, rank, verts=sel, threads=1).count
        done += sel.size
        chunk = min(chunk * 2, 1 << 16)
    el = time.perf_counter() - t0
    out = {"o2_one_thread": {"value": cliques / el if el > 0 else 0.0, "unit": "maximal cliques/s", "cores": 1,
                             "kind": "oracle", "sample": "%d of %d subproblems in uniform random order (seed %d), "
                             "%d cliques in %.1f s" % (done, g.n, seed, cliques, el)}}
    er = gg.er(2000, 0.01, seed=0)
    t0 = time.perf_counter()
    c, h, nodes = oracle.mce_root(er)
    el = time.perf_counter() - t0
    out["o1_root_er2000"] = {"value": c / el, "unit": "maximal cliques/s", "cores": 1, "kind": "oracle",
                             "sample": "Algorithm 1 from the root on er(n=2000, p=0.01, seed=0): %d cliques, hash "
                                       "%016x, %d search nodes in %.2f s" % (c, h, nodes, el)}
    return out


def rmat_family(m, scales=(15, 16)):
    """The R-MAT family (edge factor 16, .57/.19/.19/.05, seed 0, degeneracy
    rank) at the largest scales one GPU enumerates in about a minute; scale
    18 is out of reach (each scale multiplies the clique count by about 60)."""
    import graphgen as gg
    from paper_2001_11433_amd import tuner
    out = []
    for scale in scales:
        g = gg.rmat(scale, 16, 0.57, 0.19, 0.19, seed=0)
        dg = m.DeviceGraph.from_graph(g)
        knobs = tuner.lookup(g, "degeneracy", family="rmat%d" % scale)
        r = m.mce_static(dg, rank="degeneracy", **tuner.launch_kwargs(knobs))
        dev_s = (r["rank_ms"] + r["build_ms"] + r["enum_ms"]) / 1e3
        out.append({"scale": scale, "n": g.n, "m": g.m, "maximal_cliques": r["count"],
                    "set_hash": "%016x" % r["set_hash"], "search_nodes": r["nodes_total"], "max_cand": r["max_cand"],
                    "rank_ms": r["rank_ms"], "build_ms": r["build_ms"], "enum_ms": r["enum_ms"],
                    "cliques_per_s": r["count"] / dev_s, "launch": knobs})
        log("rmat scale %d: %d cliques in %.1f ms" % (scale, r["count"], r["enum_ms"]))
    return out


def _median(xs):
    return float(np.median(np.asarray(xs, dtype=np.float64)))


def _family(name: str):
    """(description, rank, graph maker by seed) of a learned-scheduling family."""
    import graphgen as gg
    if name.startswith("rmat"):
        scale = int(name[4:])
        return ("rmat(scale=%d, edge_factor=16, abcd=.57/.19/.19/.05); degeneracy rank" % scale, "degeneracy",
                lambda s: gg.rmat(scale, 16, 0.57, 0.19, 0.19, seed=s))
    if name == "cl1m-communities":
        return ("chung_lu(1e6, 2.1, 20) + 500 communities U{30..80} p=0.9; degree rank", "degree",
                lambda s: gg.plant_communities(gg.chung_lu(1_000_000, 2.1, 20, seed=2 * s),
                                               count=500, smin=30, smax=80, p=0.9, seed=2 * s + 1))
    raise ValueError(name)


def _family_graph(args):
    family, seed = args
    return seed, _family(family)[2](seed)


def pregenerate(family: str, seeds, workers: int = 12):
    """The family's graphs built in a pool of forked host processes (run
    before the GPU is first used: the children only generate graphs)."""
    import multiprocessing as mp
    with mp.get_context("fork").Pool(max(1, min(workers, len(seeds)))) as pool:
        return dict(pool.map(_family_graph, [(family, s) for s in seeds]))


def learned_sched(m, family: str, train_seeds, held_seeds, repeats: int = 3, epochs: int = 400,
                  split: int = 64, graphs=None):
    """Queue order by degree, by triangle count, by the cost model evaluated
    inside the call (MCE_SCHED_MLP: features and BF16 inference overlap the
    subproblem build), the same with the predicted-heavy roots dealt out at
    launch (`split`), and, as the ceiling of any cost-based order, by the node
    counts the enumeration itself measured (with and without the split), on
    held-out graphs of the family.  Ownership is fixed per family, so cliques,
    hash and node counts are identical across orders and only the time moves;
    times are whole calls (rank, build, inference and search) on the device."""
    import torch
    from scipy.stats import spearmanr
    from paper_2001_11433_amd import costmodel, tuner

    fam, rank, make = _family(family)
    if graphs is not None:
        make = graphs.pop
    t0 = time.perf_counter()
    train = [make(s) for s in train_seeds]
    log("learned_sched %s: training on %d graphs" % (family, len(train)))
    tr = costmodel.train_on_graphs(train, rank, epochs=epochs, lr=3e-3)
    del train
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    model = tr["model"]
    out = {"family": fam, "train_seeds": list(train_seeds), "held_out_seeds": list(held_seeds),
           "train": {"vertices": tr["n_train"], "epochs": epochs, "loss_first": tr["losses"][0],
                     "loss_last": tr["losses"][-1], "wall_s": train_s,
                     "kernels": "mce_mlp_grad + mce_mlp_adam (fp32)"},
           "inference": "inside mce_static (MCE_SCHED_MLP): mce_features' columns + BF16 forward on a second stream",
           "policies": {"degree": "vertex degree, largest first", "triangle": "triangles, largest first",
                        "learned": "MLP-predicted log search nodes, largest first, evaluated in the call",
                        "learned_split": "learned, and roots predicted above one wave's share split into up to "
                                         "%d chunks at launch" % split,
                        "measured": "the subproblem's measured search nodes, largest first (ceiling of any "
                                    "cost-based order)",
                        "measured_split": "measured, with the same split"},
           "repeats": repeats, "held_out": []}
    names = ("degree", "triangle", "learned", "learned_split", "measured", "measured_split")
    tot_enum = dict.fromkeys(names, 0.0)
    tot_wall = dict.fromkeys(names, 0.0)
    cliques_total = 0
    for s in held_seeds:
        g = make(s)
        dg = m.DeviceGraph.from_graph(g)
        knobs = tuner.lookup(g, rank, family=family)
        kw = tuner.launch_kwargs(knobs)
        feat, target, base = costmodel.collect(dg, rank)
        pred = model.predict(feat)
        measured = target.float().contiguous()
        y, t = pred.cpu().numpy().astype(np.float64), target.cpu().numpy().astype(np.float64)
        ref = (base["count"], base["set_hash"], base["nodes_total"])
        row = {"seed": s, "n": g.n, "m": g.m, "maximal_cliques": base["count"],
               "set_hash": "%016x" % base["set_hash"], "search_nodes": base["nodes_total"],
               "mse_log_nodes": float(np.mean((y - t) ** 2)), "spearman": float(spearmanr(y, t)[0]),
               "spearman_degree": float(spearmanr(np.diff(g.row_ptr).astype(np.float64), t)[0]),
               "launch": knobs}
        del g
        for name in names:
            enum, dev = [], []
            for _ in range(repeats):
                if name.startswith("learned"):
                    r = m.mce_static(dg, rank=rank, sched="mlp", model=model,
                                     split=split if name.endswith("split") else 0, **kw)
                elif name.startswith("measured"):
                    r = m.mce_static(dg, rank=rank, sched="cost", cost=measured,
                                     split=split if name.endswith("split") else 0, **kw)
                else:
                    r = m.mce_static(dg, rank=rank, sched=name, **kw)
                dev.append(r["rank_ms"] + r["build_ms"] + r["enum_ms"])
                enum.append(r["enum_ms"])
                got = (r["count"], r["set_hash"], r["nodes_total"])
                if got != ref:
                    raise SystemExit("schedule %s changed the result on seed %d: (count, hash, nodes) %r, "
                                     "expected %r" % (name, s, got, ref))
            row[name] = {"enum_ms": _median(enum), "call_ms": _median(dev),
                         "cliques_per_s": base["count"] / (_median(dev) / 1e3)}
            tot_enum[name] += _median(enum)
            tot_wall[name] += _median(dev)
        cliques_total += base["count"]
        log("learned_sched %s seed %d: call ms %s" % (family, s, {k: round(row[k]["call_ms"], 1) for k in names}))
        out["held_out"].append(row)
        del dg
    out["cliques_per_s"] = {k: cliques_total / (v / 1e3) for k, v in tot_wall.items()}
    out["gain_vs_degree"] = {k: tot_wall["degree"] / tot_wall[k] for k in names}
    out["enum_gain_vs_degree"] = {k: tot_enum["degree"] / tot_enum[k] for k in names}
    return out


def ownership_and_imbalance(m, dg, ref, launch, base_rank: str):
    """The same graph under every ownership rank (Section 4.2): the clique set
    (count and hash) must not change, the node count and the split between
    ranking time and enumeration time do.  Then the imbalance of the base
    rank's subproblems (the analog of the paper's Figure 2): the smallest share
    of subproblems that holds 90 % of the search nodes and of the cliques."""
    out = {"ranks": {}}
    for rank in ("degree", "degeneracy", "triangle", "peel", "ttt_root"):
        per_vertex = rank == base_rank
        try:
            r = m.mce_static(dg, rank=rank, per_vertex=per_vertex, **launch)
        except m.MceError as e:  # e.g. a subproblem above the supported cand size
            out["ranks"][rank] = {"error": str(e)}
            log("ownership %s: %s" % (rank, e))
            continue
        if (r["count"], r["set_hash"]) != ref:
            raise SystemExit("ownership rank %s changed the clique set: %r" % (rank, (r["count"], r["set_hash"])))
        out["ranks"][rank] = {"rank_ms": r["rank_ms"], "build_ms": r["build_ms"], "enum_ms": r["enum_ms"],
                              "search_nodes": r["nodes_total"], "max_cand": r["max_cand"]}
        log("ownership %s: rank %.1f ms, build %.1f ms, enum %.1f ms, %d nodes" % (
            rank, r["rank_ms"], r["build_ms"], r["enum_ms"], r["nodes_total"]))
        if per_vertex:
            from paper_2001_11433_amd import diagnostics
            nodes = r["nodes_v"].cpu().numpy().view(np.uint64)
            count = r["count_v"].cpu().numpy().view(np.uint64)
            out["imbalance"] = dict(rank=rank, **diagnostics.imbalance(nodes, count))
    return out


def decompositions(m, repeats: int = 3):
    """Every ownership rank (Section 4.2, plus the peel order) and ParTTT
    (Algorithm 3 applied to the whole-graph root) on the same kernels, on the
    2000-vertex ER graph, R-MAT scale 14 and the 500k Chung-Lu graph:
    rank + build + search device time, median of `repeats`.  ParTTT runs where
    the root pivot's non-neighbours fit the supported subproblem width."""
    import graphgen as gg
    from paper_2001_11433_amd import tuner
    out = {}
    for name, make, fam in (("er2000", lambda: gg.er(2000, 0.01, seed=0), None),
                            ("rmat14", lambda: gg.rmat(14, 16, 0.57, 0.19, 0.19, seed=0), "rmat14"),
                            ("cl500k", lambda: gg.chung_lu(500_000, 2.2, 16, seed=0), "cl500k")):
        g = make()
        dg = m.DeviceGraph.from_graph(g)
        row, ref = {}, None
        for rank in ("degree", "degeneracy", "triangle", "peel", "ttt_root"):
            like = {"ttt_root": "degree", "peel": "degeneracy", "triangle": "degree"}.get(rank, rank)
            kw = tuner.launch_kwargs(tuner.lookup(g, like, family=fam))
            ts = []
            try:
                for _ in range(repeats):
                    r = m.mce_static(dg, rank=rank, **kw)
                    ts.append(r["rank_ms"] + r["build_ms"] + r["enum_ms"])
            except m.MceError as e:  # e.g. a root pivot with too many non-neighbours
                row[rank] = {"error": str(e)}
                continue
            key = (r["count"], r["set_hash"])
            ref = ref or key
            if key != ref:
                raise SystemExit("decomposition %s changed the clique set on %s" % (rank, name))
            row[rank] = {"device_ms": _median(ts), "rank_ms": r["rank_ms"], "search_nodes": r["nodes_total"],
                         "max_cand": r["max_cand"]}
        row["maximal_cliques"] = ref[0]
        if "device_ms" in row["ttt_root"]:
            row["parmce_over_parttt"] = row["ttt_root"]["device_ms"] / min(
                row[k]["device_ms"] for k in ("degree", "degeneracy", "triangle", "peel") if "device_ms" in row[k])
        log("decompositions %s: %s" % (name, {k: round(v["device_ms"], 1) for k, v in row.items()
                                              if isinstance(v, dict) and "device_ms" in v}))
        out[name] = row
    return out


def serving(m, repeats: int = 3, loads=(0.5, 0.9)):
    """Online IMCE: one session, 200 edge-addition batches; closed loop
    (back to back) repeated, then open-loop Poisson arrivals at fractions of
    the measured closed-loop capacity.  Every run starts from a fresh state
    and must end with the same clique count and set hash."""
    import graphgen as gg
    from paper_2001_11433_amd import serving as sv, tuner
    g = gg.chung_lu(500_000, 2.2, 16, seed=0)
    stream = gg.edge_stream(g, 200, 1000, 5000, seed=2, triadic_fraction=0.5)
    knobs = tuner.lookup_imce(g, family="cl500k")
    launch = tuner.launch_kwargs(knobs)
    out = {"graph": "chung_lu(n=500000, gamma=2.2, mean_degree=16, seed=0); degree rank",
           "stream": "200 batches, rho ~ U{1000..5000} (seed 2), half uniform non-edges, half triadic closures",
           "edges": int(sum(len(a) for a, _ in stream)), "sessions": 1, "launch": knobs}
    finals = set()
    lat = []
    walls = []
    new_del = None
    for i in range(repeats):
        r = sv.replay([g], [stream], slots=1, rate_hz=None, **launch)
        if r["errors"]:
            raise SystemExit("serving errors: %r" % r["errors"][:3])
        reqs = r["requests"]
        finals.add((reqs[-1].result["count"], reqs[-1].result["set_hash"]))
        new_del = (sum(q.result["n_new"] for q in reqs), sum(q.result["n_del"] for q in reqs))
        lat += [q.latency_ms for q in reqs]
        walls.append(r["wall_s"])
        log("serving closed loop %d: p50 %.2f p99 %.2f ms, %.1f batches/s" % (i, r["p50_ms"], r["p99_ms"],
                                                                              r["throughput_batches_per_s"]))
    cap = len(stream) / _median(walls)
    out["closed_loop"] = {"repeats": repeats, "samples": len(lat), "p50_ms": sv.nearest_rank(lat, 50),
                          "p99_ms": sv.nearest_rank(lat, 99), "mean_ms": float(np.mean(lat)),
                          "batches_per_s": cap, "edges_per_s": out["edges"] / _median(walls)}
    out["new_cliques_total"], out["subsumed_cliques_total"] = new_del
    out["open_loop"] = []
    for load in loads:
        r = sv.replay([g], [stream], slots=1, rate_hz=load * cap, seed=3, **launch)
        if r["errors"]:
            raise SystemExit("serving errors: %r" % r["errors"][:3])
        finals.add((r["requests"][-1].result["count"], r["requests"][-1].result["set_hash"]))
        out["open_loop"].append({"load": load, "rate_hz": load * cap, "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
                                 "mean_ms": r["mean_ms"]})
        log("serving open loop %.1f: p50 %.2f p99 %.2f ms" % (load, r["p50_ms"], r["p99_ms"]))
    # two sessions (the same graph, two streams) sharing the GPU, closed loop:
    # a batch of one session is admitted while the other's is on the device
    stream2 = gg.edge_stream(g, 200, 1000, 5000, seed=4, triadic_fraction=0.5)
    r = sv.replay([g, g], [stream, stream2], slots=2, rate_hz=None, **launch)
    if r["errors"]:
        raise SystemExit("serving errors: %r" % r["errors"][:3])
    s0 = [q for q in r["requests"] if q.session == 0]
    finals.add((s0[-1].result["count"], s0[-1].result["set_hash"]))
    out["two_sessions"] = {"streams": "seed 2 and seed 4, 200 batches each", "slots": 2,
                           "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"], "mean_ms": r["mean_ms"],
                           "batches_per_s": r["throughput_batches_per_s"],
                           "max_overlap_sessions": r["max_overlap_sessions"]}
    log("serving two sessions: p50 %.2f p99 %.2f ms, %.1f batches/s" % (r["p50_ms"], r["p99_ms"],
                                                                          r["throughput_batches_per_s"]))
    # pipelined: a batch's search overlaps the previous batch's subsumed pass
    lat, walls = [], []
    for i in range(repeats):
        r = sv.replay([g], [stream], slots=2, rate_hz=None, pipeline=True, **launch)
        if r["errors"]:
            raise SystemExit("serving errors: %r" % r["errors"][:3])
        finals.add((r["requests"][-1].result["count"], r["requests"][-1].result["set_hash"]))
        lat += [q.latency_ms for q in r["requests"]]
        walls.append(r["wall_s"])
    out["pipelined_closed_loop"] = {"repeats": repeats, "window": 2, "p50_ms": sv.nearest_rank(lat, 50),
                                    "p99_ms": sv.nearest_rank(lat, 99), "mean_ms": float(np.mean(lat)),
                                    "batches_per_s": len(stream) / _median(walls)}
    log("serving pipelined: p50 %.2f p99 %.2f ms, %.1f batches/s" % (
        out["pipelined_closed_loop"]["p50_ms"], out["pipelined_closed_loop"]["p99_ms"],
        out["pipelined_closed_loop"]["batches_per_s"]))
    if len(finals) != 1:
        raise SystemExit("serving runs disagree: %r" % finals)
    cnt, h = finals.pop()
    out["final_count"], out["final_set_hash"] = cnt, "%016x" % h
    # deletions (Section 5.3): the stream's batches removed again in reverse
    # order, which must lead back to the starting graph's clique set
    from paper_2001_11433_amd import ImceState
    st = ImceState(g, **launch)
    start = (st.initial["count"], st.initial["set_hash"])
    for a, b in stream:
        st.add(a, b)
    dl = []
    for a, b in reversed(stream):
        r = st.remove(a, b)
        dl.append(r["ms"])
    st.close()
    if (r["count"], r["set_hash"]) != start:
        raise SystemExit("deleting the stream did not restore the starting clique set")
    out["deletions"] = {"batches": len(stream), "p50_ms": sv.nearest_rank(dl, 50), "p99_ms": sv.nearest_rank(dl, 99),
                        "mean_ms": float(np.mean(dl)), "restored_count": start[0],
                        "restored_set_hash": "%016x" % start[1], "note": "device time per deletion batch"}
    log("deletions: p50 %.2f p99 %.2f ms (device)" % (out["deletions"]["p50_ms"], out["deletions"]["p99_ms"]))
    out["p99_update_ms"] = out["closed_loop"]["p99_ms"]
    return out


def calibrate_copy(gib: int = 1, reps: int = 5):
    """A plain device-to-device copy of a known size, for scaling the HBM byte
    counters (FETCH_SIZE, WRITE_SIZE) of a profiler run."""
    import torch
    n = gib << 30
    x = torch.empty(n, dtype=torch.uint8, device="cuda")
    x.fill_(1)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "reps": reps}), flush=True)


def kernel_sources_digest() -> str:
    """Digest of the search kernels' sources, to tie measured counters to a
    kernel version."""
    import hashlib
    h = hashlib.sha1()
    for f in ("enum.hip", "internal.h", "dev.h", "api.hip"):
        with open(os.path.join(ROOT, "paper_2001_11433_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(ops_per_launch):
    """HBM bytes per call of the search from the committed counter summary,
    or None when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_cl1m_communities_degree.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_sources") != kernel_sources_digest():
        return None
    return t.get("bytes_per_call")


def measured_issue():
    """Scalar and vector instruction issue of k_compact as fractions of the
    per-CU issue ceiling, from the committed SQ counter summary, or None when
    the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "sq_cl1m_communities_degree.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_sources") != kernel_sources_digest():
        return None
    k = t["per_kernel"]["k_compact"]
    return {"kernel": "k_compact", "salu_frac": k["salu_frac"], "valu_frac": k["valu_frac"],
            "peak_per_s": t["peak_issue_per_s"], "unit": "wave instructions/s per class (SQ_INSTS_SALU, SQ_INSTS_VALU)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl-communities", choices=["cl-communities", "rmat", "er", "cl"])
    ap.add_argument("--scale", type=int, default=14)
    ap.add_argument("--sched", default="degree")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-ownership", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-rmat-family", action="store_true")
    ap.add_argument("--learned-family", default="rmat15",
                    help="graph family of the learned-scheduling comparison: rmat<scale> or cl1m-communities")
    ap.add_argument("--learned-out", default=None,
                    help="run only the learned-scheduling comparison and write its JSON here")
    ap.add_argument("--calibrate-copy", action="store_true", help="only run a 1 GiB device copy (counter scaling)")
    ap.add_argument("--print-digest", action="store_true", help="print the search kernels' source digest and exit")
    args = ap.parse_args()
    if args.print_digest:
        print(kernel_sources_digest())
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    pre = None
    if (not args.no_learned or args.learned_out) and args.learned_family == "cl1m-communities":
        # before anything touches the GPU: the pool forks
        log("generating the %s graphs" % args.learned_family)
        pre = pregenerate(args.learned_family, list(range(1, 13)))
    import torch
    import paper_2001_11433_amd as m
    if not torch.cuda.is_available():
        raise SystemExit("no GPU")
    if args.learned_out:
        r = learned_sched(m, args.learned_family, range(1, 11), (11, 12), graphs=pre)
        with open(args.learned_out, "w") as f:
            json.dump(r, f, indent=1)
        log("learned gain vs degree (whole call):", r["gain_vs_degree"])
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    log("generating workload", args.workload)
    g, rank, desc = make_workload(args.workload, args.scale)
    info = g.describe()
    log("graph:", {k: info[k] for k in ("n", "m", "max_degree")})
    dg = m.DeviceGraph.from_graph(g)
    stream = torch.cuda.current_stream()
    from paper_2001_11433_amd import tuner
    family = {"cl-communities": "cl1m-communities", "rmat": "rmat%d" % args.scale, "cl": "cl500k"}.get(args.workload)
    knobs = tuner.lookup(g, rank, family=family)
    launch = tuner.launch_kwargs(knobs)
    log("launch settings:", knobs)

    for i in range(args.warmup):
        r = m.mce_static(dg, rank=rank, sched=args.sched, stream=stream, **launch)
        log("warmup %d: %d cliques, enum %.1f ms" % (i, r["count"], r["enum_ms"]))
    torch.cuda.synchronize()
    res = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        res.append(m.mce_static(dg, rank=rank, sched=args.sched, stream=stream, **launch))
        log("step %d: %d cliques, enum %.1f ms" % (i, res[-1]["count"], res[-1]["enum_ms"]))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if len({(r["count"], r["set_hash"], r["nodes_total"]) for r in res}) != 1:
        raise SystemExit("steps disagree: %r" % [(r["count"], r["set_hash"]) for r in res])
    r0 = res[0]
    enum_s = np.mean([r["enum_ms"] for r in res]) / 1e3
    achieved = r0["alg_ops"] / enum_s
    out = {
        "metric": METRIC,
        "value": r0["count"] * args.steps / el,
        "unit": "maximal cliques/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": desc, "n": info["n"], "m": info["m"], "rank": rank, "sched": args.sched,
                   "maximal_cliques": r0["count"], "set_hash": "%016x" % r0["set_hash"],
                   "search_nodes": r0["nodes_total"], "rank_ms": r0["rank_ms"], "build_ms": r0["build_ms"],
                   "enum_ms": r0["enum_ms"], "compact_ms": r0["compact_ms"], "handed_off": r0["handed"],
                   "donated": r0["donated"], "launch": knobs},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": INT32_VALU_PEAK / 1e12,
                     "unit": "Tops/s (int32 VALU lane-ops)", "frac": achieved / INT32_VALU_PEAK,
                     "traffic": measured_traffic(r0["alg_ops"]),
                     "traffic_unit": "bytes per call (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy)",
                     "algorithmic_bytes": r0["arena_bytes"],
                     "algorithmic_bytes_note": "the subproblems' bit rows and ids, each read once",
                     "kernel": "k_enum + k_compact (the enumeration: both launches)",
                     "ops_per_launch": r0["alg_ops"],
                     "issue": measured_issue(),
                     "executed_width": {"achieved": r0["exec_ops"] / enum_s / 1e12,
                                        "frac": r0["exec_ops"] / enum_s / INT32_VALU_PEAK,
                                        "ops_per_launch": r0["exec_ops"],
                                        "note": "the same nodes at the row width the kernels execute (2 words "
                                                "per row for compact nodes)"},
                     "lds": {"achieved": r0["lds_bytes"] / enum_s / 1e9, "peak": LDS_PEAK / 1e9, "unit": "GB/s",
                             "frac": r0["lds_bytes"] / enum_s / LDS_PEAK, "bytes_per_launch": r0["lds_bytes"],
                             "note": "algorithmic: 4 * w * (s + |ext|) per node"}},
    }
    from paper_2001_11433_amd import diagnostics
    hs = m.mce_static(dg, rank=rank, sched=args.sched, size_hist=4097, **launch)
    out["clique_sizes"] = diagnostics.size_distribution(hs["size_hist"])
    if not args.no_rmat_family:
        log("R-MAT family ...")
        out["rmat_family"] = rmat_family(m)
    if not args.no_ownership:
        log("ownership ranks and imbalance ...")
        out["ownership"] = ownership_and_imbalance(m, dg, (r0["count"], r0["set_hash"]), launch, rank)
        out["decompositions"] = decompositions(m)
    if not args.no_learned:
        log("learned scheduling ...")
        out["learned_sched"] = learned_sched(m, args.learned_family, range(1, 11), (11, 12), graphs=pre)
    if not args.no_serving:
        log("serving ...")
        out["serving"] = serving(m)
        out["p99_update_ms"] = out["serving"]["p99_update_ms"]
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(g, rank, args.cpu_seconds)
        out["cpu_baseline_legs"] = cpu_baseline_legs(g, rank, args.cpu_seconds / 2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
