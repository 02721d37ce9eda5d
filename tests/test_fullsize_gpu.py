"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (the tuned table).

The oracle cannot enumerate these graphs whole in test time, so:
  * the 1M-vertex Chung-Lu + communities graph: the whole graph against the
    oracle's full ParMCE stored by oracle/make_golden.py
    (tests/golden/c3_totals.json: totals, a digest of every per-subproblem
    triple, the heaviest subproblems, the clique-size distribution); and the
    per-subproblem triples (search nodes, cliques, clique-set hash) of a seeded
    sample of vertices against the oracle run in the test;
  * R-MAT scale 14 (degeneracy ownership): the whole graph against the
    oracle's full ParMCE (tests/golden/rmat14_totals.json, same fields);
    scale 15: the sampled per-subproblem check; scale 18: rank metrics (degree, core number, triangles, peel
    rounds) of every vertex against the oracle (its enumeration is far beyond
    reach);
  * the 500k-vertex Chung-Lu stream: all eight result fields of all 200
    batches against the oracle's sequential IMCE (stored by
    oracle/make_golden.py in tests/golden/c5_stream.json); sampled new and
    subsumed cliques of the first batches against the definition of the two
    sets, and the running count and hash against a fresh enumeration.
"""

import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle as O

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def m():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_11433_amd as mod
    mod.lib()
    return mod


def _u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


def test_cl1m_communities_sampled_subproblems(m):
    from paper_2001_11433_amd import tuner
    g = gg.plant_communities(gg.chung_lu(1_000_000, 2.1, 20, seed=0), count=500, smin=30, smax=80, p=0.9, seed=1)
    kw = tuner.launch_kwargs(tuner.lookup(g, "degree", family="cl1m-communities"))
    got = m.mce_static(g, rank="degree", per_vertex=True, **kw)
    nodes, count, hsh = _u64(got["nodes_v"]), _u64(got["count_v"]), _u64(got["hash_v"])
    # totals are the sums of the per-subproblem triples (mod 2^64 for the hash)
    assert int(count.sum()) == got["count"]
    assert int(nodes.sum()) == got["nodes_total"]
    assert int(np.add.reduce(hsh, dtype=np.uint64)) == got["set_hash"]
    # a seeded uniform sample plus the heaviest subproblems the oracle finishes
    # in seconds (the very heaviest take it minutes each)
    rng = np.random.default_rng(11)
    order = np.argsort(nodes)
    heavy = order[nodes[order] <= 5_000_000][-12:]
    sample = np.unique(np.concatenate([rng.choice(g.n, 384, replace=False), heavy])).astype(np.uint32)
    want = O.mce_parmce(g, "degree", verts=sample, threads=8)
    assert np.array_equal(nodes[sample], want.nodes_v)
    assert np.array_equal(count[sample], want.count_v)
    assert np.array_equal(hsh[sample], want.hash_v)


def _digest(*arrays) -> str:
    import hashlib
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype="<u8").tobytes())
    return h.hexdigest()


def test_cl1m_communities_whole_graph_against_the_oracle(m):
    # every subproblem of the benchmark graph, in the tuned launch, against the
    # oracle's full ParMCE (tests/golden/c3_totals.json, oracle/make_golden.py):
    # totals, the per-subproblem triples of all 10^6 vertices (by digest), the
    # heaviest subproblems one by one, and the clique-size distribution
    g = gg.plant_communities(gg.chung_lu(1_000_000, 2.1, 20, seed=0), count=500, smin=30, smax=80, p=0.9, seed=1)
    _whole_graph_against_golden(m, g, "degree", "cl1m-communities", "c3_totals.json")


def _whole_graph_against_golden(m, g, rank, family, name):
    from paper_2001_11433_amd import tuner
    with open(os.path.join(GOLDEN, name)) as f:
        want = json.load(f)
    assert (g.n, g.m) == (want["n"], want["m"])
    kw = tuner.launch_kwargs(tuner.lookup(g, rank, family=family))
    got = m.mce_static(g, rank=rank, per_vertex=True, size_hist=4097, **kw)
    assert got["count"] == want["count"]
    assert "%016x" % got["set_hash"] == want["set_hash"]
    assert got["nodes_total"] == want["nodes_total"]
    nodes, count, hsh = _u64(got["nodes_v"]), _u64(got["count_v"]), _u64(got["hash_v"])
    for v, nv, cv, hv in want["heaviest"]:
        assert (int(nodes[v]), int(count[v]), "%016x" % int(hsh[v])) == (nv, cv, hv), v
    assert _digest(nodes, count, hsh) == want["per_vertex_sha256"]
    hist = {str(k): int(c) for k, c in enumerate(got["size_hist"]) if c}
    assert hist == want["size_hist"]


def test_rmat14_whole_graph_against_the_oracle(m):
    # the R-MAT family under degeneracy ownership, whole graph, against the
    # oracle's full ParMCE (tests/golden/rmat14_totals.json); one subproblem
    # holds most of its search nodes, which donation spreads over the waves
    g = gg.rmat(14, 16, 0.57, 0.19, 0.19, seed=0)
    _whole_graph_against_golden(m, g, "degeneracy", "rmat14", "rmat14_totals.json")


def test_rmat15_sampled_subproblems(m):
    # the largest R-MAT scale whose enumeration a test can wait for (3.4e9
    # cliques; each scale step multiplies them by 22-26), degeneracy ownership,
    # in the tuned launch: totals are the sums of the per-subproblem triples,
    # and a seeded sample plus the heaviest subproblems the oracle finishes in
    # seconds equal the oracle's
    from paper_2001_11433_amd import tuner
    g = gg.rmat(15, 16, 0.57, 0.19, 0.19, seed=0)
    kw = tuner.launch_kwargs(tuner.lookup(g, "degeneracy", family="rmat15"))
    got = m.mce_static(g, rank="degeneracy", per_vertex=True, **kw)
    nodes, count, hsh = _u64(got["nodes_v"]), _u64(got["count_v"]), _u64(got["hash_v"])
    assert int(count.sum()) == got["count"]
    assert int(nodes.sum()) == got["nodes_total"]
    assert int(np.add.reduce(hsh, dtype=np.uint64)) == got["set_hash"]
    rng = np.random.default_rng(15)
    order = np.argsort(nodes)
    heavy = order[nodes[order] <= 5_000_000][-12:]
    sample = np.unique(np.concatenate([rng.choice(g.n, 384, replace=False), heavy])).astype(np.uint32)
    want = O.mce_parmce(g, "degeneracy", verts=sample, threads=8)
    assert np.array_equal(nodes[sample], want.nodes_v)
    assert np.array_equal(count[sample], want.count_v)
    assert np.array_equal(hsh[sample], want.hash_v)


@pytest.mark.parametrize("rank", ["degree", "degeneracy", "triangle", "peel"])
def test_rmat18_rank_metrics(m, rank):
    g = gg.rmat(18, 16, 0.57, 0.19, 0.19, seed=0)
    got = m.mce_rank_metric(g, rank).cpu().numpy().astype(np.uint64)
    want = O.rank_metric(g, rank)
    assert np.array_equal(got, want)


def _adj_sets(g):
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    col = np.asarray(g.col)
    return lambda v: col[rp[v]:rp[v + 1]]


def _is_clique(nb, c):
    return all(np.isin(np.array(c[i + 1:]), nb(c[i])).all() for i in range(len(c) - 1))


def _is_maximal(nb, c):
    # no vertex outside c is adjacent to all of c
    common = set(nb(c[0]).tolist())
    for v in c[1:]:
        common &= set(nb(v).tolist())
        if not common:
            return True
    return not (common - set(c))


def test_cl500k_stream_sampled_cliques_and_recompute(m):
    from paper_2001_11433_amd import tuner
    g = gg.chung_lu(500_000, 2.2, 16, seed=0)
    stream = gg.edge_stream(g, 200, 1000, 5000, seed=2, triadic_fraction=0.5)
    kw = tuner.launch_kwargs(tuner.lookup(g, "degree", family="cl500k"))
    st = m.ImceState(g, **kw)
    rng = np.random.default_rng(5)
    cur = g
    for b in range(3):
        src, dst = stream[b]
        r = st.add(src, dst, cliques=True, cap_cliques=1 << 20, cap_verts=1 << 24)
        new_g = gg.add_edges(cur, src, dst)
        old_nb, new_nb = _adj_sets(cur), _adj_sets(new_g)
        batch = {(min(int(a), int(c)), max(int(a), int(c))) for a, c in zip(src, dst)}
        assert len(r["new"]) == r["n_new"] and len(r["del"]) == r["n_del"]
        for i in rng.choice(len(r["new"]), min(300, len(r["new"])), replace=False):
            c = r["new"][i]
            assert _is_clique(new_nb, c) and _is_maximal(new_nb, c)
            assert any((c[x], c[y]) in batch for x in range(len(c)) for y in range(x + 1, len(c)))
        for i in rng.choice(len(r["del"]), min(300, len(r["del"])), replace=False):
            c = r["del"][i]
            assert _is_clique(old_nb, c) and _is_maximal(old_nb, c)
            assert not _is_maximal(new_nb, c)
        # the incremental count and hash equal a fresh enumeration of G + H
        full = m.mce_static(new_g, rank="degree", **kw)
        assert (full["count"], full["set_hash"]) == (r["count"], r["set_hash"]), b
        cur = new_g
    st.close()


def test_cl500k_stream_every_batch_equals_the_oracle(m):
    # the benchmark's stream in the benchmark's tuned incremental launch: every
    # batch's (applied, skipped, |new|, |subsumed|, H(new), H(subsumed), count,
    # set hash) equals the oracle's, and so does the initial enumeration
    from paper_2001_11433_amd import tuner
    with open(os.path.join(GOLDEN, "c5_stream.json")) as f:
        gold = json.load(f)
    g = gg.chung_lu(500_000, 2.2, 16, seed=0)
    stream = gg.edge_stream(g, 200, 1000, 5000, seed=2, triadic_fraction=0.5)
    kw = tuner.launch_kwargs(tuner.lookup_imce(g, family="cl500k"))
    st = m.ImceState(g, **kw)
    assert (st.initial["count"], "%016x" % st.initial["set_hash"]) == (gold["initial"]["count"],
                                                                         gold["initial"]["set_hash"])
    for b, (src, dst) in enumerate(stream):
        r = st.add(src, dst)
        got = [r[k] if not k.startswith("hash") and k != "set_hash" else "%016x" % r[k] for k in gold["fields"]]
        assert got == gold["batches"][b], (b, got, gold["batches"][b])
    st.close()
