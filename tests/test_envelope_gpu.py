"""The supported envelope at its edges: cliques longer than the search wave's
LDS K list (512 vertices), candidate sets past one 64-bit word per lane (4096)
up to the largest (8192), and new cliques of more than 64 vertices in the
incremental step.

Bar: bit-exact against the oracle (count, set hash, search nodes,
per-subproblem triples, clique sets); where the oracle would take minutes
(K_4097 and beyond) against the closed forms that pin it on small graphs (one
clique, 2n - 1 search nodes under degree rank, the chain of n nodes at
vertex 0).
"""

import numpy as np
import pytest

import graphgen as gg
import oracle as O

pytestmark = pytest.mark.gpu


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


def _check(m, g, rank, cliques=True):
    got = m.mce_static(g, rank=rank, cliques=cliques, per_vertex=True)
    want = O.mce_parmce(g, rank, cliques=cliques, threads=8)
    assert (got["count"], got["set_hash"], got["nodes_total"]) == (want.count, want.set_hash, want.nodes)
    assert np.array_equal(_u64(got["nodes_v"]), want.nodes_v)
    assert np.array_equal(_u64(got["count_v"]), want.count_v)
    assert np.array_equal(_u64(got["hash_v"]), want.hash_v)
    if cliques:
        assert got["cliques"] == want.cliques
    return got


@pytest.mark.parametrize("n", [511, 512, 520, 600, 1000])
def test_complete_graphs_beyond_the_lds_k_list(m, n):
    print("K_%d" % n, flush=True)
    got = _check(m, gg.complete(n), "degree")
    assert got["count"] == 1 and got["nodes_total"] == 2 * n - 1


# vertex 0 has n - 1 candidates: the largest set of one word per lane (4096)
# and the smallest of two (the largest supported set, 8192, is the hub's below)
@pytest.mark.parametrize("n", [4097, 4098])
def test_complete_graph_up_to_the_candidate_limit(m, n):
    print("K_%d" % n, flush=True)
    g = gg.complete(n)
    got = m.mce_static(g, rank="degree", cliques=True, per_vertex=True)
    assert got["max_cand"] == n - 1
    assert (got["count"], got["set_hash"], got["nodes_total"]) == (1, O.clique_hash(range(n)), 2 * n - 1)
    assert got["cliques"] == [tuple(range(n))]
    nodes = _u64(got["nodes_v"])
    assert nodes[0] == n and (nodes[1:] == 1).all()


def test_candidate_set_above_the_limit_is_rejected(m):
    import paper_2001_11433_amd as mod
    with pytest.raises(mod.MceError) as e:
        m.mce_static(gg.complete(8194), rank="degree")
    assert e.value.code == -5  # MCE_ENOTSUP


def _hub(n, p, k, seed=51):
    """ER(n, p) on vertices 1..n plus vertex 0 adjacent to k of them: vertex 0
    has degree exactly k, the largest, and the smallest id."""
    base = gg.er(n, p, seed=seed)
    u0, v0 = gg.edges_of(base)
    nb = np.sort(np.random.default_rng(seed + 1).choice(n, k, replace=False)) + 1
    return gg.csr_from_edges(n + 1, np.concatenate([u0 + 1, np.zeros(k, dtype=u0.dtype)]),
                             np.concatenate([v0 + 1, nb.astype(v0.dtype)]))


@pytest.mark.parametrize("kw", [{}, {"donate_interval": 1, "waves_per_cu": 16}], ids=["default", "donation"])
def test_two_word_candidate_set_in_the_ttt_root_split(m, kw):
    # the root's pivot is the hub; its child has the hub's 7000 neighbours as cand
    g = _hub(8000, 0.0012, 7000)
    print("hub 7000, ttt_root", kw, flush=True)
    got = m.mce_static(g, rank="ttt_root", **kw)
    assert got["max_cand"] == 7000
    want = O.mce_root(g)
    assert (got["count"], got["set_hash"], got["nodes_total"]) == want


def test_two_word_candidate_set_under_degeneracy_rank(m):
    # the hub shares the core number of most of its neighbours and has the
    # smallest id, so it owns them: a subproblem of about 6000 candidates
    g = _hub(8000, 0.0012, 7000)
    print("hub 7000, degeneracy", flush=True)
    got = _check(m, g, "degeneracy")
    assert got["max_cand"] > 4096


def test_two_word_root_split(m):
    # the hub's subproblem dominates the cost and is dealt out at launch
    import torch
    g = _hub(8000, 0.0012, 7000)
    want = O.mce_parmce(g, "degeneracy", threads=8)
    cost = torch.from_numpy(np.log(want.nodes_v.astype(np.float64) + 1.0).astype(np.float32)).cuda()
    print("hub 7000, degeneracy, split 64", flush=True)
    got = m.mce_static(g, rank="degeneracy", sched="cost", cost=cost, split=64, waves_per_cu=4, per_vertex=True)
    assert (got["count"], got["set_hash"], got["nodes_total"]) == (want.count, want.set_hash, want.nodes)
    assert np.array_equal(_u64(got["nodes_v"]), want.nodes_v)
    assert got["donated"] > 0


def test_ttt_root_at_the_candidate_limit(m):
    g = _hub(9000, 0.001, 8192)
    print("hub 8192, ttt_root", flush=True)
    got = m.mce_static(g, rank="ttt_root")
    assert got["max_cand"] == 8192
    assert (got["count"], got["set_hash"], got["nodes_total"]) == O.mce_root(g)


def test_ttt_root_above_the_limit_is_rejected(m):
    import paper_2001_11433_amd as mod
    with pytest.raises(mod.MceError) as e:
        m.mce_static(_hub(9000, 0.001, 8193), rank="ttt_root")
    assert e.value.code == -5  # MCE_ENOTSUP


@pytest.mark.parametrize("rank", ["degree", "degeneracy", "triangle", "peel"])
def test_large_clique_planted_in_a_sparse_graph(m, rank):
    base = gg.er(3000, 0.002, seed=41)
    rng = np.random.default_rng(42)
    members = np.sort(rng.choice(base.n, 600, replace=False))
    iu, ju = np.triu_indices(600, 1)
    u0, v0 = gg.edges_of(base)
    g = gg.csr_from_edges(base.n, np.concatenate([u0, members[iu]]), np.concatenate([v0, members[ju]]))
    print("planted 600-clique", rank, flush=True)
    got = _check(m, g, rank)
    assert max(len(c) for c in got["cliques"]) >= 600


def _complete_minus(n, a, b):
    iu, ju = np.triu_indices(n, 1)
    keep = ~((iu == a) & (ju == b))
    return gg.csr_from_edges(n, iu[keep], ju[keep])


@pytest.mark.parametrize("n", [65, 70, 600])
def test_incremental_new_clique_above_64_vertices(m, n):
    # K_n minus one edge, then the edge: one new clique (all n vertices) that
    # subsumes the two maximal cliques of K_n - e (each misses one end)
    print("K_%d - e + e" % n, flush=True)
    g = _complete_minus(n, 0, n - 1)
    st = m.ImceState(g)
    assert st.initial["count"] == 2
    r = st.add([n - 1], [0], cliques=True, cap_verts=1 << 20)
    ost = O.Imce(g)
    w = ost.add([n - 1], [0], cliques=True)
    assert r["new"] == w["new"] == [tuple(range(n))]
    assert r["del"] == w["del"] == sorted([tuple(range(1, n)), tuple(range(n - 1))])
    for k in ("n_new", "n_del", "hash_new", "hash_del", "count", "set_hash"):
        assert r[k] == w[k], k
    st.close()


def test_incremental_large_clique_with_several_batch_edges(m):
    # K_90 minus a matching of four edges; the batch restores them (together
    # with two edges on a path elsewhere): the new 90-clique splits into 2^4
    # subsets, the 16 maximal cliques of K_90 minus the matching, all
    # subsumed; the chord (n, n+2) closes a triangle and subsumes its two path
    # edges; the chord (n+5, n+9) is a new clique that subsumes nothing
    n = 90
    missing = [(0, 89), (3, 40), (10, 11), (50, 70)]
    iu, ju = np.triu_indices(n, 1)
    keep = np.ones(iu.size, bool)
    for a, b in missing:
        keep &= ~((iu == a) & (ju == b))
    extra_u = np.arange(n, n + 30)
    g = gg.csr_from_edges(n + 31, np.concatenate([iu[keep], extra_u]), np.concatenate([ju[keep], extra_u + 1]))
    src = [b for a, b in missing] + [n, n + 5]
    dst = [a for a, b in missing] + [n + 2, n + 9]
    st = m.ImceState(g)
    ost = O.Imce(g)
    r = st.add(src, dst, cliques=True, cap_verts=1 << 20)
    w = ost.add(src, dst, cliques=True, check_form=True)
    assert r["new"] == w["new"] and r["del"] == w["del"]
    assert len(w["del"]) == 16 + 2 and tuple(range(n)) in w["new"]
    assert (n, n + 1) in w["del"] and (n + 1, n + 2) in w["del"] and (n + 5, n + 9) in w["new"]
    for k in ("n_new", "n_del", "hash_new", "hash_del", "count", "set_hash"):
        assert r[k] == w[k], k
    st.close()
