"""Pins for the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against the definition of a maximal clique
(Section 1), closed forms (Moon-Moser, complete multipartite, complete,
edgeless, cycle), the paper's worked IMCE examples (Section 5), invariants of
the decomposition (Algorithm 4: each clique is found by its lowest-rank
vertex), textbook definitions of the rank metrics, and published splitmix64
output values for the hash.
"""

import itertools
import json
import math
import os

import numpy as np
import pytest

import graphgen as gg
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RANKS = ("degree", "degeneracy", "triangle", "peel")


# --------------------------------------------------------------------------
# hash

def test_mix64_matches_published_splitmix64_outputs():
    # splitmix64 seeded with 0: first output 0xe220a8397b1dcdaf; seeded with
    # 1234567: 6457827717110365317, 3203168211198807973, ... (published test
    # vectors of the generator; the state advances by the golden gamma)
    G = 0x9E3779B97F4A7C15
    M = (1 << 64) - 1
    assert O.mix64(0) == 0xE220A8397B1DCDAF
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [O.mix64((1234567 + i * G) & M) for i in range(5)] == want


def _splitmix64_finaliser(x):
    # splitmix64's output step, written from its published definition (add the
    # golden gamma, then xor-shift 30 / multiply / xor-shift 27 / multiply /
    # xor-shift 31), independent of the oracle's code
    M = (1 << 64) - 1
    z = (x + 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def test_clique_hash_composition_by_hand():
    # hc(c) = mix(sum_{v in c} mix(v) + |c| * G) mod 2^64 (the set hash's
    # per-clique term).  The Python finaliser is first tied to the published
    # splitmix64 outputs, then composed by hand for an empty set, a singleton
    # and a triangle; literal values guard the composition itself.
    G = 0x9E3779B97F4A7C15
    M = (1 << 64) - 1
    f = _splitmix64_finaliser
    assert f(0) == 0xE220A8397B1DCDAF
    assert [f((1234567 + i * G) & M) for i in range(3)] == [6457827717110365317, 3203168211198807973,
                                                           9817491932198370423]
    # empty set: no vertex terms and |c| = 0, so hc is the generator's first output from seed 0
    assert O.lib().orc_clique_hash(None, 0) == 0xE220A8397B1DCDAF
    single = f((f(1234567) + G) & M)
    assert single == f((6457827717110365317 + G) & M)
    assert O.clique_hash([1234567]) == single
    tri = f((f(1) + f(2) + f(3) + 3 * G) & M)
    assert O.clique_hash([3, 1, 2]) == tri
    assert (single, tri) == (0xB49A95E7EB5B2DB7, 0x0770BF84CF6243D9)
    # each part of the composition matters: without the size term, without the
    # outer mix, or with XOR instead of the sum the values differ
    assert O.clique_hash([1, 2, 3]) != f((f(1) + f(2) + f(3)) & M)
    assert O.clique_hash([1, 2, 3]) != (f(1) + f(2) + f(3) + 3 * G) & M
    assert O.clique_hash([1, 2, 3]) != f((f(1) ^ f(2) ^ f(3)) + 3 * G & M)


def test_clique_hash_is_order_free_and_separates_small_families():
    assert O.clique_hash([3, 1, 2]) == O.clique_hash([1, 2, 3])
    seen = {}
    for k in range(1, 4):
        for c in itertools.combinations(range(12), k):
            h = O.clique_hash(c)
            assert h not in seen, (c, seen.get(h))
            seen[h] = c


# --------------------------------------------------------------------------
# definition: brute force

def _cliques_by_hand(n, edges):
    adj = {v: set() for v in range(n)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    out = []
    for k in range(1, n + 1):
        for s in itertools.combinations(range(n), k):
            if all(b in adj[a] for a, b in itertools.combinations(s, 2)):
                if not any(all(w in adj[x] for x in s) for w in range(n) if w not in s):
                    out.append(s)
    return sorted(out)


@pytest.mark.parametrize("n,edges,expect", [
    (3, [(0, 1), (1, 2), (0, 2)], [(0, 1, 2)]),
    (3, [(0, 1), (1, 2)], [(0, 1), (1, 2)]),
    (4, [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3)], [(0, 1, 2), (0, 1, 3)]),
    (3, [], [(0,), (1,), (2,)]),
    (5, [(0, 1), (2, 3)], [(0, 1), (2, 3), (4,)]),
])
def test_brute_force_on_hand_checked_graphs(n, edges, expect):
    g = gg.from_edge_list(n, edges)
    cnt, h, cl = O.mce_brute(g, cliques=True)
    assert cl == expect
    assert cnt == len(expect)
    assert h == sum(O.clique_hash(c) for c in expect) % (1 << 64)


def test_brute_force_matches_python_definition():
    rng = np.random.default_rng(7)
    for t in range(40):
        n = int(rng.integers(1, 9))
        p = float(rng.random())
        g = gg.er(n, p, seed=100 + t)
        u, v = gg.edges_of(g)
        assert O.mce_brute(g, cliques=True)[2] == _cliques_by_hand(n, list(zip(u.tolist(), v.tolist())))


def test_empty_graph_has_no_cliques():
    g = gg.edgeless(0)
    assert O.mce_brute(g)[:2] == (0, 0)
    assert O.mce_root(g)[:2] == (0, 0)
    r = O.mce_parmce(g)
    assert (r.count, r.set_hash) == (0, 0)


def test_ttt_and_parmce_equal_brute_force_on_random_small_graphs():
    rng = np.random.default_rng(11)
    for t in range(400):
        n = int(rng.integers(1, 19))
        p = float(rng.choice([0.1, 0.3, 0.5, 0.7, 0.9, rng.random()]))
        g = gg.er(n, p, seed=t)
        cnt, h, cl = O.mce_brute(g, cliques=True)
        c2, h2, _, cl2 = O.mce_root(g, cliques=True)
        assert (c2, h2, cl2) == (cnt, h, cl)
        for rk in RANKS:
            r = O.mce_parmce(g, rk, cliques=True)
            assert (r.count, r.set_hash) == (cnt, h)
            assert r.cliques == cl


# --------------------------------------------------------------------------
# closed forms

def _moon_moser_count(n):
    if n % 3 == 0:
        return 3 ** (n // 3)
    if n % 3 == 1:
        return 4 * 3 ** ((n - 4) // 3)
    return 2 * 3 ** ((n - 2) // 3)


@pytest.mark.parametrize("n", list(range(2, 31)) + [33, 36])
def test_moon_moser_count(n):
    g = gg.moon_moser(n)
    want = _moon_moser_count(n) if n >= 4 or n % 3 != 1 else 1
    assert O.mce_root(g)[0] == want
    assert O.mce_parmce(g, "degree").count == want


def test_complete_multipartite_cliques_are_the_transversals():
    for sizes in ([1], [2, 3], [3, 1, 2], [4, 4, 1, 2], [5, 3, 2, 2]):
        g = gg.complete_multipartite(sizes)
        parts, off = [], 0
        for s in sizes:
            parts.append(list(range(off, off + s)))
            off += s
        transversals = sorted(tuple(sorted(t)) for t in itertools.product(*parts))
        want_h = sum(O.clique_hash(t) for t in transversals) % (1 << 64)
        c, h, _, cl = O.mce_root(g, cliques=True)
        assert c == math.prod(sizes) and cl == transversals and h == want_h
        for rk in RANKS:
            r = O.mce_parmce(g, rk)
            assert (r.count, r.set_hash) == (c, want_h)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 40, 100])
def test_complete_graph_one_clique_and_node_count(n):
    g = gg.complete(n)
    r = O.mce_parmce(g, "degree")
    assert r.count == 1 and r.set_hash == O.clique_hash(range(n))
    # degree ranking on K_n: vertex 0 walks a chain of n nodes; every other
    # vertex has a fini vertex adjacent to all of cand, so one node each.
    assert r.nodes == 2 * n - 1


@pytest.mark.parametrize("k", [2, 3, 17, 200])
@pytest.mark.parametrize("rank", ["degree", "degeneracy"])
def test_star_node_count(k, rank):
    # star with centre 0 and k leaves.  Degree rank: each leaf owns its edge
    # (root with cand = {centre}, then the leaf K = {leaf, centre}: 2 nodes)
    # and the centre's cand is empty (1 dead-end node).  Degeneracy rank (all
    # core numbers 1, ties by id): the centre owns everything (root + k leaf
    # children, the pivot is a leaf with t = 0 so ext = all leaves) and each
    # leaf has an empty cand (1 node).  Either way 2k + 1 nodes, k cliques.
    g = gg.star(k + 1)
    r = O.mce_parmce(g, rank)
    assert r.count == k
    assert r.nodes == 2 * k + 1


@pytest.mark.parametrize("n", [1, 5, 64])
def test_edgeless_graph_singletons(n):
    g = gg.edgeless(n)
    r = O.mce_parmce(g, "degree")
    assert r.count == n and r.nodes == n
    assert r.set_hash == sum(O.clique_hash([v]) for v in range(n)) % (1 << 64)


@pytest.mark.parametrize("n", [4, 5, 9, 50])
def test_cycle_cliques_are_its_edges(n):
    g = gg.cycle(n)
    c, h, _, cl = O.mce_root(g, cliques=True)
    assert cl == sorted(tuple(sorted((i, (i + 1) % n))) for i in range(n))


def test_disjoint_union_adds_and_relabelling_maps():
    a = gg.er(14, 0.5, seed=3)
    b = gg.er(11, 0.6, seed=4)
    u = gg.disjoint_union(a, b)
    ca, _, _, cla = O.mce_root(a, cliques=True)
    cb, _, _, clb = O.mce_root(b, cliques=True)
    cu, hu, _, clu = O.mce_root(u, cliques=True)
    assert cu == ca + cb
    assert clu == sorted(cla + [tuple(x + a.n for x in c) for c in clb])
    perm = np.random.default_rng(5).permutation(u.n)
    cr, _, _, clr = O.mce_root(gg.relabel(u, perm), cliques=True)
    assert clr == sorted(tuple(sorted(int(perm[x]) for x in c)) for c in clu)


def test_er_clique_count_near_expectation():
    # E|C| for G(n,p) = sum_k C(n,k) p^C(k,2) (1-p^k)^(n-k)
    n, p = 2000, 0.01
    e = sum(math.comb(n, k) * p ** math.comb(k, 2) * (1 - p ** k) ** (n - k) for k in range(1, 8))
    c = O.mce_root(gg.er(n, p, 0))[0]
    assert abs(c - e) / e < 0.03


# --------------------------------------------------------------------------
# decomposition (Algorithm 4)

def test_each_clique_is_found_by_its_lowest_rank_vertex():
    for seed in range(6):
        g = gg.er(40, 0.25, seed=seed)
        cl = O.mce_root(g, cliques=True)[3]
        for rk in RANKS:
            m = O.rank_metric(g, rk)
            r = O.mce_parmce(g, rk)
            owners = np.zeros(g.n, dtype=np.int64)
            for c in cl:
                owners[min(c, key=lambda v: (int(m[v]), v))] += 1
            assert np.array_equal(owners, r.count_v.astype(np.int64))
            assert int(r.count_v.sum()) == len(cl)


def test_subset_of_subproblems_matches_full_run():
    g = gg.er(300, 0.05, seed=9)
    full = O.mce_parmce(g, "degeneracy")
    sel = np.array([5, 17, 100, 299, 3], dtype=np.uint32)
    part = O.mce_parmce(g, "degeneracy", verts=sel)
    assert np.array_equal(part.nodes_v, full.nodes_v[sel])
    assert np.array_equal(part.count_v, full.count_v[sel])
    assert np.array_equal(part.hash_v, full.hash_v[sel])


def test_threads_do_not_change_results():
    g = gg.rmat(9, seed=3)
    a = O.mce_parmce(g, "degeneracy", threads=1)
    b = O.mce_parmce(g, "degeneracy", threads=4)
    assert (a.count, a.set_hash, a.nodes) == (b.count, b.set_hash, b.nodes)
    assert np.array_equal(a.nodes_v, b.nodes_v)


# --------------------------------------------------------------------------
# rank metrics (Section 4.2)

def _k_core_numbers(g):
    n = g.n
    adj = [set(g.neighbors(v).tolist()) for v in range(n)]
    core = np.zeros(n, dtype=np.int64)
    k = 0
    alive = set(range(n))
    while alive:
        # the k-core: repeatedly delete vertices of degree < k
        sub = set(alive)
        changed = True
        while changed:
            changed = False
            for v in list(sub):
                if len(adj[v] & sub) < k:
                    sub.discard(v)
                    changed = True
        for v in sub:
            core[v] = k
        alive = sub
        k += 1
    return core


def test_rank_metrics_match_definitions():
    for seed in range(4):
        g = gg.er(60, 0.12, seed=seed)
        deg = np.diff(g.row_ptr).astype(np.int64)
        assert np.array_equal(O.rank_metric(g, "degree").astype(np.int64), deg)
        assert np.array_equal(O.rank_metric(g, "degeneracy").astype(np.int64), _k_core_numbers(g))
        A = np.zeros((g.n, g.n), dtype=np.int64)
        u, v = gg.edges_of(g)
        A[u, v] = 1
        A[v, u] = 1
        tri = np.diag(A @ A @ A) // 2
        assert np.array_equal(O.rank_metric(g, "triangle").astype(np.int64), tri)


# Peel rounds: closed forms on paths, cycles and stars.
@pytest.mark.parametrize("n", [1, 2, 3, 4, 9, 40])
def test_peel_rounds_on_paths_cycles_stars(n):
    path = gg.path(n)
    assert list(O.rank_metric(path, "peel")) == [min(i, n - 1 - i) for i in range(n)]
    if n >= 3:
        cyc = gg.cycle(n)
        assert list(O.rank_metric(cyc, "peel")) == [0] * n
    if n >= 3:
        star = gg.star(n)
        assert list(O.rank_metric(star, "peel")) == [1] + [0] * (n - 1)


def test_peel_rounds_invariants():
    rng = np.random.default_rng(5)
    for seed in range(12):
        n = int(rng.integers(5, 70))
        g = gg.er(n, float(rng.choice([0.05, 0.15, 0.4])), seed=seed)
        r = O.rank_metric(g, "peel").astype(np.int64)
        deg = np.diff(g.row_ptr).astype(np.int64)
        # the first round takes exactly the vertices of minimum degree
        assert set(np.flatnonzero(r == 0)) == set(np.flatnonzero(deg == deg.min()))
        # rounds do not depend on vertex ids: relabel and compare
        perm = rng.permutation(n)
        h = gg.relabel(g, perm)
        rh = O.rank_metric(h, "peel").astype(np.int64)
        assert np.array_equal(rh[perm], r)
        # Eppstein's bound: neighbours later in (round, id) number at most the
        # core number
        core = _k_core_numbers(g)
        for x in range(n):
            nb = g.col[g.row_ptr[x]:g.row_ptr[x + 1]]
            later = sum(1 for w in nb if (r[w], w) > (r[x], x))
            assert later <= core[x]


# --------------------------------------------------------------------------
# IMCE (Section 5)

def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _as_ids(fx, items):
    if "vertices" in fx:
        m = fx["vertices"]
        return [tuple(sorted(m[x] for x in it)) for it in items]
    return [tuple(sorted(it)) for it in items]


@pytest.mark.parametrize("name", ["fig3_imce.json", "cut_figure_imce.json"])
def test_imce_worked_examples(name):
    fx = _load(name)
    edges = _as_ids(fx, fx["edges"])
    g = gg.from_edge_list(fx["n"], edges)
    st = O.Imce(g)
    c, h, cl = st.snapshot(cliques=True)
    assert cl == sorted(_as_ids(fx, fx["initial_cliques"]))
    for b in fx["batches"]:
        add = _as_ids(fx, b["add"])
        r = st.add([a for a, _ in add], [x for _, x in add], cliques=True, check_form=True)
        assert r["new"] == sorted(_as_ids(fx, b["new"]))
        assert r["del"] == sorted(_as_ids(fx, b["subsumed"]))


@pytest.mark.parametrize("n", [3, 5, 12, 30])
def test_imce_complete_minus_one_edge(n):
    iu, ju = np.triu_indices(n, 1)
    keep = ~((iu == 0) & (ju == n - 1))
    g = gg.csr_from_edges(n, iu[keep], ju[keep])
    st = O.Imce(g)
    r = st.add([0], [n - 1], cliques=True, check_form=True)
    assert r["new"] == [tuple(range(n))]
    assert r["del"] == sorted([tuple(range(1, n)), tuple(range(n - 1))])
    assert (r["n_new"], r["n_del"]) == (1, 2)


@pytest.mark.parametrize("k", [2, 3, 5, 7])
def test_imce_moon_moser_plus_one_edge(k):
    g = gg.moon_moser(3 * k)
    st = O.Imce(g)
    r = st.add([0], [1], check_form=True)  # two vertices of the first part
    assert (r["n_new"], r["n_del"]) == (3 ** (k - 1), 2 * 3 ** (k - 1))
    assert r["count"] == 3 ** k - 3 ** (k - 1)


def test_imce_batch_canonicalisation():
    g = gg.from_edge_list(6, [(0, 1), (1, 2)])
    st = O.Imce(g)
    with pytest.raises(ValueError):
        st.add([0], [0])
    with pytest.raises(ValueError):
        st.add([0], [9])
    assert st.snapshot()[0] == 5  # state unchanged by rejected batches
    r = st.add([1, 2, 0, 3], [0, 1, 2, 4])  # (1,0) (2,1) exist; (0,2) new; (3,4) new
    assert (r["n_applied"], r["n_skipped"]) == (2, 2)
    r = st.add([4, 3, 3], [3, 4, 5])  # (4,3) exists, (3,4) exists, (3,5) new
    assert (r["n_applied"], r["n_skipped"]) == (1, 2)
    r = st.add([], [])
    assert (r["n_applied"], r["n_new"], r["n_del"]) == (0, 0, 0)


# --------------------------------------------------------------------------
# decremental step (Section 5.3): deletions by reduction to additions

@pytest.mark.parametrize("name", ["fig3_imce.json", "cut_figure_imce.json"])
def test_deletion_undoes_the_worked_examples(name):
    # replay the example forwards, then delete its batches in reverse order:
    # each deletion removes exactly the batch's new cliques and restores
    # exactly the cliques it had subsumed, back to the initial clique set
    fx = _load(name)
    g = gg.from_edge_list(fx["n"], _as_ids(fx, fx["edges"]))
    st = O.Imce(g)
    start = st.snapshot(cliques=True)
    for b in fx["batches"]:
        add = _as_ids(fx, b["add"])
        st.add([a for a, _ in add], [x for _, x in add])
    for b in reversed(fx["batches"]):
        rem = _as_ids(fx, b["add"])
        r = st.remove([x for _, x in rem], [a for a, _ in rem], cliques=True)
        assert r["del"] == sorted(_as_ids(fx, b["new"]))
        assert r["new"] == sorted(_as_ids(fx, b["subsumed"]))
    assert st.snapshot(cliques=True) == start


@pytest.mark.parametrize("n", [3, 5, 12, 30])
def test_deletion_from_a_complete_graph(n):
    # K_n minus one edge: the one clique goes, the two cliques missing one end come
    st = O.Imce(gg.complete(n))
    r = st.remove([n - 1], [0], cliques=True)
    assert r["del"] == [tuple(range(n))]
    assert r["new"] == sorted([tuple(range(1, n)), tuple(range(n - 1))])
    assert (r["n_new"], r["n_del"], r["count"]) == (2, 1, 2)


@pytest.mark.parametrize("k", [2, 3, 5])
def test_deletion_from_moon_moser(k):
    # K_{3,...,3} minus an edge between two parts: the 3^(k-2) transversals
    # through both ends go, and nothing new is maximal (each leftover extends
    # by the removed end's part mates)
    st = O.Imce(gg.moon_moser(3 * k))
    r = st.remove([0], [3])  # vertex 0 of part 0, vertex 3 of part 1
    assert (r["n_del"], r["n_new"]) == (3 ** (k - 2), 0)
    assert r["count"] == 3 ** k - 3 ** (k - 2)


def test_deletion_canonicalisation():
    g = gg.from_edge_list(6, [(0, 1), (1, 2), (3, 4)])
    st = O.Imce(g)
    before = st.snapshot()
    with pytest.raises(ValueError):
        st.remove([0], [0])
    with pytest.raises(ValueError):
        st.remove([0], [9])
    assert st.snapshot() == before  # state unchanged by rejected batches
    r = st.remove([1, 0, 2, 4, 5], [0, 1, 0, 3, 0])  # (1,0) once, repeat, two non-edges, (4,3)
    assert (r["n_applied"], r["n_skipped"]) == (2, 3)
    r = st.remove([], [])
    assert (r["n_applied"], r["n_new"], r["n_del"]) == (0, 0, 0)


def test_deletion_streams_equal_recompute_and_diff():
    for seed in range(10):
        n = 12 + seed * 2
        g = gg.er(n, 0.25 + 0.02 * seed, seed=seed)
        st = O.Imce(g)
        cur = g
        for s, d in gg.deletion_stream(g, 4, 1, 8, seed=70 + seed, junk_fraction=0.3):
            nxt = gg.remove_edges(cur, s, d)
            want_new, want_del = _recompute_diff(cur, nxt)
            r = st.remove(s, d, cliques=True)
            assert r["new"] == want_new and r["del"] == want_del
            assert (r["count"], r["set_hash"]) == O.mce_root(nxt)[:2]
            cur = nxt


def test_deletion_of_an_added_batch_is_its_inverse():
    for seed in range(8):
        g = gg.er(40, 0.12, seed=200 + seed)
        st = O.Imce(g)
        for s, d in gg.edge_stream(g, 3, 2, 10, seed=300 + seed):
            before = st.snapshot()
            a = st.add(s, d, cliques=True)
            r = st.remove(d, s, cliques=True)
            assert r["del"] == a["new"] and r["new"] == a["del"]
            assert (r["n_applied"], r["hash_new"], r["hash_del"]) == (a["n_applied"], a["hash_del"], a["hash_new"])
            assert st.snapshot() == before
            st.add(s, d)


def _recompute_diff(g_old, g_new):
    old = set(O.mce_root(g_old, cliques=True)[3])
    new = set(O.mce_root(g_new, cliques=True)[3])
    return sorted(new - old), sorted(old - new)


def test_imce_random_streams_equal_recompute_and_diff():
    for seed in range(12):
        n = 12 + seed * 2
        g = gg.er(n, 0.15 + 0.02 * seed, seed=seed)
        st = O.Imce(g)
        stream = gg.edge_stream(g, 4, 1, 6, seed=50 + seed)
        cur = g
        for s, d in stream:
            nxt = gg.add_edges(cur, s, d)
            want_new, want_del = _recompute_diff(cur, nxt)
            r = st.add(s, d, cliques=True, check_form=True)
            assert r["new"] == want_new and r["del"] == want_del
            c, h = st.snapshot()
            c2, h2, _ = O.mce_root(nxt)
            assert (c, h) == (c2, h2)
            cur = nxt


# --------------------------------------------------------------------------
# CSR validity (the input contract of Section 3: simple undirected graphs)

def _raw(n, row_ptr, col):
    return gg.Graph(n, np.asarray(row_ptr, np.uint64), np.asarray(col, np.uint32))


def test_csr_validity_rejects_each_malformation():
    ok = gg.from_edge_list(4, [(0, 1), (1, 2), (2, 3), (0, 3)])
    assert O.csr_valid(ok)
    assert O.csr_valid(gg.edgeless(5))
    # path 0-1-2 written out by hand: row_ptr [0,1,3,4], col [1, 0,2, 1]
    assert O.csr_valid(_raw(3, [0, 1, 3, 4], [1, 0, 2, 1]))
    assert not O.csr_valid(_raw(3, [1, 2, 4, 5], [1, 0, 2, 1]))      # row_ptr[0] != 0 (shifted)
    assert not O.csr_valid(_raw(3, [0, 2, 1, 4], [1, 0, 2, 1]))      # row_ptr decreasing
    assert not O.csr_valid(_raw(3, [0, 1, 3, 4], [1, 2, 0, 1]))      # row 1 unsorted
    assert not O.csr_valid(_raw(3, [0, 1, 3, 4], [1, 0, 0, 1]))      # repeated entry in row 1
    assert not O.csr_valid(_raw(3, [0, 1, 3, 4], [1, 0, 1, 1]))      # self-loop 1-1
    assert not O.csr_valid(_raw(3, [0, 1, 3, 4], [1, 0, 7, 1]))      # id >= n
    assert not O.csr_valid(_raw(3, [0, 1, 2, 3], [1, 0, 1]))         # 1-2 stored on one side only
    assert not O.csr_valid(_raw(3, [0, 1, 3, 3], [1, 0, 2]))         # 1-2 stored on one side only


# --------------------------------------------------------------------------
# clique-size distribution (the per-graph histogram of Section 6.1)

def test_size_histogram_closed_forms_and_brute_force():
    def hist(r):
        return {k: int(c) for k, c in enumerate(r.sizes) if c}
    assert hist(O.mce_parmce(gg.complete(9))) == {9: 1}
    assert hist(O.mce_parmce(gg.edgeless(6))) == {1: 6}
    assert hist(O.mce_parmce(gg.cycle(7))) == {2: 7}
    # Moon-Moser n = 3k: 3^k cliques of size k (one vertex per part)
    assert hist(O.mce_parmce(gg.moon_moser(12))) == {4: 81}
    # complete multipartite: every transversal, of size = number of parts
    assert hist(O.mce_parmce(gg.complete_multipartite([2, 3, 1]))) == {3: 6}
    rng = np.random.default_rng(5)
    for t in range(30):
        n = int(rng.integers(1, 14))
        g = gg.er(n, float(rng.random()), seed=500 + t)
        _, _, cl = O.mce_brute(g, cliques=True)
        want = {}
        for c in cl:
            want[len(c)] = want.get(len(c), 0) + 1
        for rank in RANKS:
            r = O.mce_parmce(g, rank)
            assert hist(r) == want
            assert int(r.sizes.sum()) == r.count
