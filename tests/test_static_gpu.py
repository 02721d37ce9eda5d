"""GPU parity of static MCE (mce_static) against the CPU oracle.

Bar: bit-exact.  Clique sets (small graphs), count, 64-bit set hash, total
search nodes and the per-vertex (nodes, count, hash) triples must equal the
oracle's sequential ParMCE (Algorithm 4 over Algorithm 1) under the same rank.
"""

import numpy as np
import pytest

import graphgen as gg
import oracle as O

pytestmark = pytest.mark.gpu

RANKS = ("degree", "degeneracy", "triangle", "peel")


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


def _check(m, g, rank, cliques=False, **kw):
    got = m.mce_static(g, rank=rank, cliques=cliques, per_vertex=True, **kw)
    want = O.mce_parmce(g, rank, cliques=cliques, threads=8)
    assert got["count"] == want.count, (rank, got["count"], want.count)
    assert got["set_hash"] == want.set_hash
    assert got["nodes_total"] == want.nodes
    assert np.array_equal(_u64(got["nodes_v"]), want.nodes_v)
    assert np.array_equal(_u64(got["count_v"]), want.count_v)
    assert np.array_equal(_u64(got["hash_v"]), want.hash_v)
    if cliques:
        assert got["cliques"] == want.cliques
    return got, want


SMALL = [
    ("K1", lambda: gg.complete(1)),
    ("K2", lambda: gg.complete(2)),
    ("K40", lambda: gg.complete(40)),
    ("edgeless7", lambda: gg.edgeless(7)),
    ("C9", lambda: gg.cycle(9)),
    ("P6", lambda: gg.path(6)),
    ("star50", lambda: gg.star(50)),
    ("moon_moser24", lambda: gg.moon_moser(24)),
    ("multipartite", lambda: gg.complete_multipartite([4, 1, 3, 5, 2])),
    ("union", lambda: gg.disjoint_union(gg.complete(5), gg.edgeless(3))),
]


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("rank", RANKS)
def test_small_families(m, name, make, rank):
    _check(m, make(), rank, cliques=True)


def test_random_small_graphs_full_sets(m):
    rng = np.random.default_rng(3)
    for t in range(60):
        n = int(rng.integers(1, 40))
        p = float(rng.choice([0.05, 0.2, 0.5, 0.8, rng.random()]))
        g = gg.er(n, p, seed=1000 + t)
        _check(m, g, RANKS[t % len(RANKS)], cliques=True)


def test_empty_graph(m):
    got = m.mce_static(gg.edgeless(0), cliques=True)
    assert (got["count"], got["set_hash"], got["cliques"]) == (0, 0, [])


def test_er_2000_degree_rank(m):
    # G(2000, 0.01), seed 0, degree ranking: the small parity configuration
    g = gg.er(2000, 0.01, seed=0)
    got, want = _check(m, g, "degree", cliques=True)
    assert got["count"] == O.mce_root(g)[0]


@pytest.mark.parametrize("scale", [9, 10, 11, 12])
def test_rmat_degeneracy(m, scale):
    # R-MAT (.57,.19,.19,.05), edge factor 16: heavy-tailed subproblems, p > 64
    g = gg.rmat(scale, seed=0)
    got, _ = _check(m, g, "degeneracy")
    assert got["max_cand"] > 64 or scale < 11


def test_wide_subproblems(m):
    # |cand| up to 299 (5 words) with a large fini
    g = gg.disjoint_union(gg.complete(300), gg.er(200, 0.3, seed=4))
    _check(m, g, "degree")
    g = gg.er(150, 0.55, seed=5)
    _check(m, g, "degeneracy")


def test_planted_dense_communities(m):
    base = gg.chung_lu(3000, 2.1, 10, seed=0)
    g = gg.plant_communities(base, count=6, smin=30, smax=45, p=0.9, seed=1)
    _check(m, g, "degree")


@pytest.mark.parametrize("sched", ["degree", "triangle", "id"])
def test_schedule_never_changes_results(m, sched):
    g = gg.rmat(11, seed=2)
    _check(m, g, "degeneracy", sched=sched)


def test_cost_schedule(m):
    import torch
    g = gg.rmat(10, seed=5)
    cost = torch.rand(g.n, device="cuda")
    _check(m, g, "degree", sched="cost", cost=cost)


@pytest.mark.parametrize("split", [2, 64, 4096])
def test_root_split_never_changes_results(m, split):
    # cost = log of the oracle's node counts: the hub's root is far above a
    # wave's share and is dealt out in up to `split` chunks at launch
    import torch
    g = gg.rmat(12, seed=3)
    want = O.mce_parmce(g, "degeneracy", threads=8)
    cost = torch.from_numpy(np.log(want.nodes_v.astype(np.float64) + 1.0).astype(np.float32)).cuda()
    got, _ = _check(m, g, "degeneracy", sched="cost", cost=cost, split=split, waves_per_cu=4)
    assert got["donated"] > 0


def test_root_split_with_extreme_costs(m):
    # any float is accepted: huge, tiny, NaN and infinite predictions
    import torch
    g = gg.rmat(10, seed=6)
    cost = torch.rand(g.n, device="cuda") * 200.0 - 100.0
    cost[::7] = float("nan")
    cost[1::11] = float("inf")
    cost[2::13] = -float("inf")
    _check(m, g, "degeneracy", sched="cost", cost=cost, split=1000)


def test_donation_stress_keeps_node_counts(m):
    g = gg.rmat(11, seed=1)
    _check(m, g, "degeneracy", donate_interval=1, waves_per_cu=16)


def test_repeated_runs_with_heavy_block_recycling(m):
    # Donation records recycle through a lock-free free list; a wrong ordering
    # there lost or duplicated whole donated subtrees only now and then, so
    # the same graph runs several times under different launch shapes.
    g = gg.rmat(12, seed=12)
    want = O.mce_parmce(g, "degeneracy", threads=8)
    dg = m.DeviceGraph.from_graph(g)
    for wpc, iv in ((2, 1), (16, 1), (2, 64), (8, 4), (16, 16), (4, 1), (1, 1), (16, 2)):
        got = m.mce_static(dg, rank="degeneracy", waves_per_cu=wpc, donate_interval=iv)
        assert (got["count"], got["set_hash"], got["nodes_total"]) == (want.count, want.set_hash, want.nodes), \
            (wpc, iv)
        assert got["donated"] > 0


TTT_ROOT_GRAPHS = [
    ("K1", lambda: gg.complete(1)),
    ("K40", lambda: gg.complete(40)),
    ("edgeless7", lambda: gg.edgeless(7)),
    ("C9", lambda: gg.cycle(9)),
    ("star50", lambda: gg.star(50)),
    ("moon_moser24", lambda: gg.moon_moser(24)),
    ("multipartite", lambda: gg.complete_multipartite([4, 1, 3, 5, 2])),
    ("er300", lambda: gg.er(300, 0.08, seed=3)),
    ("rmat10", lambda: gg.rmat(10, seed=2)),
    ("rmat11", lambda: gg.rmat(11, seed=4)),
    ("communities", lambda: gg.plant_communities(gg.chung_lu(3000, 2.1, 10, seed=0), count=6, smin=30, smax=45,
                                                 p=0.9, seed=1)),
]


@pytest.mark.parametrize("name,make", TTT_ROOT_GRAPHS, ids=[x[0] for x in TTT_ROOT_GRAPHS])
def test_whole_graph_ttt_root_split(m, name, make):
    # Algorithm 3 on the root of Algorithm 1: same clique set as Algorithm 1
    # from the root, and the same recursion tree (node count, root included)
    g = make()
    got = m.mce_static(g, rank="ttt_root", cliques=g.n <= 400)
    want = O.mce_root(g, cliques=g.n <= 400)
    assert (got["count"], got["set_hash"], got["nodes_total"]) == tuple(want[:3])
    if g.n <= 400:
        assert got["cliques"] == want[3]


def test_ttt_root_metric_marks_the_pivot_neighbours(m):
    g = gg.rmat(10, seed=8)
    deg = np.diff(np.asarray(g.row_ptr, dtype=np.int64))
    u = int(np.flatnonzero(deg == deg.max())[0])
    want = np.zeros(g.n, dtype=np.uint64)
    want[g.neighbors(u)] = np.uint64(1) << np.uint64(63)
    got = m.mce_rank_metric(g, "ttt_root").cpu().numpy().view(np.uint64)
    assert np.array_equal(got, want)


def test_stack_overflow_retries(m):
    # K_300: 5-word bitsets, too deep for the LDS stack; 4 global frames overflow
    g = gg.complete(300)
    got, _ = _check(m, g, "degree", frame_cap=4)
    assert got["retries"] >= 1


def test_clique_buffer_too_small_reports_sizes(m):
    import ctypes
    import torch
    g = gg.er(60, 0.2, seed=2)
    want = O.mce_parmce(g, "degree", cliques=True)
    dg = m.DeviceGraph.from_graph(g)
    off = torch.zeros(4, dtype=torch.int64, device="cuda")
    vert = torch.zeros(4, dtype=torch.int32, device="cuda")
    buf = m._CliqueBuf(3, 4, off.data_ptr(), vert.data_ptr(), 1, 0, 0)
    res = m._Result()
    csr = dg.csr()
    o = m._opts()
    rc = m.lib().mce_static(ctypes.byref(csr), 0, ctypes.byref(o), ctypes.byref(res), ctypes.byref(buf), None)
    assert rc == m.MCE_ENOSPC
    assert buf.n_cliques == want.count
    assert buf.n_verts == sum(len(c) for c in want.cliques)
    assert res.count == want.count and res.set_hash == want.set_hash


def test_validation_rejects_malformed_csr(m):
    g = gg.er(30, 0.3, seed=1)
    bad = gg.Graph(g.n, g.row_ptr.copy(), g.col.copy())
    bad.col[0], bad.col[1] = bad.col[1], bad.col[0]  # unsorted row
    with pytest.raises(m.MceError) as e:
        m.mce_static(bad, validate=True)
    assert e.value.code == m.MCE_EINVAL
    asym = gg.Graph(3, np.array([0, 1, 1, 1], np.uint64), np.array([1], np.uint32))
    with pytest.raises(m.MceError):
        m.mce_static(asym, validate=True)


def test_host_csr_input_path(m):
    import ctypes
    g = gg.er(200, 0.05, seed=8)
    rp = np.ascontiguousarray(g.row_ptr)
    col = np.ascontiguousarray(g.col)
    csr = m._Csr(g.n, rp.ctypes.data, col.ctypes.data, 0)
    res = m._Result()
    o = m._opts()
    m._check(m.lib().mce_static(ctypes.byref(csr), 1, ctypes.byref(o), ctypes.byref(res), None, None))
    want = O.mce_parmce(g, "degeneracy")
    assert (res.count, res.set_hash, res.nodes_total) == (want.count, want.set_hash, want.nodes)


@pytest.mark.parametrize("rank", RANKS)
def test_rank_metric_kernels(m, rank):
    for g in (gg.rmat(12, seed=3), gg.er(500, 0.02, seed=1), gg.edgeless(5), gg.path(3001), gg.cycle(7)):
        got = _u64(m.mce_rank_metric(g, rank))
        assert np.array_equal(got, O.rank_metric(g, rank))


def test_feature_kernel(m):
    g = gg.rmat(10, seed=4)
    f = m.mce_features(g).cpu().numpy()
    deg = np.diff(g.row_ptr).astype(np.float64)
    core = O.rank_metric(g, "degeneracy").astype(np.float64)
    tri = O.rank_metric(g, "triangle").astype(np.float64)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr).astype(np.int64))
    walks = np.bincount(src, weights=deg[g.col] - 1, minlength=g.n)
    want = np.log1p(np.stack([deg, core, tri, walks], 1))
    assert np.allclose(f, want, rtol=1e-6, atol=1e-6)


HIST_GRAPHS = [
    ("er2000", lambda: gg.er(2000, 0.01, seed=0)),
    ("rmat11", lambda: gg.rmat(11, 16, 0.57, 0.19, 0.19, seed=3)),
    ("communities", lambda: gg.plant_communities(gg.chung_lu(3000, 2.1, 8, seed=5), count=6, smin=30, smax=60,
                                                 p=0.9, seed=6)),
    ("moon_moser24", lambda: gg.moon_moser(24)),
    ("K600+isolated", lambda: gg.disjoint_union(gg.complete(600), gg.edgeless(5))),
]


@pytest.mark.parametrize("name,make", HIST_GRAPHS, ids=[h[0] for h in HIST_GRAPHS])
@pytest.mark.parametrize("rank", ["degree", "degeneracy"])
def test_clique_size_histogram(m, name, make, rank):
    # the distribution of maximal-clique sizes (Section 6.1) against the
    # oracle's, bin by bin; its sum is the clique count
    g = make()
    got = m.mce_static(g, rank=rank, size_hist=O.HIST_LEN)
    want = O.mce_parmce(g, rank, threads=8)
    assert np.array_equal(got["size_hist"], want.sizes)
    assert int(got["size_hist"].sum()) == got["count"] == want.count
    # a short histogram folds every larger size into its last bin
    short = m.mce_static(g, rank=rank, size_hist=4)["size_hist"]
    assert list(short[:3]) == list(want.sizes[:3]) and short[3] == want.sizes[3:].sum()


def test_clique_size_histogram_with_in_place_compact_search(m):
    g = HIST_GRAPHS[2][1]()
    want = O.mce_parmce(g, "degree", threads=8)
    for kw in ({"inline_compact": True}, {"waves_per_cu": 1, "donate_interval": 16}):
        got = m.mce_static(g, rank="degree", size_hist=O.HIST_LEN, cliques=True, **kw)
        assert np.array_equal(got["size_hist"], want.sizes), kw


def test_imbalance_shares_from_gpu_outputs(m):
    # the Figure 2 analog computed from the library's per-subproblem outputs
    # equals the one computed from the oracle's
    from paper_2001_11433_amd import diagnostics as D
    g = gg.rmat(11, 16, 0.57, 0.19, 0.19, seed=3)
    got = m.mce_static(g, rank="degeneracy", per_vertex=True)
    want = O.mce_parmce(g, "degeneracy", threads=8)
    assert D.imbalance(_u64(got["nodes_v"]), _u64(got["count_v"])) == D.imbalance(want.nodes_v, want.count_v)


@pytest.mark.parametrize("words", [256, 1024, 4096])
def test_lds_row_cache_width_classes(m, words):
    # the same subproblems searched with their rows in the LDS row cache when
    # they fit it (a class boundary of `words` 64-bit words) and from device
    # memory when not: identical cliques, hashes and node counts
    for g, rank in ((gg.disjoint_union(gg.complete(300), gg.er(200, 0.3, seed=4)), "degree"),
                    (gg.er(150, 0.55, seed=5), "degeneracy"),
                    (gg.plant_communities(gg.chung_lu(4000, 2.1, 10, seed=8), count=6, smin=70, smax=100, p=0.6,
                                          seed=9), "degree")):
        _check(m, g, rank, cliques=True, lds_row_words=words)
        _check(m, g, rank, lds_row_words=words, waves_per_cu=2, donate_interval=16)


def test_lds_row_cache_in_the_incremental_step(m):
    from paper_2001_11433_amd import serving
    g = gg.plant_communities(gg.chung_lu(5000, 2.2, 12, seed=10), count=5, smin=70, smax=100, p=0.6, seed=11)
    stream = gg.edge_stream(g, 4, 200, 800, seed=12)
    ref = serving.run_alone(g, stream)
    got = serving.run_alone(g, stream, lds_row_words=2048)
    for a, b in zip(ref, got):
        assert [a[k] for k in serving.RESULT_KEYS] == [b[k] for k in serving.RESULT_KEYS]


def test_handoff_budget_overflow_is_searched_in_place(m):
    # a tiny handoff budget (1 MiB): the nodes past it are searched in place by
    # the first kernel; results, node counts and per-subproblem triples are
    # those of the default budget, for static and exclusion-mode searches
    g = gg.plant_communities(gg.chung_lu(200_000, 2.1, 16, seed=21), count=80, smin=30, smax=60, p=0.85, seed=22)
    want = m.mce_static(g, rank="degree", per_vertex=True)
    got = m.mce_static(g, rank="degree", per_vertex=True, hand_mb=1)
    assert (got["count"], got["set_hash"], got["nodes_total"]) == (want["count"], want["set_hash"], want["nodes_total"])
    for k in ("nodes_v", "count_v", "hash_v"):
        assert bool((got[k] == want[k]).all()), k
    assert got["handed"] < want["handed"]
    ref = O.mce_parmce(g, "degree", threads=8)
    assert (got["count"], got["set_hash"], got["nodes_total"]) == (ref.count, ref.set_hash, ref.nodes)
