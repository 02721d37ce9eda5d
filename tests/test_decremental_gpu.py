"""GPU parity of the decremental step (imce_remove_edges, the reduction of
Section 5.3) against the CPU oracle's reduction and against recomputation.
Bar: bit-exact sets, counts and hashes after every batch, and the state
unchanged after a rejected batch."""

import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle as O

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
KEYS = ("n_applied", "n_skipped", "n_new", "n_del", "hash_new", "hash_del", "count", "set_hash")


@pytest.fixture(scope="module")
def m():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_11433_amd as mod
    mod.lib()
    return mod


def _as_ids(fx, items):
    if "vertices" in fx:
        mp = fx["vertices"]
        return [tuple(sorted(mp[x] for x in it)) for it in items]
    return [tuple(sorted(it)) for it in items]


@pytest.mark.parametrize("name", ["fig3_imce.json", "cut_figure_imce.json"])
def test_worked_examples_backwards(m, name):
    with open(os.path.join(GOLDEN, name)) as f:
        fx = json.load(f)
    g = gg.from_edge_list(fx["n"], _as_ids(fx, fx["edges"]))
    st = m.ImceState(g)
    start = st.info()
    for b in fx["batches"]:
        add = _as_ids(fx, b["add"])
        st.add([a for a, _ in add], [x for _, x in add])
    for b in reversed(fx["batches"]):
        rem = _as_ids(fx, b["add"])
        r = st.remove([x for _, x in rem], [a for a, _ in rem], cliques=True)
        assert r["del"] == sorted(_as_ids(fx, b["new"]))
        assert r["new"] == sorted(_as_ids(fx, b["subsumed"]))
    assert st.info() == start


@pytest.mark.parametrize("n", [3, 40, 600])
def test_deletion_from_a_complete_graph(m, n):
    st = m.ImceState(gg.complete(n))
    r = st.remove([n - 1], [0], cliques=True, cap_verts=1 << 20)
    assert r["del"] == [tuple(range(n))]
    assert r["new"] == sorted([tuple(range(1, n)), tuple(range(n - 1))])
    assert (r["n_new"], r["n_del"], r["count"]) == (2, 1, 2)
    st.close()


@pytest.mark.parametrize("k", [2, 4, 6])
def test_deletion_from_moon_moser(m, k):
    st = m.ImceState(gg.moon_moser(3 * k))
    r = st.remove([0], [3])
    assert (r["n_del"], r["n_new"], r["count"]) == (3 ** (k - 2), 0, 3 ** k - 3 ** (k - 2))
    st.close()


def test_canonicalisation_and_atomic_rejection(m):
    import paper_2001_11433_amd as mod
    g = gg.er(200, 0.05, seed=8)
    st = m.ImceState(g)
    ost = O.Imce(g)
    before = st.info()
    for bad in (([3], [3]), ([0], [200])):
        with pytest.raises(mod.MceError) as e:
            st.remove(*bad)
        assert e.value.code == mod.MCE_EINVAL
        assert st.info() == before
    u, v = gg.edges_of(g)
    # an edge twice (both orientations), another edge, and two pairs that are
    # (at this density almost surely) not edges
    src = [int(u[0]), int(v[0]), int(u[5]), 0, 1]
    dst = [int(v[0]), int(u[0]), int(v[5]), 199, 198]
    r = st.remove(src, dst, cliques=True)
    w = ost.remove(src, dst, cliques=True)
    for k in KEYS:
        assert r[k] == w[k], k
    assert r["new"] == w["new"] and r["del"] == w["del"]
    # a clique buffer that is too small leaves the state as it was
    u, v = gg.edges_of(gg.remove_edges(g, src, dst))
    before = st.info()
    with pytest.raises(mod.MceError):
        lib = mod.lib()
        import ctypes
        import torch
        s = torch.as_tensor(np.asarray(u[:20], np.uint32).view(np.int32)).cuda()
        d = torch.as_tensor(np.asarray(v[:20], np.uint32).view(np.int32)).cuda()
        res = mod._ImceResult()
        off = torch.zeros(2, dtype=torch.int64, device="cuda")
        vert = torch.zeros(1, dtype=torch.int32, device="cuda")
        cb = mod._CliqueBuf(1, 1, off.data_ptr(), vert.data_ptr(), 1, 0, 0)
        mod._check(lib.imce_remove_edges(st._h, s.data_ptr(), d.data_ptr(), 20, 1, ctypes.byref(res), ctypes.byref(cb),
                                         ctypes.byref(cb)))
    assert st.info() == before
    st.close()


def test_random_deletion_streams_match_oracle_and_recompute(m):
    for seed in range(6):
        g = gg.er(60 + 10 * seed, 0.12 + 0.03 * seed, seed=400 + seed)
        st = m.ImceState(g)
        ost = O.Imce(g)
        cur = g
        for s, d in gg.deletion_stream(g, 5, 1, 30, seed=500 + seed, junk_fraction=0.3):
            r = st.remove(s, d, cliques=True)
            w = ost.remove(s, d, cliques=True)
            assert r["new"] == w["new"] and r["del"] == w["del"]
            for k in KEYS:
                assert r[k] == w[k], (seed, k)
            cur = gg.remove_edges(cur, s, d)
            fresh = m.mce_static(cur, rank="degree")
            assert (r["count"], r["set_hash"]) == (fresh["count"], fresh["set_hash"])
        st.close()


def test_additions_and_deletions_interleaved(m):
    g = gg.plant_communities(gg.chung_lu(3000, 2.2, 10, seed=9), count=8, smin=20, smax=40, p=0.8, seed=10)
    st = m.ImceState(g)
    ost = O.Imce(g)
    adds = gg.edge_stream(g, 4, 50, 300, seed=11)
    dels = gg.deletion_stream(g, 4, 50, 300, seed=12, junk_fraction=0.1)
    for (a_s, a_d), (d_s, d_d) in zip(adds, dels):
        for kind, s, d in (("add", a_s, a_d), ("remove", d_s, d_d)):
            r = getattr(st, kind)(s, d)
            w = getattr(ost, kind)(s, d)
            for k in KEYS:
                assert r[k] == w[k], (kind, k)
    st.close()


def test_deleting_an_added_batch_restores_the_state(m):
    g = gg.chung_lu(20_000, 2.2, 12, seed=13)
    st = m.ImceState(g)
    for s, d in gg.edge_stream(g, 3, 1000, 3000, seed=14):
        before = st.info()
        a = st.add(s, d)
        r = st.remove(d, s)
        assert (r["n_del"], r["n_new"], r["hash_del"], r["hash_new"]) == (a["n_new"], a["n_del"], a["hash_new"],
                                                                         a["hash_del"])
        assert st.info() == before
        st.add(s, d)
    st.close()


def test_powerlaw_deletion_batches_match_oracle(m):
    g = gg.chung_lu(20_000, 2.2, 16, seed=15)
    st = m.ImceState(g)
    ost = O.Imce(g, threads=8)
    for s, d in gg.deletion_stream(g, 4, 1000, 5000, seed=16):
        r = st.remove(s, d)
        w = ost.remove(s, d)
        for k in KEYS:
            assert r[k] == w[k], k
    st.close()
