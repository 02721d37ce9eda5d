"""mce_static_noalloc (the entry point for callers that cannot allocate)
against mce_static, through the C ABI: bit-exact count, set hash, search
nodes, per-subproblem triples, clique sets and size histograms, on two calls
in a row with the second input smaller, and a clear rejection of a call whose
buffers exceed the fixed scratch (after which the entry point still works)."""

import numpy as np
import pytest

import graphgen as gg

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


def _same(m, g, rank, cliques):
    kw = dict(rank=rank, cliques=cliques, per_vertex=True, size_hist=128)
    got = m.mce_static(g, noalloc=True, **kw)
    want = m.mce_static(g, **kw)
    for k in ("count", "set_hash", "nodes_total", "subproblems", "max_cand", "alg_ops"):
        assert got[k] == want[k], k
    for k in ("nodes_v", "count_v", "hash_v"):
        assert np.array_equal(_u64(got[k]), _u64(want[k])), k
    assert np.array_equal(got["size_hist"], want["size_hist"])
    if cliques:
        assert got["cliques"] == want["cliques"]
    assert got["enum_ms"] == 0.0  # no events inside the allocation-free call
    return got


def test_two_calls_in_a_row_second_smaller(m):
    print("noalloc: communities 6000 then ER 300", flush=True)
    big = gg.plant_communities(gg.chung_lu(6000, 2.1, 10, seed=21), count=10, smin=30, smax=60, p=0.9, seed=22)
    small = gg.er(300, 0.08, seed=23)
    a = _same(m, big, "degree", cliques=True)
    b = _same(m, small, "degeneracy", cliques=True)
    assert a["count"] > b["count"] > 0


def test_larger_workloads_and_ranks(m):
    print("noalloc: ER(2000, 0.01), R-MAT 12, Chung-Lu 50k", flush=True)
    _same(m, gg.er(2000, 0.01, seed=0), "degree", cliques=False)
    _same(m, gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=1), "degeneracy", cliques=False)
    _same(m, gg.chung_lu(50_000, 2.2, 16, seed=2), "peel", cliques=False)


def test_host_resident_input_is_staged_through_the_scratch(m):
    import ctypes
    mod = m
    g = gg.er(500, 0.05, seed=24)
    rp = np.ascontiguousarray(g.row_ptr, np.uint64)
    col = np.ascontiguousarray(g.col, np.uint32)
    csr = mod._Csr(g.n, rp.ctypes.data, col.ctypes.data, 0)
    res = mod._Result()
    mod._check(mod.lib().mce_static_noalloc(ctypes.byref(csr), 0, None, ctypes.byref(res), None, None))
    want = m.mce_static(g)
    assert (res.count, res.set_hash, res.nodes_total) == (want["count"], want["set_hash"], want["nodes_total"])


def test_call_beyond_the_scratch_is_rejected_then_small_calls_work(m):
    print("noalloc: K_2000 beyond the scratch", flush=True)
    with pytest.raises(m.MceError) as e:
        m.mce_static(gg.complete(2000), noalloc=True)
    assert e.value.code == m.MCE_ENOTSUP
    assert "scratch" in m.lib().mce_last_error().decode()
    _same(m, gg.er(400, 0.06, seed=25), "triangle", cliques=True)
