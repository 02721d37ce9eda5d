"""Autotuner and online serving on the GPU.

The tuner may only change speed: every trial must return the same count and
hash.  The server runs several sessions concurrently (continuous batching on
per-session streams); each request's result must equal the result of the
same batch processed alone, bit for bit."""

import os

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


def test_tuner_keeps_results_and_records_the_best(m, tmp_path):
    from paper_2001_11433_amd import tuner
    g = gg.rmat(11, seed=7)
    path = str(tmp_path / "tuning.json")
    out = tuner.tune(g, "degeneracy", grid=(("compact", ("inline", 12)), ("waves_per_cu", (2, 4))),
                     space=(("donate_interval", (256,)),), path=path)
    assert len(out["trials"]) >= 4
    best = tuner.lookup(g, "degeneracy", path)
    assert best == out["best"]
    assert min(t["enum_ms"] for t in out["trials"]) == out["enum_ms"]
    assert tuner.lookup(gg.rmat(10, seed=1), "degeneracy", path) == tuner.DEFAULT


def test_incremental_tuner_keeps_results(m, tmp_path):
    from paper_2001_11433_amd import tuner
    g = gg.chung_lu(6000, 2.2, 12, seed=9)
    batches = gg.edge_stream(g, 4, 50, 300, seed=10)
    path = str(tmp_path / "tuning.json")
    space = (("donate_interval", (64,)), ("compact", ("inline",)))
    out = tuner.tune_imce(g, batches, space=space, path=path, key="k")
    assert len(out["trials"]) == 3
    assert tuner.load_table(path)["k"]["best"] == out["best"]


def _sessions():
    graphs, streams = [], []
    for s in range(3):
        g = gg.chung_lu(8000 + 2000 * s, 2.2, 12, seed=s)
        graphs.append(g)
        streams.append(gg.edge_stream(g, 6, 50, 400, seed=100 + s))
    return graphs, streams


def test_each_result_is_the_same_alone_and_in_the_mix(m):
    from paper_2001_11433_amd import serving
    graphs, streams = _sessions()
    alone = [serving.run_alone(g, st) for g, st in zip(graphs, streams)]
    for rate in (None, 400.0):
        mix = serving.replay(graphs, streams, slots=3, rate_hz=rate)
        assert not mix["errors"]
        for r in mix["requests"]:
            want = alone[r.session][r.seq]
            for k in serving.RESULT_KEYS:
                assert r.result[k] == want[k], (rate, r.session, r.seq, k)
        assert mix["max_overlap_sessions"] >= 2
        assert mix["p99_ms"] >= mix["p50_ms"] > 0



def test_pipelined_serving_matches_alone(m):
    # a session's next batch searched while its previous subsumed pass runs:
    # every result still equals the batch processed alone
    from paper_2001_11433_amd import serving
    graphs, streams = _sessions()
    removes = [[k % 3 == 2 for k in range(len(st))] for st in streams]
    alone = [serving.run_alone(g, st, removes=rm) for g, st, rm in zip(graphs, streams, removes)]
    for rate in (None, 400.0):
        mix = serving.replay(graphs, streams, slots=4, rate_hz=rate, pipeline=True, removes=removes)
        assert not mix["errors"]
        for r in mix["requests"]:
            want = alone[r.session][r.seq]
            for k in serving.RESULT_KEYS:
                assert r.result[k] == want[k], (rate, r.session, r.seq, k)


def test_admission_refuses_what_the_budget_cannot_hold(m):
    # a budget of one byte above what the fresh states hold: no second batch
    # ever fits beside a running one, so requests are held back (counted) and
    # run one at a time, and every result is unchanged
    from paper_2001_11433_amd import serving
    graphs, streams = _sessions()
    alone = [serving.run_alone(g, st) for g, st in zip(graphs, streams)]
    fresh = [m.ImceState(g) for g in graphs]
    budget = sum(st.device_bytes() for st in fresh) + 1
    assert all(st.batch_bytes(400) > 0 for st in fresh)
    for st in fresh:
        st.close()
    mix = serving.replay(graphs, streams, slots=3, mem_budget=budget)
    assert not mix["errors"]
    assert mix["refusals"] > 0 and mix["refused_requests"] > 0
    assert mix["max_in_flight"] == 1
    for r in mix["requests"]:
        for k in serving.RESULT_KEYS:
            assert r.result[k] == alone[r.session][r.seq][k]
