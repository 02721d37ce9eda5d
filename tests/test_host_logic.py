"""Host-side logic that needs no GPU: latency percentiles, tuner keys."""

import graphgen as gg


def test_nearest_rank():
    from paper_2001_11433_amd.serving import nearest_rank
    v = list(range(1, 201))
    assert nearest_rank(v, 50) == 100 and nearest_rank(v, 99) == 198 and nearest_rank(v, 100) == 200
    assert nearest_rank([5.0], 99) == 5.0


def test_tuner_signature_tracks_the_graph():
    from paper_2001_11433_amd import tuner
    a = gg.rmat(9, seed=1)
    b = gg.rmat(9, seed=2)
    assert tuner.signature(a, "degree") == tuner.signature(gg.rmat(9, seed=1), "degree")
    assert tuner.signature(a, "degree") != tuner.signature(b, "degree")
    assert tuner.signature(a, "degree") != tuner.signature(a, "degeneracy")


def test_memory_estimate_grows_with_batch():
    from paper_2001_11433_amd.serving import estimate_bytes
    assert estimate_bytes(5000) > estimate_bytes(1000) > 0
