"""GPU parity of the batched path: many independent graphs in one call.

Each graph's 17 global counts from glt_count_batch must equal the oracle's (bit-exact)
and the same graph's counts from a single-graph glt_count call.
"""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def say(msg):
    sys.__stderr__.write(f"[gpu-case] {msg}\n")
    sys.__stderr__.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_1608_05138_amd as glt
    c = glt.Context(0)
    yield c
    c.close()


def _to_device(packed):
    import torch
    d = dict(packed)
    d["row_ptr"] = torch.from_numpy(packed["row_ptr"]).cuda()
    d["col"] = torch.from_numpy(packed["col"]).cuda()
    return d


def _random_graph(rng):
    n = int(rng.integers(0, 41))
    if n < 2:
        return n, (np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32))
    iu = np.triu_indices(n, 1)
    keep = rng.random(iu[0].size) < float(rng.choice([0.0, 0.1, 0.3, 0.6, 0.9]))
    return n, gg.csr_from_pairs(n, iu[0][keep], iu[1][keep])


def test_batch_small_random_vs_brute(ctx):
    rng = np.random.default_rng(7)
    graphs = [_random_graph(rng) for _ in range(120)]
    packed = gg.pack_batch(graphs)
    for dev in (False, True):
        say(f"batch-small device={dev}")
        res = ctx.count_batch(_to_device(packed) if dev else packed)
        assert len(res) == len(graphs)
        for g, (n, (rp, col)) in enumerate(graphs):
            assert res[g] == oracle.brute(n, rp, col)["X"], g


def test_batch_mix_vs_oracle_and_alone(ctx):
    specs = gg.batch_spec(64)
    graphs = [gg.batch_graph(s) for s in specs]
    packed = gg.pack_batch(graphs)
    say(f"batch-mix-64 edges={packed['col'].size // 2}")
    res = ctx.count_batch(_to_device(packed))
    for g, (n, (rp, col)) in enumerate(graphs):
        ref = oracle.count(n, rp, col)["X"]
        assert res[g] == ref, (g, specs[g][:3])
        alone, _ = ctx.count(rp, col, n=n)
        assert alone == res[g], g


def test_batch_repeat_identical(ctx):
    specs = gg.batch_spec(40, base=12345)
    graphs = [gg.batch_graph(s) for s in specs]
    packed = _to_device(gg.pack_batch(graphs))
    say("batch-repeat")
    first = ctx.count_batch(packed)
    for _ in range(3):
        assert ctx.count_batch(packed) == first


def test_batch_invalid_graph_rejected(ctx):
    import paper_1608_05138_amd as glt
    good = gg.cycle(6)
    bad_rp = np.array([0, 1, 2, 2], dtype=np.int32)        # (0,1), (1,2): asymmetric
    bad_col = np.array([1, 2], dtype=np.int32)
    packed = gg.pack_batch([good, (3, (bad_rp, bad_col)), good])
    say("batch-invalid")
    with pytest.raises(glt.GltError) as ei:
        ctx.count_batch(packed)
    assert ei.value.status == -3
    # local id out of range in the second graph
    packed = gg.pack_batch([good, (3, (np.array([0, 1, 2, 2], dtype=np.int32),
                                       np.array([1, 7], dtype=np.int32)))])
    with pytest.raises(glt.GltError) as ei:
        ctx.count_batch(packed)
    assert ei.value.status == -1
    # the handle still works
    assert ctx.count_batch(gg.pack_batch([good]))[0][0] == 6


def test_schedule_api_and_autotuner():
    """The schedule setters reject out-of-range fields; the autotuner returns a schedule from
    its grid, installs it, and the counts under it equal the oracle's."""
    import paper_1608_05138_amd as glt
    c = glt.Context(0)
    try:
        base = c.schedule()
        assert base["tri_records"] in (0, 1) and base["wedge_range_limit"] >= 1
        for bad in ({"wedge_wave_max": 100000}, {"wedge_dense": -1}, {"wedge_range_limit": 0},
                    {"tri_records": 2}):
            with pytest.raises(glt.GltError):
                c.set_schedule(**bad)
            assert c.schedule() == base
        c.set_schedule(wedge_mid_max=0, wedge_dense=7, tri_records=0)
        specs = gg.batch_spec(24, base=gg.BASE_SEED + 77)
        graphs = [gg.batch_graph((m_, min(n, 1200), min(m, 9000), s)) for (m_, n, m, s) in specs]
        packed = _to_device(gg.pack_batch(graphs))
        expect = [oracle.count(n, rp, col)["X"] for n, (rp, col) in graphs]
        say("schedule-fixed")
        assert ctx_counts(c, packed) == expect
        say("autotune")
        best, ms = c.autotune_batch(packed)
        assert ms > 0 and best["wedge_wave_max"] in (128, 256) and best["wedge_mid_max"] in (1024, 2048, 4096)
        assert c.schedule() == best
        assert ctx_counts(c, packed) == expect
    finally:
        c.close()


def ctx_counts(c, packed):
    return c.count_batch(packed)


def _gen(spec):
    return gg.batch_graph(spec)


def test_batch_chunk_boundaries(ctx):
    """Graphs whose edge counts sit at the per-graph chunk boundaries of the batch's union
    columns and combine (8192 edges), with edgeless graphs between them: every graph's
    counts equal the oracle's and its own single-graph call's."""
    rng = np.random.default_rng(11)
    graphs = []
    for n, m in [(900, 8191), (0, 0), (1000, 8192), (5, 0), (1100, 8193), (1, 0), (2000, 16385), (40, 300)]:
        lo, hi = gg.er_pairs(n, m, rng)
        graphs.append((n, gg.csr_from_pairs(n, lo, hi)))
    packed = gg.pack_batch(graphs)
    say(f"batch-chunk-boundaries edges={packed['col'].size // 2}")
    res = ctx.count_batch(_to_device(packed))
    for g, (n, (rp, col)) in enumerate(graphs):
        assert res[g] == oracle.count(n, rp, col)["X"], g
        alone, _ = ctx.count(rp, col, n=n)
        assert alone == res[g], g


def test_batch_10k_vs_stored_oracle(ctx):
    """All 10,000 graphs of the batch mix (n ~ U{50..5000}, ER or Chung-Lu(2.5), mean degree
    ~ U[4, 64]) in one glt_count_batch call: every graph's 17 counts equal the stored
    oracle counts (digest of each graph's counts; full counts of every 100th graph)."""
    import hashlib
    import json
    import multiprocessing as mp
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "batch_10k.json")
    if not os.path.exists(path):
        pytest.skip("no stored counts")
    with open(path) as f:
        golden = json.load(f)
    specs = gg.batch_spec(golden["num_graphs"])
    say("batch-10k generating graphs")
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(procs) as pool:
        graphs = pool.map(_gen, specs, chunksize=16)
    packed = gg.pack_batch(graphs)
    del graphs
    say(f"batch-10k counting ({packed['col'].size // 2} edges)")
    res = ctx.count_batch(_to_device(packed))
    assert len(res) == len(specs)
    for key, Xs in golden["X_every_100"].items():
        assert res[int(key)] == [int(x) for x in Xs], int(key)
    bad = [g for g, X in enumerate(res)
           if hashlib.sha256(",".join(str(v) for v in X).encode()).hexdigest()[:16] != golden["X_digest"][g]]
    assert not bad, f"{len(bad)} graphs differ from the stored oracle counts, first {bad[:10]}"
