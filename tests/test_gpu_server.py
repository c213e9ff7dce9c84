"""GPU tests of the request server (continuous batching).

Every served result must equal the same graph counted alone (glt_count) and the oracle;
requests arriving while others run are batched together; an invalid request fails alone;
an admission budget smaller than the offered load delays admission but loses nothing.
"""
import sys
import time

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def say(msg):
    sys.__stderr__.write(f"[gpu-case] {msg}\n")
    sys.__stderr__.flush()


def _collect(srv, want, timeout_s=120.0):
    got = {}
    t0 = time.time()
    while len(got) < want:
        for r in srv.poll(256, 20000):
            got[r["req_id"]] = r
        assert time.time() - t0 < timeout_s, f"only {len(got)} of {want} results"
    return got


def _requests(num, seed):
    specs = gg.batch_spec(num, base=seed)
    # keep the graphs small enough for the oracle
    return [gg.batch_graph((m_, min(n, 1500), min(m, 12000), s)) for (m_, n, m, s) in specs]


def test_served_equals_alone_and_oracle():
    import paper_1608_05138_amd as glt
    graphs = _requests(150, 777)
    ctx = glt.Context(0)
    alone = [ctx.count(rp, col, n=n)[0] for n, (rp, col) in graphs]
    srv = glt.Server(0)
    say("server-mix")
    rng = np.random.default_rng(1)
    for i, (n, (rp, col)) in enumerate(graphs):
        assert srv.submit(rp, col, i, n=n) == 0
        if rng.random() < 0.3:
            time.sleep(float(rng.uniform(0, 0.002)))
    got = _collect(srv, len(graphs))
    srv.close()
    assert max(r["batch_graphs"] for r in got.values()) > 1, "no request was batched with another"
    for i, (n, (rp, col)) in enumerate(graphs):
        r = got[i]
        assert r["status"] == 0, r
        assert r["X"] == alone[i], i
        assert r["t_submit"] <= r["t_admit"] <= r["t_start"] <= r["t_done"]
    for i in range(0, len(graphs), 5):
        n, (rp, col) = graphs[i]
        assert got[i]["X"] == oracle.count(n, rp, col)["X"], i
    ctx.close()


def test_invalid_request_fails_alone():
    import paper_1608_05138_amd as glt
    graphs = _requests(40, 4242)
    bad = {7: (3, (np.array([0, 1, 2, 2], np.int32), np.array([1, 2], np.int32)), -3),   # asymmetric
           19: (2, (np.array([0, 2, 4], np.int32), np.array([0, 1, 0, 1], np.int32)), -2),  # self-loops
           30: (2, (np.array([0, 1, 2], np.int32), np.array([1, 9], np.int32)), -1)}     # id out of range
    srv = glt.Server(0)
    say("server-invalid")
    for i, (n, (rp, col)) in enumerate(graphs):
        if i in bad:
            n, (rp, col), _ = bad[i]
        assert srv.submit(rp, col, i, n=n) == 0
    got = _collect(srv, len(graphs))
    srv.close()
    for i, (n, (rp, col)) in enumerate(graphs):
        if i in bad:
            assert got[i]["status"] == bad[i][2], (i, got[i]["status"])
        else:
            assert got[i]["status"] == 0, (i, got[i]["status"])
            assert got[i]["X"] == oracle.count(n, rp, col)["X"], i


def test_small_admission_budget_and_per_graph_mode():
    import paper_1608_05138_amd as glt
    graphs = _requests(60, 99)
    expect = [oracle.count(n, rp, col)["X"] for n, (rp, col) in graphs]
    # pool of 2 MiB: only a few graphs resident at a time; one graph larger than the pool
    big_n, (big_rp, big_col) = 30000, gg.er(30000, 400000, 5)
    for opts in ({"resident_bytes": 2 << 20}, {"max_batch_graphs": 1}):
        say(f"server-opts {opts}")
        srv = glt.Server(0, **opts)
        for i, (n, (rp, col)) in enumerate(graphs):
            assert srv.submit(rp, col, i, n=n) == 0
        assert srv.submit(big_rp, big_col, 1000, n=big_n) == 0
        got = _collect(srv, len(graphs) + 1)
        assert srv.inflight() == 0
        srv.close()
        for i in range(len(graphs)):
            assert got[i]["status"] == 0 and got[i]["X"] == expect[i], (opts, i)
        if "resident_bytes" in opts:
            assert got[1000]["status"] == -4          # larger than the whole pool
        else:
            assert got[1000]["status"] == 0
            assert max(r["batch_graphs"] for r in got.values()) == 1


def test_large_requests_run_on_their_own_lane():
    """A large request runs on the second compute lane: small requests submitted right after
    it finish before it does (they are not queued behind it), and every result equals the
    graph counted alone."""
    import paper_1608_05138_amd as glt
    n_big = 200_000
    big_rp, big_col = gg.chung_lu(n_big, 2_000_000, 2.5, float(n_big - 1), 11)
    graphs = _requests(40, 515)
    ctx = glt.Context(0)
    alone = [ctx.count(rp, col, n=n)[0] for n, (rp, col) in graphs]
    alone_big = ctx.count(big_rp, big_col, n=n_big)[0]
    ctx.close()
    srv = glt.Server(0, large_edges=100_000)
    say("server-lanes")
    assert srv.submit(big_rp, big_col, 10_000, n=n_big) == 0
    for i, (n, (rp, col)) in enumerate(graphs):
        assert srv.submit(rp, col, i, n=n) == 0
    got = _collect(srv, len(graphs) + 1)
    srv.close()
    assert got[10_000]["status"] == 0 and got[10_000]["X"] == alone_big
    for i in range(len(graphs)):
        assert got[i]["status"] == 0 and got[i]["X"] == alone[i], i
    early = sum(1 for i in range(len(graphs)) if got[i]["t_done"] < got[10_000]["t_done"])
    assert early > 0, "every small request waited for the large one"
