"""The host-thread wedge pass (glt_host_wedges), the CPU side of the paper's hybrid scheme
(Section 4.3), against the device's wedge pass of the same call: the same wedges, the same
non-induced 4-cycle total, which also equals X10 + X8 + 3 X7 of the global counts (every
4-cycle, chordal cycle and 4-clique holds 1, 1 and 3 four-cycles), and per-edge credits
summing to four per 4-cycle."""
import sys

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def say(msg):
    sys.__stderr__.write(f"[gpu-case] {msg}\n")
    sys.__stderr__.flush()


def _wedges(work):
    return work["wedges_wave"] + work["wedges_mid"] + work["wedges_wg"] + work["wedges_huge"]


@pytest.mark.parametrize("n,m,seed,threads", [(20000, 200000, 8, 4), (3001, 45000, 9, 1), (50, 0, 1, 2)])
def test_host_wedges_match_device(n, m, seed, threads):
    import torch
    import paper_1608_05138_amd as glt
    say(f"host wedges chung-lu n={n} m={m} threads={threads}")
    if m:
        rp, col = gg.chung_lu(n, m, 2.1, float(n - 1), seed)
    else:
        rp, col = np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32)
    ctx = glt.Context(0)
    try:
        X, _ = ctx.count(torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(), n=n, per_edge=True)
        work = ctx.last_work()
        r = ctx.host_wedges(threads)
        assert r["threads"] == threads
        assert r["wedges"] == _wedges(work)
        assert r["cycles4"] == r["gpu_cycles4"] == X[9] + X[7] + 3 * X[6]
        assert r["credit_sum"] == 4 * r["cycles4"]
        assert r["bytes_copied"] == 4 * (n + 1) + 12 * 2 * (col.size // 2) + 4 * (col.size // 2)
    finally:
        ctx.close()


def test_host_wedges_need_a_single_graph_count():
    import torch
    import paper_1608_05138_amd as glt
    say("host wedges without a single-graph count")
    ctx = glt.Context(0)
    try:
        with pytest.raises(glt.GltError):
            ctx.host_wedges(2)
        n = 200
        rp, col = gg.chung_lu(n, 1000, 2.1, float(n - 1), 3)
        ctx.count(torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(), n=n)
        assert ctx.host_wedges(2)["cycles4"] >= 0
        ctx.count_batch(gg.pack_batch([(n, (rp, col))]))
        with pytest.raises(glt.GltError):
            ctx.host_wedges(2)
    finally:
        ctx.close()
