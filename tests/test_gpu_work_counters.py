"""glt_last_work's per-class maxima (entries [12]-[15]): the most wedges of one bottom vertex
among the bottoms each 4-cycle class was given, against the same quantity computed on the
host from its definition (degree order with ties by id; the wedges of bottom b are the paths
b - w - t with t ranked above both b and w), bucketed by the schedule's bounds."""
import sys

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def say(msg):
    sys.__stderr__.write(f"[gpu-case] {msg}\n")
    sys.__stderr__.flush()


def _wedges_per_bottom(n, rp, col):
    rp = rp.astype(np.int64)
    deg = np.diff(rp)
    rank = np.empty(n, np.int64)
    rank[np.lexsort((np.arange(n), deg))] = np.arange(n)
    w = np.zeros(n, np.int64)
    for b in range(n):
        for mid in col[rp[b]:rp[b + 1]]:
            tops = col[rp[mid]:rp[mid + 1]]
            w[b] += int(np.count_nonzero(rank[tops] > max(rank[mid], rank[b])))
    return w


def _class_maxima(w, wave_max, mid_max, wg_max):
    cls = np.where(w == 0, -1, np.where(w <= wave_max, 0, np.where(w <= mid_max, 1, np.where(w <= wg_max, 2, 3))))
    return [int(w[cls == c].max()) if (cls == c).any() else 0 for c in range(4)]


@pytest.mark.parametrize("per_edge", [False, True])
def test_class_maxima_single_graph(per_edge):
    import paper_1608_05138_amd as glt
    n = 3000
    rp, col = gg.chung_lu(n, 30000, 2.1, float(n - 1), 21)
    bounds = dict(wedge_wave_max=16, wedge_mid_max=64, wedge_wg_max=256)
    want = _class_maxima(_wedges_per_bottom(n, rp, col), 16, 64, 256)
    assert all(want), want   # every class populated
    say(f"class maxima n={n} per_edge={per_edge}")
    ctx = glt.Context(0)
    try:
        ctx.set_schedule(**bounds)
        ctx.count(rp, col, n=n, per_edge=per_edge)
        w = ctx.last_work()
        got = [w["max_wedges_wave"], w["max_wedges_mid"], w["max_wedges_wg"], w["max_wedges_huge"]]
        assert got == want
    finally:
        ctx.close()


def test_class_maxima_batch():
    import paper_1608_05138_amd as glt
    graphs = [gg.batch_graph(s) for s in gg.batch_spec(6)]
    want = [0, 0, 0, 0]
    for n, (rp, col) in graphs:
        m = _class_maxima(_wedges_per_bottom(n, rp, col), 32, 512, 1024)
        want = [max(a, b) for a, b in zip(want, m)]
    say("class maxima batch of 6")
    ctx = glt.Context(0)
    try:
        ctx.set_schedule(wedge_wave_max=32, wedge_mid_max=512, wedge_wg_max=1024)
        ctx.count_batch(gg.pack_batch(graphs))
        w = ctx.last_work()
        assert [w["max_wedges_wave"], w["max_wedges_mid"], w["max_wedges_wg"], w["max_wedges_huge"]] == want
    finally:
        ctx.close()
