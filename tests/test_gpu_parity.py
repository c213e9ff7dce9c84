"""GPU parity: libglt (HIP, gfx950) against the CPU oracle, element by element.

Every call goes through the C ABI (ctypes binding).  Counts are integers, so the bar is
bit-exact equality of all 17 global counts and all 13 x m per-edge counts.  Sizes span
every work bucket of the kernels (wave and workgroup paths, LDS and global bitmap rows,
hash-range splitting in the wedge pass) with ragged tails.
"""
import sys
from math import comb

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


@pytest.fixture(scope="module", autouse=True)
def _oracle_built():
    oracle.build(force=False)


def gpu(ctx, n, rp, col, per_edge=True, device=True):
    import torch
    if device:
        rpt = torch.from_numpy(np.ascontiguousarray(rp)).cuda()
        ct = torch.from_numpy(np.ascontiguousarray(col, dtype=np.int32)).cuda()
        X, pe = ctx.count(rpt, ct, n=n, per_edge=per_edge)
        torch.cuda.synchronize()
        if per_edge:
            pe = pe.cpu().numpy().view(np.uint64)
        return X, pe
    return ctx.count(np.ascontiguousarray(rp), np.ascontiguousarray(col, dtype=np.int32), n=n,
                     per_edge=per_edge)


def check_vs_oracle(ctx, name, n, rp, col, device=True, brute=False):
    say(f"{name} n={n} m={col.size // 2} device={device}")
    ref = oracle.brute(n, rp, col, per_edge=True) if brute else oracle.count(n, rp, col, per_edge=True)
    X, pe = gpu(ctx, n, rp, col, per_edge=True, device=device)
    assert X == ref["X"], name
    np.testing.assert_array_equal(pe, ref["per_edge"], err_msg=name)
    Xg, _ = gpu(ctx, n, rp, col, per_edge=False, device=device)
    assert Xg == ref["X"], name + " (global mode)"
    return X, pe


def _random_pairs(n, p, rng):
    iu = np.triu_indices(n, 1)
    keep = rng.random(iu[0].size) < p
    return np.stack([iu[0][keep], iu[1][keep]], 1)


def test_small_random_vs_brute(ctx):
    rng = np.random.default_rng(101)
    for trial in range(60):
        n = int(rng.integers(4, 41))
        p = float(rng.choice([0.05, 0.15, 0.3, 0.5, 0.8, 0.95]))
        n_, (rp, col) = gg.from_pairs(n, _random_pairs(n, p, rng))
        col = gg.shuffle_rows(rp, col, trial)
        check_vs_oracle(ctx, f"small-{trial}", n, rp, col, device=bool(trial % 2), brute=True)


@pytest.mark.parametrize("name,n,pairs", [
    ("no-edges", 6, []),
    ("single-edge", 2, [(0, 1)]),
    ("single-edge-isolated", 9, [(3, 7)]),
    ("triangle", 3, [(0, 1), (1, 2), (0, 2)]),
    ("two-triangles", 6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)]),
    ("star", 12, [(0, i) for i in range(1, 12)]),
    ("clique-pendant", 9, [(i, j) for i in range(7) for j in range(i + 1, 7)] + [(6, 7)]),
])
def test_degenerate(ctx, name, n, pairs):
    n_, (rp, col) = gg.from_pairs(n, pairs)
    check_vs_oracle(ctx, name, n, rp, col, brute=True)


def test_zero_vertices(ctx):
    say("zero-vertices")
    rp = np.zeros(1, dtype=np.int32)
    col = np.zeros(0, dtype=np.int32)
    X, pe = gpu(ctx, 0, rp, col, per_edge=True, device=False)
    assert X == [0] * 17


def test_config_er_1k(ctx):
    n, (rp, col) = gg.config_er_1k()
    check_vs_oracle(ctx, "er-1000-10000", n, rp, col)
    check_vs_oracle(ctx, "er-1000-10000-host", n, rp, col, device=False)


def test_chung_lu_medium(ctx):
    for n, m, seed in ((5000, 60000, 7), (20000, 200000, 8), (3001, 45000, 9)):
        rp, col = gg.chung_lu(n, m, 2.1, float(n - 1), seed)
        check_vs_oracle(ctx, f"chung-lu-{n}-{m}", n, rp, col)


def test_clique_on_noise(ctx):
    # a 300-clique (out-degrees up to 299: the LDS bitmap workgroup path) on sparse noise
    rng = np.random.default_rng(3)
    n = 2300
    lo, hi = gg.er_pairs(n, 6000, rng)
    iu = np.triu_indices(300, 1)
    a = np.concatenate([lo, iu[0]])
    b = np.concatenate([hi, iu[1]])
    key = np.unique(np.minimum(a, b) * n + np.maximum(a, b))
    perm = rng.permutation(n)
    rp, col = gg.csr_from_pairs(n, perm[key // n], perm[key % n])
    check_vs_oracle(ctx, "clique300-noise", n, rp, col)


def _closed_complete(n):
    X = [0] * 17
    X[0] = comb(n, 2); X[2] = comb(n, 3); X[6] = comb(n, 4)
    return X


def test_complete_graph_global_bitmap_path(ctx):
    # K_n: out-degrees 65..n-1 take every workgroup path: LDS bitmap rows up to 896, the
    # global-memory rows above
    n = 1000
    N, (rp, col) = gg.complete(n)
    say(f"complete-{n}")
    X, pe = gpu(ctx, N, rp, col)
    assert X == _closed_complete(n)
    m = col.size // 2
    expect = np.zeros((13, m), dtype=np.uint64)
    expect[0] = n - 2                 # triangles on each edge
    expect[3] = comb(n - 2, 2)        # 4-cliques on each edge
    np.testing.assert_array_equal(pe, expect)


def test_complete_bipartite(ctx):
    # K_{a,b}, a < b: every bottom vertex on the a-side has b wedges to each top above it
    a, b = 300, 340
    N, (rp, col) = gg.complete_bipartite(a, b)
    say(f"complete-bipartite-{a}-{b}")
    X, pe = gpu(ctx, N, rp, col)
    nz = {1: a * b, 4: a * comb(b, 2) + b * comb(a, 2), 6: comb(a, 3) + comb(b, 3),
          10: comb(a, 2) * comb(b, 2), 11: a * comb(b, 3) + b * comb(a, 3),
          17: comb(a, 4) + comb(b, 4)}
    expect = [nz.get(i, 0) for i in range(1, 18)]
    expect[1] = comb(N, 2) - a * b
    assert X == expect
    m = a * b
    want = np.zeros((13, m), dtype=np.uint64)
    want[1] = a + b - 2                                # 2-stars on the edge
    want[6] = (a - 1) * (b - 1)                        # 4-cycles on the edge
    want[7] = comb(a - 1, 2) + comb(b - 1, 2)          # 3-stars on the edge
    np.testing.assert_array_equal(pe, want)


SPLIT_CASES = {
    # name: (wave-class max, mid-class max, dense window, workgroup-class max)
    "wg-nodense": ("0", "0", "0", "1000000000"),
    "wg-dense7": ("0", "0", "7", "1000000000"),
    "mid-nodense": ("0", "1000000000", "0", "1000000000"),
    "mid-dense7": ("0", "1000000000", "7", "1000000000"),
    "wave+wg": ("256", "256", "5", "1000000000"),
    "huge-nodense": ("0", "0", "0", "0"),
    "huge-dense9": ("0", "0", "9", "0"),
}


@pytest.mark.parametrize("case", list(SPLIT_CASES))
def test_forced_classes_and_range_splitting(monkeypatch, case):
    """Wedge pass with every bottom vertex forced into one size class (workgroup, mid
    wavefront, huge workgroup, or wave + workgroup), a tiny distinct-top limit (hash ranges
    split many times) and no or a tiny dense window of top counters; results must not
    change."""
    import paper_1608_05138_amd as glt
    wave_max, mid_max, dense, wg_max = SPLIT_CASES[case]
    monkeypatch.setenv("GLT_WEDGE_WAVE_MAX", wave_max)
    monkeypatch.setenv("GLT_WEDGE_MID_MAX", mid_max)
    monkeypatch.setenv("GLT_WEDGE_WG_MAX", wg_max)
    monkeypatch.setenv("GLT_WEDGE_RANGE_LIMIT", "3")
    monkeypatch.setenv("GLT_WEDGE_DENSE", dense)
    c = glt.Context(0)
    try:
        for n, m, seed in ((3000, 30000, 31), (800, 24000, 32)):
            rp, col = gg.chung_lu(n, m, 2.1, float(n - 1), seed)
            check_vs_oracle(c, f"forced-{case}-{n}-{m}", n, rp, col)
        N, (rp, col) = gg.complete_bipartite(40, 47)
        check_vs_oracle(c, f"forced-{case}-K40,47", N, rp, col)
    finally:
        c.close()


def test_triangle_records_on_and_off(monkeypatch, ctx):
    """The triangle and gather passes walk stored triangle records when the record buffer
    fits, and re-scan the out-lists when records are switched off (here also with the 4-cycle
    pass on a second stream beside them); both must agree with each other and with the oracle
    on the wave, LDS-bitmap and global-bitmap paths."""
    import paper_1608_05138_amd as glt
    monkeypatch.setenv("GLT_TRI_RECORD_BYTES", "0")
    off = glt.Context(0)
    off.set_schedule(wedge_stream=1)   # and the 4-cycle pass on a second stream beside them
    try:
        rng = np.random.default_rng(5)
        n = 2300
        lo, hi = gg.er_pairs(n, 6000, rng)
        iu = np.triu_indices(700, 1)   # out-degrees up to 699: global-bitmap rows
        a = np.concatenate([lo, iu[0]]); b = np.concatenate([hi, iu[1]])
        key = np.unique(np.minimum(a, b) * n + np.maximum(a, b))
        perm = rng.permutation(n)
        cases = [("clique700-noise", n, gg.csr_from_pairs(n, perm[key // n], perm[key % n]))]
        cases.append(("chung-lu-4000", 4000, gg.chung_lu(4000, 60000, 2.1, 3999.0, 77)))
        for name, nn, (rp, col) in cases:
            say(f"records {name}")
            X1, pe1 = gpu(ctx, nn, rp, col)
            X0, pe0 = gpu(off, nn, rp, col)
            assert X0 == X1, name
            np.testing.assert_array_equal(pe0, pe1)
            assert X1 == oracle.count(nn, rp, col)["X"], name
            G1, _ = gpu(ctx, nn, rp, col, per_edge=False)
            G0, _ = gpu(off, nn, rp, col, per_edge=False)
            assert G0 == G1 == X1, name
    finally:
        off.close()


@pytest.mark.parametrize("records", ["on", "off"])
def test_stream_modes_agree(monkeypatch, ctx, records):
    """Stream mode 2 runs the workgroup triangle and gather paths on a second stream beside
    the wavefront paths (each gather path waiting for both triangle paths) and mode 1 the
    4-cycle pass beside them; per-edge and global counts must equal one-stream's, with and
    without triangle records, on graphs that reach the wave, LDS-bitmap and global-bitmap
    paths."""
    import paper_1608_05138_amd as glt
    if records == "off":
        monkeypatch.setenv("GLT_TRI_RECORD_BYTES", "0")
    handles = {}
    try:
        for mode in (0, 1, 2):
            handles[mode] = glt.Context(0)
            handles[mode].set_schedule(wedge_stream=mode)
        rng = np.random.default_rng(9)
        n = 3000
        lo, hi = gg.er_pairs(n, 9000, rng)
        iu = np.triu_indices(760, 1)   # out-degrees up to 759: global-bitmap rows
        a = np.concatenate([lo, iu[0]]); b = np.concatenate([hi, iu[1]])
        key = np.unique(np.minimum(a, b) * n + np.maximum(a, b))
        perm = rng.permutation(n)
        cases = [("clique760-noise", n, gg.csr_from_pairs(n, perm[key // n], perm[key % n])),
                 ("chung-lu-6000", 6000, gg.chung_lu(6000, 90000, 2.1, 5999.0, 78))]
        for name, nn, (rp, col) in cases:
            say(f"stream modes {records} {name}")
            X0, pe0 = gpu(handles[0], nn, rp, col)
            for mode in (1, 2):
                X, pe = gpu(handles[mode], nn, rp, col)
                assert X == X0, (name, mode)
                np.testing.assert_array_equal(pe, pe0)
                G, _ = gpu(handles[mode], nn, rp, col, per_edge=False)
                assert G == X0, (name, mode)
        assert X0 == oracle.count(nn, rp, col)["X"]
    finally:
        for h in handles.values():
            h.close()


def test_modes_and_layouts_agree(ctx):
    n = 4000
    rp, col = gg.chung_lu(n, 40000, 2.3, float(n - 1), 21)
    say("layouts")
    X1, pe1 = gpu(ctx, n, rp, col)
    X2, pe2 = gpu(ctx, n, rp.astype(np.int64), col)            # 64-bit offsets
    assert X1 == X2
    np.testing.assert_array_equal(pe1, pe2)
    col3 = gg.shuffle_rows(rp, col, 5)                          # neighbour order
    X3, pe3 = gpu(ctx, n, rp, col3)
    assert X3 == X1
    perm = np.random.default_rng(1).permutation(n)               # vertex names
    n4, (rp4, col4) = gg.relabel(n, rp, col, perm)
    X4, _ = gpu(ctx, n4, rp4, col4, per_edge=False)
    assert X4 == X1
    # repeated calls on one handle give identical results
    X5, pe5 = gpu(ctx, n, rp, col)
    assert X5 == X1
    np.testing.assert_array_equal(pe5, pe1)


def test_invalid_inputs_rejected(ctx):
    import paper_1608_05138_amd as glt
    say("invalid-inputs")

    def expect(status, n, rp, col):
        with pytest.raises(glt.GltError) as ei:
            ctx.count(np.asarray(rp, dtype=np.int32), np.asarray(col, dtype=np.int32), n=n)
        assert ei.value.status == status, str(ei.value)

    expect(-2, 2, [0, 2, 4], [0, 1, 0, 1])              # self-loops
    expect(-2, 3, [0, 2, 3, 4], [1, 1, 0, 0])           # duplicate entry
    expect(-3, 3, [0, 1, 2, 2], [1, 2])                 # (0,1),(1,2) without reverses
    expect(-1, 2, [0, 1, 2], [1, 5])                    # id out of range
    expect(-1, 2, [0, 2, 1], [1, 0])                    # offsets not monotone
    expect(-1, 2, [0, 1, 3], [1, 0])                    # row_ptr[n] != 2m
    # the handle still works after errors
    n, (rp, col) = gg.cycle(7)
    X, _ = gpu(ctx, n, rp, col, per_edge=False)
    assert X[0] == 7


def _row_class_graph(seed):
    """Rows of every length class of the per-row sort (a 5000-leaf star, a 1000-leaf star, a
    200-leaf star, vertices of degree ~40 and ~10) over sparse noise, ids and row order
    shuffled."""
    rng = np.random.default_rng(seed)
    n = 7000
    lo, hi = gg.er_pairs(n, 9000, rng)
    a = [lo, np.zeros(5000, np.int64), np.full(1000, 5001, np.int64), np.full(200, 6200, np.int64)]
    b = [hi, np.arange(1, 5001), np.arange(5002, 6002), np.arange(6300, 6500)]
    for v in range(6100, 6140):
        a.append(np.full(40, v, np.int64)); b.append(rng.choice(6000, 40, replace=False) + 1)
    a = np.concatenate(a); b = np.concatenate(b)
    keep = a != b
    a, b = a[keep], b[keep]
    key = np.unique(np.minimum(a, b) * n + np.maximum(a, b))
    perm = rng.permutation(n)
    rp, col = gg.csr_from_pairs(n, perm[key // n], perm[key % n])
    return n, rp, gg.shuffle_rows(rp, col, seed + 1)


def test_row_sort_classes(ctx):
    n, rp, col = _row_class_graph(41)
    d = np.diff(rp)
    assert d.max() > 2048 and ((d > 256) & (d <= 2048)).any() and ((d > 64) & (d <= 256)).any()
    assert ((d > 16) & (d <= 64)).any()
    check_vs_oracle(ctx, "row-sort-classes", n, rp, col)


@pytest.mark.parametrize("length_class", ["tiny", "wave", "wave_lds", "wg", "big"])
def test_duplicate_in_each_row_class(ctx, length_class):
    """A duplicated neighbour is found whichever per-row sort handled the row."""
    import paper_1608_05138_amd as glt
    n, rp, col = _row_class_graph(43)
    d = np.diff(rp)
    lo, hi = {"tiny": (2, 16), "wave": (17, 64), "wave_lds": (65, 256), "wg": (257, 2048),
              "big": (2049, 1 << 30)}[length_class]
    r = int(np.flatnonzero((d >= lo) & (d <= hi - 2))[0])
    c = int(col[rp[r]])
    rows = [list(col[rp[i]:rp[i + 1]]) for i in range(n)]
    # c three times in row r only (the entry count stays even; the row stays in its class)
    rows[r].insert(len(rows[r]) // 2, c)
    rows[r].append(c)
    rp2 = np.zeros(n + 1, np.int64)
    rp2[1:] = np.cumsum([len(x) for x in rows])
    col2 = np.concatenate([np.asarray(x, np.int32) for x in rows])
    say(f"duplicate-{length_class}")
    with pytest.raises(glt.GltError) as ei:
        ctx.count(rp2.astype(np.int32), col2, n=n)
    assert ei.value.status == -2, str(ei.value)


def test_budget_is_enforced():
    import paper_1608_05138_amd as glt
    say("budget")
    c = glt.Context(0, hbm_budget_bytes=1 << 16)
    n, (rp, col) = gg.config_er_1k()
    with pytest.raises(glt.GltError) as ei:
        c.count(rp, col, n=n)
    assert ei.value.status == -4
    c.close()


def _exact_sum(v):
    """Exact sum of a uint64 array as a Python int (split in 32-bit halves)."""
    v = np.asarray(v, dtype=np.uint64)
    hi = int((v >> np.uint64(32)).sum(dtype=np.uint64))
    lo = int((v & np.uint64(0xFFFFFFFF)).sum(dtype=np.uint64))
    return (hi << 32) + lo


def _edge_sum_identity(X, pe):
    for s, gid in enumerate(oracle.EDGE_SLOTS):
        assert _exact_sum(pe[s]) == oracle.GRAPHLET_EDGES[gid - 1] * X[gid - 1], gid


def _sampled_edges(n, rp, col, k, seed):
    """Edge ids of k random edges plus the edges at the highest-degree vertices."""
    m = col.size // 2
    rng = np.random.default_rng(seed)
    ids = set(int(x) for x in rng.integers(0, m, size=k))
    rp64 = np.asarray(rp, dtype=np.int64)
    src = np.repeat(np.arange(n), np.diff(rp64))
    up = col > src
    eid_of_slot = np.cumsum(up) - 1
    deg = np.diff(rp64)
    for h in np.argsort(-deg)[:3]:
        slots = np.arange(rp64[h], rp64[h + 1])
        for sl in slots[:8]:
            if up[sl]:
                ids.add(int(eid_of_slot[sl]))
            else:
                # the same edge, seen from its other endpoint's row
                other = col[sl]
                row = np.arange(rp64[other], rp64[other + 1])
                hit = row[col[row] == h]
                ids.add(int(eid_of_slot[hit[0]]))
    return np.array(sorted(ids), dtype=np.int64)


def _load_golden(name, col):
    """Stored oracle results (tests/golden/<name>), checked to belong to this graph."""
    import hashlib
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    assert hashlib.sha256(np.ascontiguousarray(col).tobytes()).hexdigest()[:16] == g["col_sha256_prefix"]
    return g


def _slot_digests(pe):
    import hashlib
    return [hashlib.sha256(np.ascontiguousarray(pe[s], dtype="<u8").tobytes()).hexdigest() for s in range(13)]


def _full_size(ctx, name, n, rp, col, golden_X=None, golden_pe=None):
    """Full-size graph: global counts against the stored oracle counts; per-edge counts
    against the stored oracle's SHA-256 of every slot array (all edges) and its counts of a
    seeded edge sample (element by element, to name a failing edge); identities that hold
    at any size; and the oracle itself on a few sampled edges."""
    say(f"{name} per-edge")
    X, pe = gpu(ctx, n, rp, col, per_edge=True)
    say(f"{name} global")
    Xg, _ = gpu(ctx, n, rp, col, per_edge=False)
    assert Xg == X
    _edge_sum_identity(X, pe)
    assert X[0] == col.size // 2
    assert sum(X[2:6]) == comb(n, 3)
    if golden_X is not None:
        assert X == golden_X, name + " vs stored oracle counts"
    if golden_pe is not None:
        eids = np.asarray(golden_pe["sample_eids"], dtype=np.int64)
        np.testing.assert_array_equal(pe[:, eids], np.asarray(golden_pe["sample_counts"], dtype=np.uint64))
        say(f"{name} per-edge digests of all {col.size // 2} edges")
        assert _slot_digests(pe) == golden_pe["slot_sha256"], name + " per-edge arrays vs stored oracle digests"
    eids = _sampled_edges(n, rp, col, 48, 7)
    say(f"{name} oracle on {eids.size} sampled edges")
    ref = oracle.count_edges(n, rp, col, eids)
    np.testing.assert_array_equal(pe[:, eids], ref)
    return X


def test_config_chung_lu_1m(ctx):
    n, (rp, col) = gg.config_chung_lu_1m()
    g = _load_golden("chung_lu_1m_global.json", col)
    gpe = _load_golden("chung_lu_1m_per_edge.json", col)
    _full_size(ctx, "chung-lu-1m-10m", n, rp, col, [int(x) for x in g["X"]] if g else None, gpe)
    if gpe is not None:
        assert [int(x) for x in gpe["X"]] == [int(x) for x in g["X"]]


def test_config_rmat_s22(ctx):
    n, (rp, col) = gg.config_rmat_s22()
    g = _load_golden("rmat_s22.json", col)
    _full_size(ctx, "rmat-s22-ef16", n, rp, col, [int(x) for x in g["X"]] if g else None, g)


def test_hub_above_46340_all_stream_modes():
    """A 50,000-leaf star over sparse ER noise: the maximum degree exceeds 46,340, so every
    per-edge accumulator is 64-bit; all 13 per-edge counts of every edge and the global
    counts must equal the oracle's in each stream mode."""
    import paper_1608_05138_amd as glt
    rng = np.random.default_rng(46341)
    n = 60000
    lo, hi = gg.er_pairs(n, 100000, rng)
    a = np.concatenate([lo, np.zeros(50000, np.int64)])
    b = np.concatenate([hi, np.arange(1, 50001)])
    key = np.unique(np.minimum(a, b) * n + np.maximum(a, b))
    perm = rng.permutation(n)
    rp, col = gg.csr_from_pairs(n, perm[key // n], perm[key % n])
    assert np.diff(rp).max() > 46340
    ref = oracle.count(n, rp, col, per_edge=True)
    for mode in (0, 1, 2):
        c = glt.Context(0)
        try:
            c.set_schedule(wedge_stream=mode)
            say(f"hub-50000-star mode {mode}")
            X, pe = gpu(c, n, rp, col)
            assert X == ref["X"], mode
            np.testing.assert_array_equal(pe, ref["per_edge"], err_msg=f"mode {mode}")
            G, _ = gpu(c, n, rp, col, per_edge=False)
            assert G == ref["X"], mode
        finally:
            c.close()


def test_inputs_pending_on_default_stream(ctx):
    """Device inputs still being written by work queued on the default stream (a
    non-blocking copy from pinned memory behind a long kernel) are read only after that
    work: the call made with no stream waits for the default stream."""
    import torch
    n = 20000
    rp, col = gg.chung_lu(n, 200000, 2.1, float(n - 1), 12)
    ref = oracle.count(n, rp, col, per_edge=True)
    say("inputs pending on the default stream")
    for trial in range(3):
        a = torch.randn(4096, 4096, device="cuda")
        b = a
        for _ in range(8):          # keeps the default stream busy for a while
            b = b @ a
        rpt = torch.from_numpy(np.ascontiguousarray(rp)).pin_memory().cuda(non_blocking=True)
        ct = torch.from_numpy(np.ascontiguousarray(col, dtype=np.int32)).pin_memory().cuda(non_blocking=True)
        out = torch.full((13, col.size // 2), -1, dtype=torch.int64, device="cuda")
        X, pe = ctx.count(rpt, ct, n=n, per_edge=True, out=out)
        torch.cuda.synchronize()
        assert X == ref["X"], trial
        np.testing.assert_array_equal(pe.cpu().numpy().view(np.uint64), ref["per_edge"])
        del b


def test_out_degree_above_lds_rows(ctx):
    """Out-degrees above 3200 in the degree order keep the workgroup passes' per-neighbour
    arrays and hash in the global slab: K_{3301,3301} (the lowest-ranked vertex of one side
    has out-degree 3301; no triangle) counts exactly, per edge
    and globally, against the complete-bipartite closed forms; K_3201 (out-degrees up to
    3200, the largest kept in LDS) still counts exactly."""
    a = b = 3301
    N, (rp, col) = gg.complete_bipartite(a, b)
    say(f"complete-bipartite-{a}-{b} (out-degree above the LDS rows)")
    X, pe = gpu(ctx, N, rp, col)
    nz = {1: a * b, 4: a * comb(b, 2) + b * comb(a, 2), 6: comb(a, 3) + comb(b, 3),
          10: comb(a, 2) * comb(b, 2), 11: a * comb(b, 3) + b * comb(a, 3),
          17: comb(a, 4) + comb(b, 4)}
    expect = [nz.get(i, 0) for i in range(1, 18)]
    expect[1] = comb(N, 2) - a * b
    assert X == expect
    m = a * b
    want = np.zeros((13, m), dtype=np.uint64)
    want[1] = a + b - 2
    want[6] = (a - 1) * (b - 1)
    want[7] = comb(a - 1, 2) + comb(b - 1, 2)
    np.testing.assert_array_equal(pe, want)
    n = 3201
    N, (rp, col) = gg.complete(n)
    say(f"complete-{n}")
    X, _ = gpu(ctx, N, rp, col, per_edge=False)
    assert X == _closed_complete(n)


def test_out_degree_above_lds_rows_cocktail_party(ctx):
    """K_3400 minus a perfect matching: every vertex has degree 3398, so the lowest-ranked
    one has out-degree 3398 with triangles and 4-cliques over all of N+(a) (the per-neighbour
    arrays and hash in the global slab); every edge's 13 counts and the global counts equal
    the closed forms (pinned against brute force in the oracle tests)."""
    from closed_forms import cocktail_party, cocktail_party_counts
    k = 3400
    rp, col = cocktail_party(k)
    X0, pe0 = cocktail_party_counts(k)
    say(f"cocktail-party-{k} (out-degree above the LDS rows)")
    X, pe = gpu(ctx, k, rp, col)
    assert X == X0
    m = col.size // 2
    want = np.repeat(np.asarray(pe0, dtype=np.uint64)[:, None], m, axis=1)
    np.testing.assert_array_equal(pe, want)
    G, _ = gpu(ctx, k, rp, col, per_edge=False)
    assert G == X0


def test_list_orders_agree():
    """The order of the workgroup work lists (largest work, degree or volume first, smallest
    degree or volume first, ascending rank, pseudo-random: the ordering study of Section 4.3
    / Table 4) changes only the schedule: all seven give the oracle's counts, global and per
    edge."""
    import paper_1608_05138_amd as glt
    n = 20000
    rp, col = gg.chung_lu(n, 200000, 2.1, float(n - 1), 8)
    ref = oracle.count(n, rp, col)["X"]
    c = glt.Context(0)
    try:
        # the defaults are the automatic choices (-1), which a schedule can also ask for
        assert c.schedule()["list_order"] == -1 and c.schedule()["wedge_stream"] == -1
        base = None
        for order in list(range(7)) + [-1]:
            c.set_schedule(list_order=order)
            assert c.schedule()["list_order"] == order
            say(f"list-order {order}")
            X, pe = gpu(c, n, rp, col)
            assert X == ref, order
            if base is None:
                base = pe
            else:
                np.testing.assert_array_equal(pe, base)
        with pytest.raises(glt.GltError):
            c.set_schedule(list_order=-2)
        with pytest.raises(glt.GltError):
            c.set_schedule(wedge_stream=3)
    finally:
        c.close()


def test_wide_edges_two_hubs_all_stream_modes():
    """Two adjacent hubs sharing 50,000 leaves, over sparse ER noise: the edge between them
    has endpoint degrees above 2^31 / dmax, so it takes the 64-bit (wide) accumulators while
    every other edge keeps 32-bit ones; all 13 per-edge counts of every edge must equal the
    oracle's in each stream mode."""
    import paper_1608_05138_amd as glt
    rng = np.random.default_rng(2031)
    n = 70000
    lo, hi = gg.er_pairs(n, 80000, rng)
    leaves = np.arange(2, 50002)
    a = np.concatenate([lo, [0], np.zeros(50000, np.int64), np.ones(50000, np.int64)])
    b = np.concatenate([hi, [1], leaves, leaves])
    keep = a != b
    a, b = a[keep], b[keep]
    key = np.unique(np.minimum(a, b) * n + np.maximum(a, b))
    perm = rng.permutation(n)
    rp, col = gg.csr_from_pairs(n, perm[key // n], perm[key % n])
    d = np.diff(rp)
    assert int(np.sort(d)[-2]) * int(d.max()) >= 2 ** 31
    ref = oracle.count(n, rp, col, per_edge=True)
    for mode in (0, 1, 2):
        c = glt.Context(0)
        try:
            c.set_schedule(wedge_stream=mode)
            say(f"two-hubs mode {mode}")
            X, pe = gpu(c, n, rp, col)
            assert X == ref["X"], mode
            np.testing.assert_array_equal(pe, ref["per_edge"], err_msg=f"mode {mode}")
        finally:
            c.close()


@pytest.mark.parametrize("wide_degree", ["60", "3"])
def test_forced_wide_edges(monkeypatch, wide_degree):
    """Edges whose lower endpoint has degree >= GLT_WIDE_DEGREE forced onto the 64-bit
    accumulators: with 60 a suffix of the oriented edges (at most a quarter) is wide and the
    rest narrow; with 3 more than a quarter would be, so every edge is wide.  Per-edge and
    global counts must equal the oracle's on graphs that reach every triangle and wedge
    path."""
    import paper_1608_05138_amd as glt
    monkeypatch.setenv("GLT_WIDE_DEGREE", wide_degree)
    c = glt.Context(0)
    try:
        cases = [("chung-lu-6000", 6000, gg.chung_lu(6000, 90000, 2.1, 5999.0, 78))]
        rng = np.random.default_rng(9)
        nn = 3000
        lo, hi = gg.er_pairs(nn, 9000, rng)
        iu = np.triu_indices(760, 1)   # out-degrees up to 759: global-bitmap rows
        a = np.concatenate([lo, iu[0]]); b = np.concatenate([hi, iu[1]])
        key = np.unique(np.minimum(a, b) * nn + np.maximum(a, b))
        perm = rng.permutation(nn)
        cases.append(("clique760-noise", nn, gg.csr_from_pairs(nn, perm[key // nn], perm[key % nn])))
        for name, n, (rp, col) in cases:
            check_vs_oracle(c, f"wide-{wide_degree}-{name}", n, rp, col)
    finally:
        c.close()
