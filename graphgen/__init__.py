"""Seeded synthetic graph generators shared by the oracle, the tests and the benchmark.

This module only draws random simple undirected graphs and lays them out as CSR arrays.
It holds none of the counting arithmetic: both the GPU library and the CPU oracle read the
arrays it returns, and neither imports the other.

Graph families follow the workloads the paper evaluates on (power-law social/web graphs
and the Erdos-Renyi comparison graphs of its Experiments section):

* ``er(n, m, seed)``: m distinct uniform vertex pairs, no self-loops.
* ``chung_lu(n, m, gamma, cap, seed)``: expected-degree model, weights (i+1)^(-1/(gamma-1))
  rescaled to mean 2m/n and capped, both endpoints drawn proportionally to weight; self-loops
  and duplicates are dropped until exactly m unique edges remain. Vertex ids are shuffled.
* ``rmat(scale, edge_factor, abcd, seed)``: recursive-matrix sampling, bit by bit, without
  noise; self-loops and duplicates removed, the result symmetrised.
* ``batch_spec`` / ``batch_graph``: the mixed batch of small ER / Chung-Lu graphs.

Every CSR is symmetric: ``row_ptr`` has n+1 entries, ``col`` holds both directions of every
edge, neighbours within a row in generation order (not sorted).
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 160805138
_M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One step of the SplitMix64 output function (Steele, Lea, Flood 2014)."""
    x = (x + 0x9E3779B97F4A7C15) & _M64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def graph_seed(base: int, index: int) -> int:
    """Seed for graph ``index`` of a family drawn from ``base``."""
    return splitmix64((base ^ index) & _M64)


# --------------------------------------------------------------------------------------
# edge-list helpers
# --------------------------------------------------------------------------------------

def _canon_keys(a: np.ndarray, b: np.ndarray, n: int) -> np.ndarray:
    lo = np.minimum(a, b).astype(np.int64)
    hi = np.maximum(a, b).astype(np.int64)
    keep = lo != hi
    return lo[keep] * n + hi[keep]


def _first_unique(keys: np.ndarray) -> np.ndarray:
    """Unique keys in order of first appearance."""
    _, idx = np.unique(keys, return_index=True)
    idx.sort()
    return keys[idx]


def csr_from_pairs(n: int, lo: np.ndarray, hi: np.ndarray, offsets64: bool = False):
    """Symmetric CSR from undirected pairs (no self-loops, no duplicates).

    Returns (row_ptr, col) with row_ptr int32 (or int64) of length n+1, col int32 of 2m.
    """
    lo = np.asarray(lo, dtype=np.int64)
    hi = np.asarray(hi, dtype=np.int64)
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    order = np.argsort(src, kind="stable")
    col = dst[order].astype(np.int32)
    deg = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    if not offsets64:
        if row_ptr[-1] > np.iinfo(np.int32).max:
            raise ValueError("2m does not fit int32 offsets")
        row_ptr = row_ptr.astype(np.int32)
    return row_ptr, col


def pairs_from_keys(keys: np.ndarray, n: int):
    return keys // n, keys % n


# --------------------------------------------------------------------------------------
# families
# --------------------------------------------------------------------------------------

def er_pairs(n: int, m: int, rng: np.random.Generator):
    maxm = n * (n - 1) // 2
    if m > maxm:
        raise ValueError(f"m={m} exceeds C(n,2)={maxm}")
    if m == 0:
        e = np.zeros(0, dtype=np.int64)
        return e, e
    if m > maxm // 2:
        # dense: choose the edge set as a random subset of all pairs
        iu = np.triu_indices(n, 1)
        pick = rng.permutation(maxm)[:m]
        return iu[0][pick].astype(np.int64), iu[1][pick].astype(np.int64)
    keys = np.zeros(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        k = int(need * 1.2) + 16
        a = rng.integers(0, n, size=k)
        b = rng.integers(0, n, size=k)
        keys = _first_unique(np.concatenate([keys, _canon_keys(a, b, n)]))
    keys = keys[:m]
    return pairs_from_keys(keys, n)


def er(n: int, m: int, seed: int, offsets64: bool = False):
    rng = np.random.default_rng(seed)
    lo, hi = er_pairs(n, m, rng)
    return csr_from_pairs(n, lo, hi, offsets64)


def chung_lu_weights(n: int, m: int, gamma: float, cap: float) -> np.ndarray:
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    target = 2.0 * m
    for _ in range(100):
        w *= target / w.sum()
        over = w > cap
        if not over.any():
            break
        w[over] = cap
    return w


def chung_lu_pairs(n: int, m: int, gamma: float, cap: float, rng: np.random.Generator):
    maxm = n * (n - 1) // 2
    if m > maxm:
        raise ValueError("m exceeds C(n,2)")
    w = chung_lu_weights(n, m, gamma, cap)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    keys = np.zeros(0, dtype=np.int64)
    rounds = 0
    while keys.size < m:
        need = m - keys.size
        k = int(need * 1.3) + 64
        a = np.searchsorted(cdf, rng.random(k), side="right")
        b = np.searchsorted(cdf, rng.random(k), side="right")
        a = np.minimum(a, n - 1)
        b = np.minimum(b, n - 1)
        keys = _first_unique(np.concatenate([keys, _canon_keys(a, b, n)]))
        rounds += 1
        if rounds > 200:
            raise RuntimeError("chung_lu: cannot reach m unique edges (graph too dense)")
    keys = keys[:m]
    lo, hi = pairs_from_keys(keys, n)
    perm = rng.permutation(n)
    return perm[lo], perm[hi]


def chung_lu(n: int, m: int, gamma: float, cap: float, seed: int, offsets64: bool = False):
    rng = np.random.default_rng(seed)
    lo, hi = chung_lu_pairs(n, m, gamma, cap, rng)
    return csr_from_pairs(n, lo, hi, offsets64)


def rmat_pairs(scale: int, edge_factor: int, abcd, rng: np.random.Generator,
               chunk: int = 1 << 23):
    a, b, c, d = abcd
    n = 1 << scale
    total = edge_factor * n
    out = []
    done = 0
    while done < total:
        k = min(chunk, total - done)
        src = np.zeros(k, dtype=np.int64)
        dst = np.zeros(k, dtype=np.int64)
        for _ in range(scale):
            r = rng.random(k)
            # quadrant: a -> (0,0), b -> (0,1), c -> (1,0), d -> (1,1)
            sbit = (r >= a + b).astype(np.int64)
            dbit = (((r >= a) & (r < a + b)) | (r >= a + b + c)).astype(np.int64)
            src = (src << 1) | sbit
            dst = (dst << 1) | dbit
        out.append(_canon_keys(src, dst, n))
        done += k
    keys = np.unique(np.concatenate(out))
    return pairs_from_keys(keys, n)


def rmat(scale: int, edge_factor: int, abcd, seed: int, offsets64: bool = True):
    rng = np.random.default_rng(seed)
    lo, hi = rmat_pairs(scale, edge_factor, abcd, rng)
    return csr_from_pairs(1 << scale, lo, hi, offsets64)


# --------------------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------------------

def config_er_1k(seed_offset: int = 0):
    """Erdos-Renyi G(n=1000, m=10000), int32 CSR."""
    return 1000, er(1000, 10_000, BASE_SEED + 0 + seed_offset)


def config_chung_lu_1m(seed_offset: int = 0):
    """Chung-Lu n=1e6, m=1e7, exponent 2.1, weight cap 50,000, int32 CSR."""
    n = 1_000_000
    return n, chung_lu(n, 10_000_000, 2.1, 50_000.0, BASE_SEED + 1 + seed_offset)


def config_rmat_s22(seed_offset: int = 0):
    """R-MAT scale 22, edge factor 16, (0.57,0.19,0.19,0.05), int64 row offsets."""
    scale = 22
    return 1 << scale, rmat(scale, 16, (0.57, 0.19, 0.19, 0.05), BASE_SEED + 2 + seed_offset)


def batch_spec(num_graphs: int = 10_000, base: int = BASE_SEED + 3):
    """Per-graph (model, n, m, seed) of the mixed batch.

    n ~ U{50..5000}; model ER or Chung-Lu (exponent 2.5) with probability 1/2 each; average
    degree ~ U[4, 64], clamped to n-1 (ER) or (n-1)/2 (Chung-Lu); m = round(n * dbar / 2).
    """
    specs = []
    for g in range(num_graphs):
        s = graph_seed(base, g)
        rng = np.random.default_rng(s)
        n = int(rng.integers(50, 5001))
        model = "er" if rng.random() < 0.5 else "cl"
        dbar = float(rng.uniform(4.0, 64.0))
        cap = (n - 1) if model == "er" else (n - 1) / 2.0
        m = int(round(n * min(dbar, cap) / 2.0))
        specs.append((model, n, m, int(rng.integers(0, 2**63 - 1))))
    return specs


def batch_graph(spec):
    model, n, m, s = spec
    if model == "er":
        return n, er(n, m, s)
    return n, chung_lu(n, m, 2.5, float(n - 1), s)


def pack_batch(graphs):
    """Pack (n, (row_ptr, col)) graphs into one buffer set with per-graph bases.

    Returns dict with vtx_base int64[B+1] (graph g's rows start at row_ptr[vtx_base[g]+g]),
    slot_base int64[B+1] (graph g's col entries start at slot_base[g]), row_ptr int32 (local
    offsets, n_g+1 per graph), col int32 (local vertex ids).
    """
    B = len(graphs)
    vtx_base = np.zeros(B + 1, dtype=np.int64)
    slot_base = np.zeros(B + 1, dtype=np.int64)
    for g, (n, (rp, col)) in enumerate(graphs):
        vtx_base[g + 1] = vtx_base[g] + n
        slot_base[g + 1] = slot_base[g] + col.size
    row_ptr = np.concatenate([np.asarray(rp, dtype=np.int32) for _, (rp, _) in graphs]) \
        if B else np.zeros(0, dtype=np.int32)
    col = np.concatenate([np.asarray(c, dtype=np.int32) for _, (_, c) in graphs]) \
        if B else np.zeros(0, dtype=np.int32)
    return {"vtx_base": vtx_base, "slot_base": slot_base, "row_ptr": row_ptr, "col": col}


# --------------------------------------------------------------------------------------
# small structured graphs (closed-form checks and edge cases)
# --------------------------------------------------------------------------------------

def complete(n):
    iu = np.triu_indices(n, 1)
    return n, csr_from_pairs(n, iu[0], iu[1])


def cycle(n):
    a = np.arange(n)
    return n, csr_from_pairs(n, a, (a + 1) % n)


def path(n):
    a = np.arange(n - 1)
    return n, csr_from_pairs(n, a, a + 1)


def star(s):
    return s + 1, csr_from_pairs(s + 1, np.zeros(s, dtype=np.int64), np.arange(1, s + 1))


def complete_bipartite(a, b):
    x, y = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return a + b, csr_from_pairs(a + b, x.ravel(), y.ravel())


def from_pairs(n, pairs):
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return n, csr_from_pairs(n, pairs[:, 0], pairs[:, 1])


def complement(n, row_ptr, col):
    """Complement graph (same vertex set) as CSR."""
    adj = np.zeros((n, n), dtype=bool)
    src = np.repeat(np.arange(n), np.diff(np.asarray(row_ptr, dtype=np.int64)))
    adj[src, col] = True
    iu = np.triu_indices(n, 1)
    keep = ~adj[iu]
    return n, csr_from_pairs(n, iu[0][keep], iu[1][keep])


def shuffle_rows(row_ptr, col, seed):
    """Same graph, neighbours permuted within each row."""
    rng = np.random.default_rng(seed)
    rp = np.asarray(row_ptr, dtype=np.int64)
    col = np.array(col, copy=True)
    for i in range(rp.size - 1):
        s, e = rp[i], rp[i + 1]
        if e - s > 1:
            col[s:e] = col[s:e][rng.permutation(e - s)]
    return col


def relabel(n, row_ptr, col, perm):
    """Same graph with vertex x renamed perm[x]."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    src = np.repeat(np.arange(n), np.diff(rp))
    a = perm[src]
    b = perm[np.asarray(col, dtype=np.int64)]
    keep = a < b
    return n, csr_from_pairs(n, a[keep], b[keep], offsets64=rp.dtype == np.int64 and False)
