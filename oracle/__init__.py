"""CPU oracle for exact 2-, 3- and 4-node graphlet counts -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library (``paper_1608_05138_amd``) and never
imports it.

Contents
* ``glo_oracle.c`` (compiled here with gcc): the brute-force definition (every 3-/4-vertex
  subset, Section 3, Definitions 1-3 and Problem 1) and the paper's edge-centric method
  (Section 4: hash Psi with per-edge tags, clique and cycle neighbour iteration, local and
  unrestricted counts of Section 4.5, global frequencies of Section 4.6).
  ``count_range`` runs that method over a block of edges (partial unrestricted sums and the
  block's per-edge counts), so that long runs proceed block by block.
* ``global_substructures``: global counts of graphs far too large for the edge-centric method,
  from the triangles on every edge (by definition), the 4-cliques and the 4-cycles, each
  counted once at its lowest vertex, through Sections 4.5-4.6.
* ``per_edge_substructures``: per-edge and global counts of such graphs from per-edge
  triangles, 4-cliques, 4-cycles and triangle-weighted sums, each sub-structure enumerated
  once, through the same class-pair formulas as the edge-centric method.
* ``brute_py``: a pure-Python enumeration for tiny graphs that pins the C brute force.

Global counts are returned as Python ints (exact, they exceed 64 bits for large n).
Per-edge counts are ``numpy.uint64`` arrays of shape [13, m] in the slot order
H3, H4, H5, H7, H8, H9, H10, H11, H12, H13, H14, H15, H16.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from itertools import combinations

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "glo_oracle.c")
_LIB = os.path.join(_HERE, "libglo_oracle.so")
_lib = None

GRAPHLETS = ["edge", "2-node-indep", "triangle", "2-star", "3-node-1-edge", "3-node-indep",
             "4-clique", "chordal-cycle", "tailed-triangle", "4-cycle", "3-star", "4-path",
             "4-node-1-triangle", "4-node-2-edge", "4-node-2-star", "4-node-1-edge",
             "4-node-indep"]
# graphlet ids (1-based) of the 13 per-edge slots
EDGE_SLOTS = [3, 4, 5, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16]
# edges of each graphlet H1..H17
GRAPHLET_EDGES = [1, 0, 3, 2, 1, 0, 6, 5, 4, 4, 3, 3, 3, 2, 2, 1, 0]


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.brute_count.argtypes = [ctypes.c_int64, P, P, P, P]
        lib.glo_count.argtypes = [ctypes.c_int64, P, P, ctypes.c_int, P, P, P]
        lib.glo_count_edges.argtypes = [ctypes.c_int64, P, P, ctypes.c_int, P, ctypes.c_int64, P]
        lib.glo_count_range.argtypes = [ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, P, P]
        lib.glo_global_from_c.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P]
        lib.glo_global_substructures.argtypes = [ctypes.c_int64, P, P, ctypes.c_int, P, P, P]
        lib.glo_per_edge_substructures.argtypes = [ctypes.c_int64, P, P, ctypes.c_int, P, P, P]
        for f in (lib.brute_count, lib.glo_count, lib.glo_count_edges, lib.glo_count_range,
                  lib.glo_global_from_c, lib.glo_global_substructures,
                  lib.glo_per_edge_substructures):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _prep(n, row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    if rp.size != n + 1:
        raise ValueError("row_ptr must have n+1 entries")
    return rp, c


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def num_edges(n, row_ptr, col) -> int:
    rp = np.asarray(row_ptr, dtype=np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    return int(np.count_nonzero(np.asarray(col, dtype=np.int64) > src))


def _u128(words):
    return [int(words[2 * i]) | (int(words[2 * i + 1]) << 64) for i in range(17)]


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


def count(n, row_ptr, col, per_edge: bool = False, nthreads: int | None = None):
    """The paper's method.  Returns dict(X=[17 ints], C=[17 ints], per_edge=[13,m] or None)."""
    lib = _load()
    rp, c = _prep(n, row_ptr, col)
    m = num_edges(n, rp, c)
    X = np.zeros(34, dtype=np.uint64)
    C = np.zeros(34, dtype=np.uint64)
    pe = np.zeros((13, m), dtype=np.uint64) if per_edge else None
    rc = lib.glo_count(n, _ptr(rp), _ptr(c), nthreads or default_threads(), _ptr(X), _ptr(C),
                       _ptr(pe) if pe is not None else None)
    if rc != 0:
        raise RuntimeError(f"oracle glo_count failed: {rc}")
    return {"X": _u128(X), "C": _u128(C), "per_edge": pe}


def count_edges(n, row_ptr, col, eids, nthreads: int | None = None):
    """Per-edge counts [13, k] of the listed edges, by the paper's method."""
    lib = _load()
    rp, c = _prep(n, row_ptr, col)
    e = np.ascontiguousarray(eids, dtype=np.int64)
    out = np.zeros((13, e.size), dtype=np.uint64)
    rc = lib.glo_count_edges(n, _ptr(rp), _ptr(c), nthreads or default_threads(), _ptr(e),
                             e.size, _ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle glo_count_edges failed: {rc}")
    return out


def count_range(n, row_ptr, col, k0: int, k1: int, per_edge: bool = False,
                nthreads: int | None = None):
    """The paper's method over edges [k0, k1) only.  Returns dict(C=[17 ints], the block's
    terms of the unrestricted sums; per_edge=[13, k1-k0] or None)."""
    lib = _load()
    rp, c = _prep(n, row_ptr, col)
    C = np.zeros(34, dtype=np.uint64)
    pe = np.zeros((13, max(0, k1 - k0)), dtype=np.uint64) if per_edge else None
    rc = lib.glo_count_range(n, _ptr(rp), _ptr(c), nthreads or default_threads(), k0, k1, _ptr(C),
                             _ptr(pe) if pe is not None else None)
    if rc != 0:
        raise RuntimeError(f"oracle glo_count_range failed: {rc}")
    return {"C": _u128(C), "per_edge": pe}


def global_from_c(n: int, m: int, C):
    """Global counts X1..X17 (Section 4.6) from unrestricted sums C (17 Python ints, as
    count_range returns them, summed over a partition of the edges)."""
    lib = _load()
    words = np.zeros(34, dtype=np.uint64)
    for i, v in enumerate(C):
        v = int(v) % (1 << 128)
        words[2 * i] = v & ((1 << 64) - 1)
        words[2 * i + 1] = v >> 64
    X = np.zeros(34, dtype=np.uint64)
    rc = lib.glo_global_from_c(n, m, _ptr(words), _ptr(X))
    if rc != 0:
        raise RuntimeError(f"oracle glo_global_from_c failed: {rc}")
    return _u128(X)


def global_substructures(n, row_ptr, col, per_edge3: bool = False, nthreads: int | None = None):
    """Global counts from per-edge triangles, 4-cliques and 4-cycles.  Returns dict(X=[17 ints],
    k4, c4, per_edge3=[3, m] (triangles, 2-stars, H5 per edge) or None)."""
    lib = _load()
    rp, c = _prep(n, row_ptr, col)
    m = num_edges(n, rp, c)
    X = np.zeros(34, dtype=np.uint64)
    W = np.zeros(4, dtype=np.uint64)
    pe = np.zeros((3, m), dtype=np.uint64) if per_edge3 else None
    rc = lib.glo_global_substructures(n, _ptr(rp), _ptr(c), nthreads or default_threads(), _ptr(X),
                                      _ptr(pe) if pe is not None else None, _ptr(W))
    if rc != 0:
        raise RuntimeError(f"oracle glo_global_substructures failed: {rc}")
    return {"X": _u128(X), "k4": int(W[0]) | (int(W[1]) << 64), "c4": int(W[2]) | (int(W[3]) << 64),
            "per_edge3": pe}


def per_edge_substructures(n, row_ptr, col, per_edge: bool = True, nthreads: int | None = None):
    """Per-edge and global counts from per-edge triangles, 4-cliques, 4-cycles and
    triangle-weighted sums (each sub-structure enumerated once).  Returns dict(X=[17 ints],
    k4, c4, per_edge=[13, m] or None)."""
    lib = _load()
    rp, c = _prep(n, row_ptr, col)
    m = num_edges(n, rp, c)
    X = np.zeros(34, dtype=np.uint64)
    W = np.zeros(4, dtype=np.uint64)
    pe = np.zeros((13, m), dtype=np.uint64) if per_edge else None
    rc = lib.glo_per_edge_substructures(n, _ptr(rp), _ptr(c), nthreads or default_threads(),
                                        _ptr(X), _ptr(pe) if pe is not None else None, _ptr(W))
    if rc != 0:
        raise RuntimeError(f"oracle glo_per_edge_substructures failed: {rc}")
    return {"X": _u128(X), "k4": int(W[0]) | (int(W[1]) << 64), "c4": int(W[2]) | (int(W[3]) << 64),
            "per_edge": pe}


def brute(n, row_ptr, col, per_edge: bool = False):
    """Brute force from the definition (C).  n <= a few hundred."""
    lib = _load()
    rp, c = _prep(n, row_ptr, col)
    m = num_edges(n, rp, c)
    X = np.zeros(17, dtype=np.uint64)
    pe = np.zeros((13, m), dtype=np.uint64) if per_edge else None
    rc = lib.brute_count(n, _ptr(rp), _ptr(c), _ptr(X), _ptr(pe) if pe is not None else None)
    if rc != 0:
        raise RuntimeError(f"oracle brute_count failed: {rc}")
    return {"X": [int(x) for x in X], "per_edge": pe}


# ---------------------------------------------------------------------------------------
# pure-Python brute force (tiny graphs), written independently of the C code
# ---------------------------------------------------------------------------------------

def _iso_class(vs, adj):
    """Graphlet id of the subgraph induced by vertex tuple vs (2, 3 or 4 vertices), by
    checking isomorphism against explicit Table 1 representatives over all vertex
    permutations."""
    from itertools import permutations
    k = len(vs)
    E = frozenset((i, j) for i in range(k) for j in range(i + 1, k) if adj[vs[i]][vs[j]])
    for gid, (kk, rep) in _REPS.items():
        if kk != k or len(rep) != len(E):
            continue
        for p in permutations(range(k)):
            mapped = frozenset(tuple(sorted((p[a], p[b]))) for a, b in rep)
            if mapped == E:
                return gid
    raise AssertionError("unclassified subgraph")


# Table 1 representatives on vertices 0..k-1
_REPS = {
    1: (2, [(0, 1)]), 2: (2, []),
    3: (3, [(0, 1), (0, 2), (1, 2)]), 4: (3, [(0, 1), (1, 2)]), 5: (3, [(0, 1)]), 6: (3, []),
    7: (4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]),
    8: (4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3)]),           # K4 minus one edge
    9: (4, [(0, 1), (0, 2), (1, 2), (2, 3)]),                   # triangle + pendant
    10: (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),                  # 4-cycle
    11: (4, [(0, 1), (0, 2), (0, 3)]),                          # 3-star
    12: (4, [(0, 1), (1, 2), (2, 3)]),                          # 4-path
    13: (4, [(0, 1), (0, 2), (1, 2)]),                          # triangle + isolated
    14: (4, [(0, 1), (2, 3)]),                                  # two disjoint edges
    15: (4, [(0, 1), (1, 2)]),                                  # 2-star + isolated
    16: (4, [(0, 1)]),                                          # edge + 2 isolated
    17: (4, []),
}


def brute_py(n, pairs):
    """Global counts X1..X17 and per-edge counts (dict edge->13 list) by enumeration."""
    adj = [[False] * n for _ in range(n)]
    for a, b in pairs:
        adj[a][b] = adj[b][a] = True
    X = [0] * 18
    for k in (2, 3, 4):
        for vs in combinations(range(n), k):
            X[_iso_class(vs, adj)] += 1
    per = {}
    for a in range(n):
        for b in range(a + 1, n):
            if not adj[a][b]:
                continue
            cnt = [0] * 18
            others = [w for w in range(n) if w not in (a, b)]
            for w in others:
                cnt[_iso_class((a, b, w), adj)] += 1
            for w, r in combinations(others, 2):
                cnt[_iso_class((a, b, w, r), adj)] += 1
            per[(a, b)] = [cnt[g] for g in EDGE_SLOTS]
    return X[1:], per
