"""Writes stored expected values computed by the CPU oracle only.

Usage: python tests/golden/make_golden.py TARGET [threads]

Targets (every value below comes from ``oracle/``; nothing is read back from the GPU library):

chung_lu_1m          global counts X1..X17 of the Chung-Lu graph n=1e6, m=1e7, exponent 2.1,
                     weight cap 50,000 (graphgen.config_chung_lu_1m), by the paper's
                     edge-centric method -> chung_lu_1m_global.json
chung_lu_1m_per_edge the 13 per-edge counts of every edge of the same graph by the per-edge
                     sub-structure method, then by the paper's edge-centric method run block by
                     block (glo_count_range; blocks checkpointed under _work/golden_ckpt so an
                     interrupted run resumes), which must agree on every count: SHA-256 of each
                     slot's little-endian uint64 array in the caller's edge order, the global
                     counts and the counts of a seeded edge sample -> chung_lu_1m_per_edge.json
rmat_s22             R-MAT scale 22, edge factor 16 (graphgen.config_rmat_s22): per-edge and
                     global counts by the per-edge sub-structure method (the edge-centric method
                     would take hundreds of core-hours here), SHA-256 of each of the 13 per-edge
                     slot arrays, and the 13 counts of a seeded edge sample (uniform edges plus
                     edges at the highest-degree vertices) by the edge-centric method, which
                     must agree -> rmat_s22.json
batch_10k            global counts of each of the 10,000 graphs of the batch mix
                     (graphgen.batch_spec / batch_graph), edge-centric method: a 16-hex digest
                     per graph and the full counts of every 100th graph -> batch_10k.json

Each file records the generator recipe so a reader can regenerate the inputs.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

CKPT = os.path.join(ROOT, "_work", "golden_ckpt")


def log(msg):
    print(f"[golden] {time.strftime('%H:%M:%S')} {msg}", flush=True)


def sha_u64(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


def col_prefix(col):
    return hashlib.sha256(np.ascontiguousarray(col).tobytes()).hexdigest()[:16]


def x_digest(X):
    return hashlib.sha256(",".join(str(int(v)) for v in X).encode()).hexdigest()[:16]


def sample_edges(n, rp, col, k, seed, hubs=4, per_hub=16):
    """Edge ids (shared numbering) of k seeded uniform edges plus up to per_hub edges at each
    of the `hubs` highest-degree vertices, sorted."""
    m = col.size // 2
    rng = np.random.default_rng(seed)
    ids = set(int(x) for x in rng.integers(0, m, size=k))
    rp64 = np.asarray(rp, dtype=np.int64)
    deg = np.diff(rp64)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    up = col > src
    eid_of_slot = np.cumsum(up) - 1
    for h in np.argsort(-deg, kind="stable")[:hubs]:
        for sl in range(int(rp64[h]), int(rp64[h + 1]))[:per_hub]:
            if up[sl]:
                ids.add(int(eid_of_slot[sl]))
            else:   # the same edge, seen from its other endpoint's row
                other = int(col[sl])
                row = np.arange(rp64[other], rp64[other + 1])
                ids.add(int(eid_of_slot[row[col[row] == h][0]]))
    return np.array(sorted(ids), dtype=np.int64)


def write(name, out):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)
    log(f"wrote {name}")


def target_chung_lu_1m(threads):
    n, (rp, col) = gg.config_chung_lu_1m()
    t0 = time.time()
    r = oracle.count(n, rp, col, per_edge=False, nthreads=threads)
    write("chung_lu_1m_global.json", {
        "graph": "graphgen.config_chung_lu_1m(): Chung-Lu n=1000000 m=10000000 gamma=2.1 cap=50000 "
                 f"seed={gg.BASE_SEED + 1}",
        "n": n, "m": int(col.size // 2), "col_sha256_prefix": col_prefix(col),
        "X": [str(x) for x in r["X"]],
        "oracle_seconds": round(time.time() - t0, 1), "oracle_threads": threads,
    })


def edge_sums_check(pe, X):
    """Sum over edges of each per-edge count = (edges of the graphlet) x (its global count)."""
    for s_, gid in enumerate(oracle.EDGE_SLOTS):
        if int(pe[s_].sum(dtype=np.uint64)) % (1 << 64) != (oracle.GRAPHLET_EDGES[gid - 1] * X[gid - 1]) % (1 << 64):
            raise SystemExit(f"edge sum of slot {s_} does not match the global count")


def target_chung_lu_1m_per_edge(threads, blocks=8):
    """Per-edge counts by the per-edge sub-structure method, then by the paper's
    edge-centric method block by block; the two must agree on every count."""
    n, (rp, col) = gg.config_chung_lu_1m()
    m = col.size // 2
    os.makedirs(CKPT, exist_ok=True)
    t0 = time.time()
    sub = oracle.per_edge_substructures(n, rp, col, nthreads=threads)
    t_sub = time.time() - t0
    log(f"per-edge sub-structure method {t_sub:.0f} s")
    pe = sub["per_edge"]
    edge_sums_check(pe, sub["X"])
    cuts = [m * b // blocks for b in range(blocks + 1)]
    t0 = time.time()
    C = [0] * 17
    for b in range(blocks):
        k0, k1 = cuts[b], cuts[b + 1]
        path = os.path.join(CKPT, f"chung_lu_1m_block{b}_of{blocks}.npz")
        if os.path.exists(path):
            z = np.load(path)
            part_pe, part_c = z["pe"], [int(v) for v in z["C"].astype(object)]
            log(f"block {b}: [{k0}, {k1}) from checkpoint")
        else:
            log(f"block {b}: [{k0}, {k1}) ...")
            r = oracle.count_range(n, rp, col, k0, k1, per_edge=True, nthreads=threads)
            part_pe, part_c = r["per_edge"], r["C"]
            np.savez(path + ".tmp.npz", pe=part_pe, C=np.array([str(v) for v in part_c]))
            os.replace(path + ".tmp.npz", path)
            log(f"block {b} done ({time.time() - t0:.0f} s so far)")
        if not np.array_equal(pe[:, k0:k1], part_pe):
            raise SystemExit(f"oracle methods disagree in block {b}")
        C = [C[i] + int(part_c[i]) for i in range(17)]
    X = oracle.global_from_c(n, m, C)
    if X != sub["X"]:
        raise SystemExit("oracle methods disagree on the global counts")
    eids = sample_edges(n, rp, col, 256, 11)
    write("chung_lu_1m_per_edge.json", {
        "graph": "graphgen.config_chung_lu_1m(): Chung-Lu n=1000000 m=10000000 gamma=2.1 cap=50000 "
                 f"seed={gg.BASE_SEED + 1}",
        "n": n, "m": int(m), "col_sha256_prefix": col_prefix(col),
        "method": "per-edge sub-structure method, and the edge-centric method over 8 blocks of the "
                  "shared edge numbering; both gave every count below",
        "X": [str(x) for x in X], "k4": str(sub["k4"]), "c4": str(sub["c4"]),
        "slot_sha256": [sha_u64(pe[s_]) for s_ in range(13)],
        "sample_eids": [int(e) for e in eids],
        "sample_counts": [[int(v) for v in pe[s_, eids]] for s_ in range(13)],
        "oracle_seconds_substructures": round(t_sub, 1), "oracle_threads": threads,
    })


def target_rmat_s22(threads):
    """Per-edge and global counts by the per-edge sub-structure method (the edge-centric
    method would take hundreds of core-hours here), checked on a seeded edge sample (uniform
    edges plus edges at the highest-degree vertices) against the edge-centric method."""
    log("generating R-MAT scale 22")
    n, (rp, col) = gg.config_rmat_s22()
    m = col.size // 2
    t0 = time.time()
    r = oracle.per_edge_substructures(n, rp, col, nthreads=threads)
    t_sub = time.time() - t0
    log(f"per-edge sub-structure method {t_sub:.0f} s")
    pe = r["per_edge"]
    edge_sums_check(pe, r["X"])
    eids = sample_edges(n, rp, col, 384, 12)
    t0 = time.time()
    ref = oracle.count_edges(n, rp, col, eids, nthreads=threads)
    log(f"edge-centric method on {eids.size} sampled edges {time.time() - t0:.0f} s")
    if not np.array_equal(ref, pe[:, eids]):
        raise SystemExit("oracle methods disagree on the sampled edges")
    write("rmat_s22.json", {
        "graph": "graphgen.config_rmat_s22(): R-MAT scale 22 edge factor 16 (0.57,0.19,0.19,0.05) "
                 f"seed={gg.BASE_SEED + 2}, duplicates and self-loops removed, int64 offsets",
        "n": n, "m": int(m), "col_sha256_prefix": col_prefix(col),
        "method": "per-edge sub-structure method (all counts); edge-centric method on the sample",
        "X": [str(x) for x in r["X"]], "k4": str(r["k4"]), "c4": str(r["c4"]),
        "slot_sha256": [sha_u64(pe[s_]) for s_ in range(13)],
        "sample_eids": [int(e) for e in eids],
        "sample_counts": [[int(v) for v in ref[s_]] for s_ in range(13)],
        "oracle_seconds_substructures": round(t_sub, 1), "oracle_threads": threads,
    })


def _batch_one(args):
    spec, threads = args
    n, (rp, col) = gg.batch_graph(spec)
    return oracle.count(n, rp, col, nthreads=threads)["X"]


def target_batch_10k(threads, num=10_000):
    import multiprocessing as mp
    specs = gg.batch_spec(num)
    os.makedirs(CKPT, exist_ok=True)
    path = os.path.join(CKPT, "batch_10k_X.json")
    done = {}
    if os.path.exists(path):
        with open(path) as f:
            done = {int(k): [int(x) for x in v] for k, v in json.load(f).items()}
        log(f"{len(done)} graphs from checkpoint")
    todo = [g for g in range(num) if g not in done]
    t0 = time.time()
    with mp.get_context("fork").Pool(threads) as pool:
        for i, X in enumerate(pool.imap(_batch_one, [(specs[g], 1) for g in todo], chunksize=4)):
            done[todo[i]] = X
            if (i + 1) % 500 == 0 or i + 1 == len(todo):
                with open(path + ".tmp", "w") as f:
                    json.dump({str(k): [str(x) for x in v] for k, v in done.items()}, f)
                os.replace(path + ".tmp", path)
                log(f"{i + 1} of {len(todo)} graphs ({time.time() - t0:.0f} s)")
    write("batch_10k.json", {
        "graphs": "graphgen.batch_spec(10000) / graphgen.batch_graph: n~U{50..5000}, ER or Chung-Lu(2.5) "
                  f"with probability 1/2, mean degree ~U[4,64]; base seed {gg.BASE_SEED + 3}",
        "num_graphs": num, "method": "edge-centric (glo_count per graph)",
        "digest": "first 16 hex digits of SHA-256 of the 17 decimal counts joined by commas",
        "X_digest": [x_digest(done[g]) for g in range(num)],
        "X_every_100": {str(g): [str(x) for x in done[g]] for g in range(0, num, 100)},
    })


def main():
    which = sys.argv[1]
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else oracle.default_threads()
    fn = {"chung_lu_1m": target_chung_lu_1m, "chung_lu_1m_per_edge": target_chung_lu_1m_per_edge,
          "rmat_s22": target_rmat_s22, "batch_10k": target_batch_10k}.get(which)
    if fn is None:
        raise SystemExit("unknown target")
    fn(threads)


if __name__ == "__main__":
    main()
