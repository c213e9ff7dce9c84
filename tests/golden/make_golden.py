"""Writes stored expected values computed by the CPU oracle only.

Usage: python tests/golden/make_golden.py chung_lu_1m [threads]

chung_lu_1m: global counts X1..X17 of the Chung-Lu graph n=1e6, m=1e7, exponent 2.1,
weight cap 50,000 (graphgen.config_chung_lu_1m), by the oracle's edge-centric method.
The file records the generator recipe so a reader can regenerate the graph.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402


def main():
    which = sys.argv[1]
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else oracle.default_threads()
    if which != "chung_lu_1m":
        raise SystemExit("unknown target")
    n, (rp, col) = gg.config_chung_lu_1m()
    t0 = time.time()
    r = oracle.count(n, rp, col, per_edge=False, nthreads=threads)
    dt = time.time() - t0
    out = {
        "graph": "graphgen.config_chung_lu_1m(): Chung-Lu n=1000000 m=10000000 gamma=2.1 cap=50000 "
                 f"seed={gg.BASE_SEED + 1}",
        "n": n, "m": int(col.size // 2),
        "col_sha256_prefix": __import__("hashlib").sha256(np.ascontiguousarray(col).tobytes()).hexdigest()[:16],
        "X": [str(x) for x in r["X"]],
        "oracle_seconds": round(dt, 1), "oracle_threads": threads,
    }
    with open(os.path.join(HERE, "chung_lu_1m_global.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
