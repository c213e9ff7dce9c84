"""Benchmark: exact 4-node graphlet counts (global + per-edge) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat_s22]

One step is one full glt_count call (validation, degree-order relabel, sorted oriented CSR,
triangle / 4-clique pass, per-edge gather pass, 4-cycle wedge pass, combine and 128-bit
reduction) producing all 17 global counts and the 13 per-edge counts of every edge, with
the input CSR already resident in HBM.  The default workload is the largest single-graph
one, R-MAT scale 22 (edge factor 16, 64.2M edges); the Chung-Lu graph (10^6 vertices, 10^7
edges) is timed in the same run and reported beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X published HBM3E bandwidth

# Measured HBM traffic (bytes per execution of each kernel group: FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0, summed over the group's launches in one step) per workload, per-edge run:
# rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE, each a separate run of
# `python3 bench.py --workload W --steps 1 --warmup 0 --no-cpu-baseline [--no-side-workload]
# --no-probe`.  The scales come from two calibration points: a 1 GiB device copy
# (--copy-probe) reads FETCH_SIZE = 0.5 GiB and writes WRITE_SIZE = 1.0 GiB, and the
# library's read-only probe over 1 GiB (--read-probe) reads FETCH_SIZE = 0.5 GiB.  The
# figures belong to the kernel sources with the hash below and are reported only while
# they are unchanged.
TRAFFIC_SOURCES = ["paper_1608_05138_amd/csrc/count.hip", "paper_1608_05138_amd/csrc/prep.hip",
                   "paper_1608_05138_amd/csrc/glt_internal.h", "paper_1608_05138_amd/csrc/prims.h",
                   "paper_1608_05138_amd/csrc/api.hip"]   # api.hip: the schedule the call runs with
TRAFFIC = {
    "sha256": "a32756adea52ce7d0b9e11a89f021c8a047c6674208b23aff82e4616f6de318b",
    "workloads": {
        "rmat_s22": {"tri_wave": 26754102624, "tri_wg": 171670047392,
                     "gather_wave": 3116758560, "gather_wg": 111686691360,
                     "wedge_wave": 73624096, "wedge_mid": 3706287072,
                     "wedge_wg": 81436944512, "wedge_huge": 465226400000},
        "chung_lu_1m": {"tri_wave": 3302695552, "tri_wg": 3941510144,
                        "gather_wave": 1472885888, "gather_wg": 2902371008,
                        "wedge_wave": 82312128, "wedge_mid": 3526405280,
                        "wedge_wg": 8986584000, "wedge_huge": 33792},
    },
}


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        try:
            with open(os.path.join(ROOT, rel), "rb") as f:
                h.update(f.read())
        except OSError:
            return None
    return h.hexdigest()


def measured_traffic(workload, per_edge, group):
    rec = TRAFFIC["workloads"].get(workload)
    if rec is None or not per_edge or TRAFFIC["sha256"] is None or sources_sha256() != TRAFFIC["sha256"]:
        return None
    return rec.get(group)


WORKLOADS = {
    "chung_lu_1m": ("Chung-Lu n=1,000,000 m=10,000,000 exponent 2.1 weight cap 50,000, int32 CSR",
                    "config_chung_lu_1m"),
    "er_1k": ("Erdos-Renyi n=1000 m=10000, int32 CSR", "config_er_1k"),
    "rmat_s22": ("R-MAT scale 22 edge factor 16 (0.57,0.19,0.19,0.05), int64 offsets", "config_rmat_s22"),
}

# kernel groups timed by the library (HIP events on the call's stream) and their kernels
GROUPS = {"tri_wave": "k_tri_wave", "tri_wg": "k_tri_blk", "gather_wave": "k_gather_wave",
          "gather_wg": "k_gather_blk", "wedge_wave": "k_wedge (wave class: 64 threads, 4 per block)",
          "wedge_mid": "k_wedge (mid class: 64 threads, one per block)",
          "wedge_wg": "k_wedge (workgroup class: 256 threads)",
          "wedge_huge": "k_wedge (huge class: 1024 threads, one resident per CU)"}


def _gen_batch_graph(spec):
    import graphgen as gg
    return gg.batch_graph(spec)


# Host processes that generate the batch and served graphs (not timed).  1: threads of this
# process instead (numpy releases the interpreter lock in most of the work): under a
# profiler that runs threads of its own in the process (rocprofv3 --pmc), forked generators
# can deadlock on a lock one of those threads held at the fork.
GEN_PROCS = [max(1, min(16, len(os.sched_getaffinity(0))))]


def _gen_map(fn, items, chunksize):
    import multiprocessing as mp
    from multiprocessing.pool import ThreadPool
    if GEN_PROCS[0] <= 1:
        with ThreadPool(max(1, min(16, len(os.sched_getaffinity(0))))) as pool:
            return pool.map(fn, items, chunksize=chunksize)
    with mp.get_context("fork").Pool(GEN_PROCS[0]) as pool:
        return pool.map(fn, items, chunksize=chunksize)


def gen_batch(num_graphs, base=None):
    """The mixed batch, generated in parallel host processes (not timed)."""
    import graphgen as gg
    specs = gg.batch_spec(num_graphs) if base is None else gg.batch_spec(num_graphs, base=base)
    return specs, _gen_map(_gen_batch_graph, specs, 16)


def _gen_large(seed):
    import graphgen as gg
    n = 200_000
    return n, gg.chung_lu(n, 2_000_000, 2.5, float(n - 1), seed)


def gen_served_pools(pool_small, pool_large):
    """The served benchmark's request pools (small graphs of the batch mix, large Chung-Lu
    graphs), generated in parallel host processes before any device work."""
    import graphgen as gg
    print(f"[bench] generating request pool: {pool_small} small + {pool_large} large",
          file=sys.stderr, flush=True)
    specs = gg.batch_spec(pool_small, base=gg.BASE_SEED + 4)
    small = _gen_map(_gen_batch_graph, specs, 8)
    large = _gen_map(_gen_large, [gg.graph_seed(gg.BASE_SEED + 5, i) for i in range(pool_large)], 1)
    return small, large


def bench_served(args, pools=None, emit=True):
    """Open-loop Poisson request stream against the continuous-batching server, beside the
    same stream served one request per launch (FIFO).  Latency is measured from each
    request's scheduled arrival time."""
    import threading

    import numpy as np

    import graphgen as gg
    import paper_1608_05138_amd as glt

    small, large = pools if pools is not None else gen_served_pools(args.pool_small, args.pool_large)
    ctx = glt.Context(0)
    alone_small = [ctx.count(rp, col, n=n)[0] for n, (rp, col) in small]
    alone_large = [ctx.count(rp, col, n=n)[0] for n, (rp, col) in large]
    ctx.close()
    rng = np.random.default_rng(gg.BASE_SEED + 6)
    arrivals = []
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / args.rate))
        if t >= args.serve_seconds:
            break
        if large and rng.random() < 0.01:
            arrivals.append((t, 1, int(rng.integers(0, len(large)))))
        else:
            arrivals.append((t, 0, int(rng.integers(0, len(small)))))

    def serve(max_batch_graphs):
        srv = glt.Server(0, max_batch_graphs=max_batch_graphs)
        got = {}
        done_flag = threading.Event()

        def poller():
            while not done_flag.is_set() or len(got) < len(arrivals):
                for r in srv.poll(256, 2000):
                    got[r["req_id"]] = r
                if done_flag.is_set() and len(got) >= len(arrivals):
                    break

        th = threading.Thread(target=poller, daemon=True)
        th.start()
        t0 = srv.clock() + 0.2
        sched = np.empty(len(arrivals))
        next_note = time.time() + 10.0

        def note(what):
            print(f"[bench] {what}: {len(got)} of {len(arrivals)} requests done", file=sys.stderr, flush=True)

        for i, (ta, kind, idx) in enumerate(arrivals):
            if time.time() >= next_note:
                note(f"submitted {i}")
                next_note += 10.0
            target = t0 + ta
            while True:
                d = target - srv.clock()
                if d <= 0:
                    break
                if d > 0.0005:
                    time.sleep(d - 0.0003)
            n, (rp, col) = (large if kind else small)[idx]
            rc = srv.submit(rp, col, i, n=n)
            if rc != 0:
                raise RuntimeError(f"submit failed: {rc}")
            sched[i] = target
        done_flag.set()
        deadline = time.time() + 600
        while len(got) < len(arrivals) and time.time() < deadline:
            time.sleep(0.01)
            if time.time() >= next_note:
                note("all submitted")
                next_note += 10.0
        th.join(timeout=5)
        srv.close()
        if len(got) < len(arrivals):
            raise RuntimeError(f"only {len(got)} of {len(arrivals)} requests completed")
        lat = np.array([got[i]["t_done"] - sched[i] for i in range(len(arrivals))]) * 1e3
        kinds = np.array([kind for (_, kind, _) in arrivals])
        bad = sum(1 for i, (ta, kind, idx) in enumerate(arrivals)
                  if got[i]["status"] != 0 or got[i]["X"] != (alone_large if kind else alone_small)[idx])
        span = max(got[i]["t_done"] for i in got) - t0
        sizes = [got[i]["batch_graphs"] for i in got]

        def pct(x):
            return None if x.size == 0 else {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99)),
                                             "max": float(x.max())}
        return {"completed": len(got), "req_per_s": len(got) / span, "latency_ms": pct(lat),
                "latency_ms_small": pct(lat[kinds == 0]), "latency_ms_large": pct(lat[kinds == 1]),
                "mean_batch": float(np.mean(sizes)), "mismatches_vs_alone": bad}

    print(f"[bench] serving {len(arrivals)} requests over {args.serve_seconds} s (continuous batching)",
          file=sys.stderr, flush=True)
    cb = serve(0)
    print(f"[bench] continuous batching: {cb}", file=sys.stderr, flush=True)
    fifo = None
    if not args.no_per_graph:
        print("[bench] same stream, one request per launch", file=sys.stderr, flush=True)
        fifo = serve(1)
        print(f"[bench] per-request FIFO: {fifo}", file=sys.stderr, flush=True)
    line = {
        "metric": "served requests/sec for exact 4-node motif counts, Poisson arrivals (1 GPU); p99 latency",
        "value": cb["req_per_s"], "unit": "requests/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "served", "rate_per_s": args.rate, "seconds": args.serve_seconds,
                   "requests": len(arrivals), "pool": f"{len(small)} mixed small + {len(large)} "
                   "Chung-Lu n=200000 m=2000000 (1% of arrivals)", "latency": "t_done - scheduled arrival"},
        "latency_ms": cb["latency_ms"], "continuous_batching": cb, "per_request_fifo": fifo,
    }
    if emit:
        print(json.dumps(line), flush=True)
    return line


def bench_batch(args, graphs=None, emit=True):
    """Batched global counts of the 10,000-graph mix: graphs/s of one glt_count_batch call,
    next to the plain per-graph path (glt_count looped over the same graphs)."""
    import numpy as np
    import torch

    import graphgen as gg
    import paper_1608_05138_amd as glt

    if graphs is None:
        print(f"[bench] generating {args.batch_graphs} batch graphs", file=sys.stderr, flush=True)
        _, graphs = gen_batch(args.batch_graphs)
    packed = gg.pack_batch(graphs)
    m_total = int(packed["col"].size // 2)
    dev = torch.device("cuda:0")
    dpk = dict(packed)
    dpk["row_ptr"] = torch.from_numpy(packed["row_ptr"]).to(dev)
    dpk["col"] = torch.from_numpy(packed["col"]).to(dev)
    ctx = glt.Context(0)
    stream = torch.cuda.current_stream(dev).cuda_stream
    tuned = None
    if args.schedule:
        ctx.set_schedule(**parse_schedule(args.schedule))
    elif not args.no_autotune:
        # the schedule is picked on a separate draw of the same mix (other seeds), not on the
        # timed graphs
        _, tgraphs = gen_batch(args.tune_graphs, base=gg.BASE_SEED + 1003)
        tpk = gg.pack_batch(tgraphs)
        tpk["row_ptr"] = torch.from_numpy(tpk["row_ptr"]).to(dev)
        tpk["col"] = torch.from_numpy(tpk["col"]).to(dev)
        best, best_ms = ctx.autotune_batch(tpk, stream=stream)
        tuned = {"schedule": best, "tuned_on": f"{len(tgraphs)} graphs of the same mix drawn with other seeds",
                 "tuned_device_ms": round(best_ms, 3)}
        print(f"[bench] autotuned schedule {best} ({best_ms:.2f} ms on the tuning batch)", file=sys.stderr, flush=True)
        del tpk
    if args.stream_mode is not None:
        ctx.set_schedule(wedge_stream=args.stream_mode)
    print(f"[bench] batch: {len(graphs)} graphs, {m_total} edges; warmup {args.warmup}", file=sys.stderr,
          flush=True)
    for _ in range(args.warmup):
        raw = ctx.count_batch(dpk, stream=stream, raw=True)
    torch.cuda.synchronize()
    timings = []
    # each step is one glt_count_batch call with its 17 x B 128-bit results in host memory; the
    # binding's conversion of them into Python ints is left out of the timed loop
    t0 = time.perf_counter()
    for _ in range(args.steps):
        raw = ctx.count_batch(dpk, stream=stream, raw=True)
        timings.append(ctx.last_timing())
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    res = glt.batch_counts(raw)
    timing = mean_timing(timings)
    work = ctx.last_work()
    # plain per-graph path over the same device-resident graphs (one call per graph)
    per_graph_ms = None
    if not args.no_per_graph:
        offs_v, offs_s = packed["vtx_base"], packed["slot_base"]
        views = []
        for g in range(len(graphs)):
            n = int(offs_v[g + 1] - offs_v[g])
            r0 = int(offs_v[g]) + g
            views.append((n, dpk["row_ptr"][r0: r0 + n + 1], dpk["col"][int(offs_s[g]): int(offs_s[g + 1])]))
        for n, rpv, cv in views[:50]:
            ctx.count(rpv, cv, n=n, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        alone = [ctx.count(rpv, cv, n=n, stream=stream)[0] for n, rpv, cv in views]
        torch.cuda.synchronize()
        per_graph_ms = (time.perf_counter() - t0) * 1e3
        assert alone == res, "batched and per-graph counts differ"
    maxdeg = int(np.diff(packed["row_ptr"]).max()) if packed["row_ptr"].size else 0
    line = {
        "metric": "graphs/sec for exact 4-node motif counts of a 10,000-graph batch (1 GPU)",
        "value": len(graphs) / (ms * 1e-3), "unit": "graphs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "batch_10k", "graphs": len(graphs), "edges": m_total,
                   "mix": "n~U{50..5000}, ER or Chung-Lu(2.5) 1/2 each, mean degree ~U[4,64]",
                   "outputs": "global X1..X17 (u128) per graph"},
        "edges_per_s": m_total / (ms * 1e-3),
        "per_graph_path": None if per_graph_ms is None else {
            "ms": round(per_graph_ms, 1), "graphs_per_s": len(graphs) / (per_graph_ms * 1e-3)},
        "kernel_groups_ms": {k: round(float(v), 4) for k, v in timing.items()},
        "kernel_groups_note": ("the library counts a batch of at least 64 graphs and 2^26 entries as four "
                               "parts at the same time: each group's time is the longest part's, and the "
                               "groups of different parts overlap") if len(graphs) >= 64 and 2 * m_total >= (1 << 26)
                              else None,
        "work": work,
        "autotune": tuned,
        "schedule": ctx.schedule(),
        "roofline": roofline(timing, work, False, acc_width(maxdeg),
                             prep=prep_bytes(int(packed["vtx_base"][-1]), m_total, 4)),
    }
    ctx.close()
    if emit:
        print(json.dumps(line), flush=True)
    return line


# The short runs of the batch and served workloads reported beside the R-MAT line (the full
# lines come from --workload batch_10k and --workload served).  The batch runs with the
# schedule the autotuner picks for it on a separate draw of the mix (wave bound 128, mid
# bound 4096, dense window 4096, stream mode 1), without re-tuning.
SIDE_BATCH = {"steps": 3, "warmup": 1,
              "schedule": "wedge_wave_max=128,wedge_mid_max=4096,wedge_dense=4096,wedge_stream=1"}
SIDE_SERVED = {"seconds": 10.0, "pool_small": 2000, "pool_large": 16}


def side_batch_run(args, graphs):
    import copy
    a = copy.copy(args)
    a.steps, a.warmup = SIDE_BATCH["steps"], SIDE_BATCH["warmup"]
    a.schedule, a.no_per_graph, a.stream_mode = SIDE_BATCH["schedule"], True, None
    try:
        line = bench_batch(a, graphs=graphs, emit=False)
    except Exception as exc:   # an auxiliary measurement: reported, never fatal to the line
        return {"workload": "batch_10k", "error": repr(exc)}
    out = {k: line[k] for k in ("value", "unit", "ms_per_step", "steps", "warmup", "kernel_groups_ms", "schedule")}
    out.update({"workload": "batch_10k", "config": line["config"],
                "note": "short run; the full line: bench.py --workload batch_10k"})
    return out


def side_served_run(args, pools):
    import copy
    a = copy.copy(args)
    a.serve_seconds, a.no_per_graph = SIDE_SERVED["seconds"], True
    try:
        line = bench_served(a, pools=pools, emit=False)
    except Exception as exc:   # an auxiliary measurement: reported, never fatal to the line
        return {"workload": "served", "error": repr(exc)}
    cb = line["continuous_batching"]
    return {"workload": "served", "value": line["value"], "unit": line["unit"], "latency_ms": cb["latency_ms"],
            "latency_ms_small": cb["latency_ms_small"], "latency_ms_large": cb["latency_ms_large"],
            "mean_batch": cb["mean_batch"], "mismatches_vs_alone": cb["mismatches_vs_alone"],
            "config": line["config"], "note": "short run; the full line: bench.py --workload served"}


def group_bytes(work, per_edge, acc_bytes, records=True):
    """Algorithmic bytes of each counting kernel group: the bytes the method must move per
    unit of work (list entry, triangle, wedge), times the units the call counted.
    Triangle pass: one 4 B id per out-list entry scanned, and per triangle its 4 B triangle
    credit plus (per-edge mode) one 4-clique credit, plus, with triangle records, the 8 B
    record written and read back.  Gather pass: per triangle its record (or, without records,
    the re-scanned list entries), the three 4 B triangle counts and two credits.  Wedge pass:
    per wedge one 4 B top id plus (per-edge mode) one 4-cycle credit.  Credits are acc_bytes
    wide."""
    ab = acc_bytes
    rec = 16 if records else 0
    wb = 4 + (ab if per_edge else 0)
    tb = 4 + (ab if per_edge else 0) + rec
    out = {
        "tri_wave": 4 * work["tri_list_wave"] + tb * work["triangles_wave"],
        "tri_wg": 4 * work["tri_list_wg"] + tb * work["triangles_wg"],
        "wedge_wave": wb * work["wedges_wave"],
        "wedge_mid": wb * work["wedges_mid"],
        "wedge_wg": wb * work["wedges_wg"],
        "wedge_huge": wb * work["wedges_huge"],
    }
    if per_edge:
        for path in ("wave", "wg"):
            scan = 8 * work["triangles_" + path] if records else 4 * work["tri_list_" + path]
            out["gather_" + path] = scan + (12 + 2 * ab) * work["triangles_" + path]
    return out


def prep_bytes(n, m, rp_width):
    """Algorithmic bytes of preprocessing (validation, degree order, sorted and oriented
    CSR): the input CSR read once (4 B per column entry, rp_width B per offset), the
    relabelled, row-sorted CSR written once (4 B per entry and per offset) and the oriented
    CSR written once (4 B per oriented edge and per offset)."""
    return (8 * m + rp_width * (n + 1)) + (8 * m + 4 * (n + 1)) + (4 * m + 4 * (n + 1))


def group_atomics(work, per_edge):
    """Global atomic credits the 4-cycle wedge classes issue per launch: one per wedge (its
    4-cycle credit to the top edge w - x) in per-edge mode; global-only counting credits in
    LDS and adds one total per group."""
    if not per_edge:
        return {}
    return {"wedge_" + c: work["wedges_" + c] for c in ("wave", "mid", "wg", "huge")}


def roofline(timing, work, per_edge, acc_bytes, workload=None, records=True, prep=None, atomic_rate=None):
    """The roofline record of the kernel group with the largest HIP-event time (counting
    groups and, when prep is given, preprocessing): its algorithmic bytes over its time
    against HBM's peak and, for a wedge class in per-edge mode, its global atomic credits
    over its time against the measured rate of such atomics (atomic_rate, atomics/s)."""
    gb = group_bytes(work, per_edge, acc_bytes, records)
    if prep is not None:
        gb["prep"] = prep
    dom = max(gb, key=lambda g: timing[g])
    achieved = gb[dom] / (timing[dom] * 1e-3) / 1e9
    rec = {"bound": "hbm", "kernel": GROUPS.get(dom, dom), "group": dom, "achieved": round(achieved, 1),
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": measured_traffic(workload, per_edge, dom),
           "alg_bytes": int(gb[dom]), "kernel_ms": round(float(timing[dom]), 4)}
    atoms = group_atomics(work, per_edge)
    if dom in atoms and atomic_rate:
        a = atoms[dom] / (timing[dom] * 1e-3)
        rec["atomic_roof"] = {"achieved": round(a / 1e9, 3), "peak": round(atomic_rate["rate"] / 1e9, 3),
                              "unit": "Gatomics/s", "frac": round(a / atomic_rate["rate"], 4),
                              "atomics": int(atoms[dom]), "peak_from": atomic_rate["what"]}
        rec["closest_roof"] = "atomics" if rec["atomic_roof"]["frac"] > rec["frac"] else "hbm"
    return rec


def atomic_rate(nbytes, wide):
    """Measured rate of global atomic adds in runs of 64 consecutive words per wavefront over
    an array of nbytes (the pattern of the wedge pass's credits to one vertex's out-edges)."""
    import paper_1608_05138_amd as glt
    kind = "atomic_runs64" if wide else "atomic_runs"
    ms, ops = glt.probe(kind, max(int(nbytes), 1 << 20), reps=5)
    return {"rate": ops / (ms * 1e-3),
            "what": f"glt_probe {kind}: {ops} atomic adds of {'64' if wide else '32'}-bit words in runs of 64 per "
                    f"wavefront over {max(int(nbytes), 1 << 20)} bytes, {ms:.3f} ms per launch"}


AUTO_LARGE_EDGES = 1 << 25   # the library's automatic schedule: see glt_schedule in include/glt.h


def resolved_schedule(sched, m, batch=False):
    """The stream mode and list order a call runs with: the schedule's, or (-1) the library's
    automatic choice (mode 2; largest degree first for a single graph of >= 2^25 edges, else
    the bucketing order)."""
    large = not batch and m >= AUTO_LARGE_EDGES
    mode = sched["wedge_stream"] if sched["wedge_stream"] >= 0 else 2
    order = sched["list_order"] if sched["list_order"] >= 0 else (1 if large else 2)
    return {"wedge_stream": mode, "list_order": order}


def parse_schedule(spec):
    """'k=v,k=v' -> {k: int(v)} (schedule fields by their glt_schedule names)."""
    out = {}
    for item in (spec or "").split(","):
        if item.strip():
            k, v = item.split("=")
            out[k.strip()] = int(v)
    return out


def mean_timing(samples):
    keys = samples[0].keys()
    return {k: sum(t[k] for t in samples) / len(samples) for k in keys}


def acc_width(max_degree):
    """Width of the per-edge credits: 32-bit for every narrow edge (all edges when the maximum
    degree is at most 46,340, all but a small suffix of the degree order otherwise)."""
    return 4


def host_cpu():
    """CPU model name and the counts of logical CPUs on the host and available to us."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline(n, rp, col, budget_s=15.0):
    """The oracle (paper's method), per-edge counts of a uniform random edge sample, on the
    host threads available to this process (at most 16: the host's share per GPU here)."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    cpu = host_cpu()
    threads = max(1, min(16, cpu["affinity"]))
    m = col.size // 2
    rng = np.random.default_rng(2024)
    k = 256
    spent, done = 0.0, 0
    while spent < budget_s and done < m:
        eids = rng.integers(0, m, size=k).astype(np.int64)
        t0 = time.perf_counter()
        oracle.count_edges(n, rp, col, eids, nthreads=threads)
        dt = time.perf_counter() - t0
        spent += dt
        done += k
        if dt < budget_s / 8:
            k *= 2
    return {"value": done / spent, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} uniformly drawn edges of the same graph, per-edge counts by the "
                      f"paper's edge-centric method (vertex terms for their endpoints included), "
                      f"{spent:.1f} s on {threads} threads",
            "host": cpu}


def time_graph(ctx, rpt, ct, n, per_edge, out, stream, steps, warmup):
    """Warm-up calls, then `steps` timed glt_count calls (host clock around them, the
    library's HIP-event kernel-group times per call)."""
    import torch
    X = None
    for _ in range(warmup):
        X, _ = ctx.count(rpt, ct, n=n, per_edge=per_edge, out=out, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    timings = []
    t0 = time.perf_counter()
    for _ in range(steps):
        X, _ = ctx.count(rpt, ct, n=n, per_edge=per_edge, out=out, stream=stream.cuda_stream)
        timings.append(ctx.last_timing())
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
    return ms, mean_timing(timings), X


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat_s22", choices=sorted(WORKLOADS) + ["batch_10k", "served"])
    ap.add_argument("--batch-graphs", type=int, default=10_000)
    ap.add_argument("--no-per-graph", action="store_true", help="batch/served: skip the per-graph comparison")
    ap.add_argument("--no-autotune", action="store_true", help="batch: keep the default schedule")
    ap.add_argument("--tune-graphs", type=int, default=1000, help="batch: graphs in the autotuning draw")
    ap.add_argument("--rate", type=float, default=2000.0, help="served: arrivals per second")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="served: length of the arrival stream")
    ap.add_argument("--pool-small", type=int, default=10000, help="served: pool of small request graphs")
    ap.add_argument("--pool-large", type=int, default=64, help="served: pool of large request graphs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side-workload", action="store_true",
                    help="single graph: skip the second workload timed beside the line (the Chung-Lu "
                         "graph beside R-MAT)")
    ap.add_argument("--no-probe", action="store_true", help="skip the atomic-rate calibration of the roofline")
    ap.add_argument("--no-side-serving", action="store_true",
                    help="R-MAT line: skip the short batch and served runs reported beside it")
    ap.add_argument("--gen-procs", type=int, default=None,
                    help="host processes generating the batch / served graphs (default: up to 16; 1: threads "
                         "of this process instead, for runs under a profiler)")
    ap.add_argument("--compare-modes", action="store_true",
                    help="single graph: also time the other stream modes (reported beside the line)")
    ap.add_argument("--schedule", default=None, metavar="K=V,...",
                    help="set schedule fields (glt_schedule names, e.g. wedge_stream=1,list_order=1) before timing; "
                         "for the batch it replaces the autotuner")
    ap.add_argument("--stream-mode", type=int, default=None, choices=[0, 1, 2],
                    help="single graph: the schedule's stream mode (default: the library's, 2 = workgroup "
                         "triangle/gather paths beside the wavefront paths, 4-cycle pass alone)")
    ap.add_argument("--global-only", action="store_true", help="skip per-edge output")
    ap.add_argument("--order-study", action="store_true",
                    help="also time each order of the workgroup work lists (reported as order_study)")
    ap.add_argument("--host-path", action="store_true",
                    help="also run the 4-cycle pass on the host's threads (glt_host_wedges) after the timed "
                         "steps and report its rate beside the device's (the hybrid scheme's CPU share)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES, 3 times (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters against a known traffic)")
    ap.add_argument("--read-probe", type=int, default=0, metavar="BYTES",
                    help="only run the library's read-only probe over BYTES (1 untimed + 3 timed launches): "
                         "a second calibration point of FETCH_SIZE")
    args = ap.parse_args()
    if args.gen_procs is not None:
        GEN_PROCS[0] = max(1, args.gen_procs)
    if args.read_probe:
        import paper_1608_05138_amd as glt
        ms, nbytes = glt.probe("read", args.read_probe, reps=3)
        print(json.dumps({"read_probe_bytes": nbytes, "launches": 4, "ms_per_launch": ms}))
        return
    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe // 4, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is not implemented", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch_10k":
        bench_batch(args)
        return
    if args.workload == "served":
        bench_served(args)
        return

    # the batch and served workloads timed beside the R-MAT line: their graphs are generated
    # first, by forked host processes, before this process touches the device
    side_runs = args.workload == "rmat_s22" and not args.no_side_workload and not args.no_side_serving
    if side_runs:
        side_batch_graphs = gen_batch(args.batch_graphs)[1]
        side_pools = gen_served_pools(SIDE_SERVED["pool_small"], SIDE_SERVED["pool_large"])

    import numpy as np
    import torch

    import graphgen as gg
    import paper_1608_05138_amd as glt

    desc, fn = WORKLOADS[args.workload]
    print(f"[bench] generating {desc}", file=sys.stderr, flush=True)
    n, (rp, col) = getattr(gg, fn)()
    m = col.size // 2
    dev = torch.device("cuda:0")
    rpt = torch.from_numpy(rp).to(dev)
    ct = torch.from_numpy(col).to(dev)
    per_edge = not args.global_only
    out = torch.empty((13, m), dtype=torch.int64, device=dev) if per_edge else None
    ctx = glt.Context(0)
    if args.schedule:
        ctx.set_schedule(**parse_schedule(args.schedule))
    if args.stream_mode is not None:
        ctx.set_schedule(wedge_stream=args.stream_mode)
    mode = ctx.schedule()["wedge_stream"]
    stream = torch.cuda.current_stream(dev)
    print(f"[bench] n={n} m={m}; warmup {args.warmup}, {args.steps} timed steps", file=sys.stderr, flush=True)
    ms_per_step, timing, X = time_graph(ctx, rpt, ct, n, per_edge, out, stream, args.steps, args.warmup)
    work = ctx.last_work()
    print(f"[bench] {ms_per_step:.3f} ms/step; kernel groups " +
          ", ".join(f"{k}={v:.3f}" for k, v in timing.items()), file=sys.stderr, flush=True)

    host_path = None
    if args.host_path and per_edge:
        # Section 4.3's hybrid scheme on this machine: the host's threads run the 4-cycle pass of
        # the same graph; a CPU share of the wedges could save at most that share of the device's
        # wedge pass, and needs the relabelled graph on the host every step (the copy below)
        print("[bench] host path: the 4-cycle pass on host threads", file=sys.stderr, flush=True)
        hr = ctx.host_wedges(0)
        dev_ms = sum(timing[k] for k in ("wedge_wave", "wedge_mid", "wedge_wg", "wedge_huge"))
        host_rate = hr["wedges"] / (hr["count_ms"] * 1e-3)
        dev_rate = hr["wedges"] / (dev_ms * 1e-3)
        share = host_rate / (host_rate + dev_rate)
        host_path = {"threads": hr["threads"], "host": host_cpu(), "wedges": hr["wedges"],
                     "host_ms": round(hr["count_ms"], 1), "host_wedges_per_s": host_rate,
                     "device_wedge_pass_ms": round(dev_ms, 3), "device_wedges_per_s": dev_rate,
                     "best_host_share": share, "best_saving_ms": round(share * dev_ms, 3),
                     "copy_bytes": hr["bytes_copied"], "copy_ms": round(hr["copy_ms"], 3),
                     "cycles4_agree": hr["cycles4"] == hr["gpu_cycles4"] and hr["credit_sum"] == 4 * hr["cycles4"]}
        print(f"[bench] host path: {host_path}", file=sys.stderr, flush=True)
        assert host_path["cycles4_agree"], "host and device 4-cycle totals differ"

    maxdeg = int(np.diff(rp.astype(np.int64)).max()) if n else 0
    acc = acc_width(maxdeg)
    arate = None
    if not args.no_probe and per_edge:
        arate = atomic_rate(acc * m, acc == 8)
        print(f"[bench] atomic calibration: {arate['what']}", file=sys.stderr, flush=True)
    roof = roofline(timing, work, per_edge, acc, args.workload, bool(ctx.schedule()["tri_records"]),
                    prep=prep_bytes(n, m, rp.dtype.itemsize), atomic_rate=arate)
    study = None
    if args.order_study:
        # the ordering study (Section 4.3, Table 4) on the same graph: step time per order of the
        # workgroup work lists, each after one warm-up step
        names = ["largest work first", "largest degree first", "ascending rank", "pseudo-random",
                 "largest volume first", "smallest degree first", "smallest volume first"]
        study = {}
        default_order = ctx.schedule()["list_order"]
        for order, name in enumerate(names):
            ctx.set_schedule(list_order=order, record_balance=0)
            oms, otiming, Xo = time_graph(ctx, rpt, ct, n, per_edge, out, stream, args.steps, 1)
            assert Xo == X, "list order changed the counts"
            # one more step with the workgroup wedge class's entries timed (load balance)
            ctx.set_schedule(record_balance=1)
            time_graph(ctx, rpt, ct, n, per_edge, out, stream, 1, 0)
            w = ctx.last_work()
            study[name] = {"ms_per_step": round(oms, 3), "wedge_wg_ms": round(otiming["wedge_wg"], 3),
                           "wedge_wg_tail_ms": round(w.get("wg_tail_ns", 0) / 1e6, 3),
                           "wedge_wg_span_ms": round(w.get("wg_span_ns", 0) / 1e6, 3)}
        ctx.set_schedule(list_order=default_order, record_balance=0)
        print(f"[bench] ordering study (ms/step): {study}", file=sys.stderr, flush=True)
    other = {}
    if args.compare_modes and args.steps > 0:
        # the same step under the other stream modes, reported beside the line
        for om in (0, 1, 2):
            if om == mode:
                continue
            ctx.set_schedule(wedge_stream=om)
            oms, _, X2 = time_graph(ctx, rpt, ct, n, per_edge, out, stream, args.steps, 1)
            other[str(om)] = round(oms, 3)
            assert X2 == X, "the stream mode changed the counts"
        ctx.set_schedule(wedge_stream=mode)
        print(f"[bench] other stream modes (ms/step): {other}", file=sys.stderr, flush=True)
    side = None
    if args.workload == "rmat_s22" and not args.no_side_workload:
        # the Chung-Lu graph, timed in the same run and reported beside the line
        del out
        torch.cuda.empty_cache()
        sdesc, sfn = WORKLOADS["chung_lu_1m"]
        print(f"[bench] side workload: generating {sdesc}", file=sys.stderr, flush=True)
        sn, (srp, scol) = getattr(gg, sfn)()
        sm = scol.size // 2
        srpt = torch.from_numpy(srp).to(dev)
        sct = torch.from_numpy(scol).to(dev)
        sout = torch.empty((13, sm), dtype=torch.int64, device=dev) if per_edge else None
        sms, stiming, _ = time_graph(ctx, srpt, sct, sn, per_edge, sout, stream, 20, 5)
        swork = ctx.last_work()
        sacc = acc_width(int(np.diff(srp.astype(np.int64)).max()))
        sarate = atomic_rate(sacc * sm, sacc == 8) if (not args.no_probe and per_edge) else None
        side = {"workload": "chung_lu_1m", "graph": sdesc, "n": sn, "m": sm, "steps": 20, "warmup": 5,
                "ms_per_step": round(sms, 4), "edges_per_s": sm / (sms * 1e-3),
                "kernel_groups_ms": {k: round(float(v), 4) for k, v in stiming.items()},
                "roofline": roofline(stiming, swork, per_edge, sacc, "chung_lu_1m",
                                     bool(ctx.schedule()["tri_records"]), prep=prep_bytes(sn, sm, srp.dtype.itemsize),
                                     atomic_rate=sarate)}
        print(f"[bench] side workload: {sms:.3f} ms/step", file=sys.stderr, flush=True)
        del sout, srpt, sct
    line = {
        "metric": "edges/sec for exact 4-node motif counts (1 GPU)",
        "value": m / (ms_per_step * 1e-3),
        "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": args.workload, "graph": desc, "n": n, "m": m,
                   "outputs": "global X1..X17 (u128) + 13 per-edge counts (u64)" if per_edge
                   else "global X1..X17 (u128)"},
        "schedule": ctx.schedule(),
        "schedule_resolved": resolved_schedule(ctx.schedule(), m),
        "kernel_groups_ms": {k: round(float(v), 4) for k, v in timing.items()},
        "work": work,
        "roofline": roof,
        **({"side_workload": side} if side else {}),
        **({"order_study_ms_per_step": study} if study else {}),
        **({"other_stream_modes_ms_per_step": other} if other else {}),
        **({"host_path": host_path} if host_path else {}),
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(n, rp, col)
    ctx.close()
    if side_runs:
        print("[bench] side runs: the batch and served workloads (short)", file=sys.stderr, flush=True)
        line["side_batch"] = side_batch_run(args, side_batch_graphs)
        del side_batch_graphs
        line["side_served"] = side_served_run(args, side_pools)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
