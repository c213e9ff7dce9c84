"""Exact 2-, 3- and 4-node graphlet counts on an AMD MI355X (libglt, HIP for gfx950).

Thin ctypes binding over the C ABI declared in ``include/glt.h``: every count is computed by
the library's kernels; this module only marshals pointers and sizes.  PyTorch provides
device memory and streams.  There is no CPU fallback: if ``libglt.so`` is missing the
import of the binding raises.

Example::

    import torch, paper_1608_05138_amd as glt
    ctx = glt.Context()
    X, per_edge = ctx.count(row_ptr_cuda, col_cuda, per_edge=True)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libglt.so")

GRAPHLETS = ["edge", "2-node-indep", "triangle", "2-star", "3-node-1-edge", "3-node-indep",
             "4-clique", "chordal-cycle", "tailed-triangle", "4-cycle", "3-star", "4-path",
             "4-node-1-triangle", "4-node-2-edge", "4-node-2-star", "4-node-1-edge",
             "4-node-indep"]
# graphlet ids (1-based, Table 1) of the 13 per-edge slots
EDGE_SLOTS = [3, 4, 5, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16]

GLT_GLOBAL = 1
GLT_PER_EDGE = 2

STATUS = {0: "GLT_OK", -1: "GLT_E_INVALID_ARG", -2: "GLT_E_NOT_SIMPLE", -3: "GLT_E_NOT_SYMMETRIC",
          -4: "GLT_E_OOM", -5: "GLT_E_DEVICE", -6: "GLT_E_UNSUPPORTED", -7: "GLT_E_INTERNAL",
          -8: "GLT_E_BUSY"}

# the C-ABI symbols declared in include/glt.h
EXPORTS = ["glt_create", "glt_destroy", "glt_last_error", "glt_version", "glt_count",
           "glt_last_timing", "glt_last_work", "glt_count_batch", "glt_server_create",
           "glt_server_submit", "glt_server_poll", "glt_server_inflight", "glt_server_clock",
           "glt_server_destroy", "glt_get_schedule", "glt_set_schedule", "glt_autotune_batch",
           "glt_probe", "glt_count_noalloc", "glt_host_wedges"]


class GltError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class glt_host_wedge_report(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("wedges", ctypes.c_uint64), ("cycles4", ctypes.c_uint64),
                ("gpu_cycles4", ctypes.c_uint64), ("credit_sum", ctypes.c_uint64),
                ("bytes_copied", ctypes.c_uint64), ("copy_ms", ctypes.c_double), ("count_ms", ctypes.c_double)]


class glt_u128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]


class glt_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("offsets_are_64bit", ctypes.c_int32),
                ("on_device", ctypes.c_int32)]


class glt_batch(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int64), ("vtx_base", ctypes.c_void_p),
                ("slot_base", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("on_device", ctypes.c_int32)]


class glt_schedule(ctypes.Structure):
    _fields_ = [("wedge_wave_max", ctypes.c_int32), ("wedge_mid_max", ctypes.c_int32),
                ("wedge_dense", ctypes.c_int32), ("wedge_range_limit", ctypes.c_int32),
                ("tri_records", ctypes.c_int32), ("wedge_wg_max", ctypes.c_int32),
                ("wedge_stream", ctypes.c_int32), ("list_order", ctypes.c_int32),
                ("record_balance", ctypes.c_int32)]


SCHEDULE_KEYS = ["wedge_wave_max", "wedge_mid_max", "wedge_dense", "wedge_range_limit", "tri_records",
                 "wedge_wg_max", "wedge_stream", "list_order", "record_balance"]


class glt_server_opts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_batch_graphs", ctypes.c_int32),
                ("max_batch_edges", ctypes.c_int64), ("resident_bytes", ctypes.c_size_t),
                ("workspace_bytes", ctypes.c_size_t), ("max_pending", ctypes.c_int32),
                ("large_edges", ctypes.c_int32)]


class glt_result(ctypes.Structure):
    _fields_ = [("req_id", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("batch_graphs", ctypes.c_int32), ("X", glt_u128 * 17),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libglt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libglt.so not found at {path}; build it with "
                           "`python paper_1608_05138_amd/build.py` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.glt_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(P)]
    lib.glt_create.restype = ctypes.c_int
    lib.glt_destroy.argtypes = [P]
    lib.glt_destroy.restype = None
    lib.glt_last_error.argtypes = [P]
    lib.glt_last_error.restype = ctypes.c_char_p
    lib.glt_version.argtypes = []
    lib.glt_version.restype = ctypes.c_char_p
    lib.glt_count.argtypes = [P, ctypes.POINTER(glt_csr), ctypes.c_uint32,
                              ctypes.POINTER(glt_u128), P, P]
    lib.glt_count.restype = ctypes.c_int
    lib.glt_last_timing.argtypes = [P, ctypes.POINTER(ctypes.c_float), ctypes.c_int]
    lib.glt_last_timing.restype = ctypes.c_int
    lib.glt_last_work.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
    lib.glt_last_work.restype = ctypes.c_int
    lib.glt_count_batch.argtypes = [P, ctypes.POINTER(glt_batch), ctypes.c_uint32,
                                    ctypes.POINTER(glt_u128), P]
    lib.glt_count_batch.restype = ctypes.c_int
    lib.glt_server_create.argtypes = [ctypes.POINTER(glt_server_opts), ctypes.POINTER(P)]
    lib.glt_server_create.restype = ctypes.c_int
    lib.glt_server_submit.argtypes = [P, ctypes.POINTER(glt_csr), ctypes.c_uint64]
    lib.glt_server_submit.restype = ctypes.c_int
    lib.glt_server_poll.argtypes = [P, ctypes.POINTER(glt_result), ctypes.c_int, ctypes.c_int]
    lib.glt_server_poll.restype = ctypes.c_int
    lib.glt_server_inflight.argtypes = [P]
    lib.glt_server_inflight.restype = ctypes.c_int64
    lib.glt_server_clock.argtypes = []
    lib.glt_server_clock.restype = ctypes.c_double
    lib.glt_server_destroy.argtypes = [P]
    lib.glt_server_destroy.restype = None
    lib.glt_get_schedule.argtypes = [P, ctypes.POINTER(glt_schedule)]
    lib.glt_get_schedule.restype = ctypes.c_int
    lib.glt_set_schedule.argtypes = [P, ctypes.POINTER(glt_schedule)]
    lib.glt_set_schedule.restype = ctypes.c_int
    lib.glt_autotune_batch.argtypes = [P, ctypes.POINTER(glt_batch), ctypes.POINTER(glt_schedule),
                                       ctypes.POINTER(ctypes.c_float), P]
    lib.glt_autotune_batch.restype = ctypes.c_int
    lib.glt_probe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_size_t, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_uint64)]
    lib.glt_probe.restype = ctypes.c_int
    lib.glt_count_noalloc.argtypes = [P, ctypes.POINTER(glt_csr), ctypes.c_uint32,
                                      ctypes.POINTER(glt_u128), P, P]
    lib.glt_count_noalloc.restype = ctypes.c_int
    lib.glt_host_wedges.argtypes = [P, ctypes.c_int, ctypes.POINTER(glt_host_wedge_report)]
    lib.glt_host_wedges.restype = ctypes.c_int
    _lib = lib
    return lib


def batch_counts(raw):
    """[B, 17, 2] uint64 (low, high) halves -> B lists of 17 Python ints."""
    lo = raw[..., 0].reshape(-1).tolist()
    hi = raw[..., 1].reshape(-1).tolist()
    flat = [l | (h << 64) if h else l for l, h in zip(lo, hi)]
    return [flat[17 * g: 17 * g + 17] for g in range(len(flat) // 17)]


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class Context:
    """A libglt handle bound to one HIP device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        rc = self._lib.glt_create(device, hbm_budget_bytes, ctypes.byref(h))
        if rc != 0:
            raise GltError(rc, "glt_create failed")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            self._lib.glt_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return self._lib.glt_last_error(self._h).decode()

    TIMING_KEYS = ["prep", "tri_wave", "tri_wg", "gather_wave", "gather_wg", "wedge_wave", "wedge_mid",
                   "wedge_wg", "wedge_huge", "combine", "total"]
    WORK_KEYS = ["n", "m", "wedges_wave", "wedges_wg", "tri_list_wave", "tri_list_wg", "triangles_wave",
                 "triangles_wg", "wedges_mid", "wedges_huge", "wg_tail_ns", "wg_span_ns",
                 "max_wedges_wave", "max_wedges_mid", "max_wedges_wg", "max_wedges_huge"]

    def last_timing(self):
        """dict of kernel-group times (ms) of the last count (HIP events on the stream each
        group runs on; with wedge_stream = 1 the wedge groups share the chip with the triangle
        and gather groups, with wedge_stream = 2 the workgroup groups share it with the
        wavefront groups and the mid wedge class with the wave class; "total" is the whole
        call)."""
        buf = (ctypes.c_float * len(self.TIMING_KEYS))()
        k = self._lib.glt_last_timing(self._h, buf, len(self.TIMING_KEYS))
        return {name: float(buf[i]) for i, name in enumerate(self.TIMING_KEYS[:k])}

    def last_work(self):
        """dict of work counters of the last count."""
        buf = (ctypes.c_uint64 * len(self.WORK_KEYS))()
        k = self._lib.glt_last_work(self._h, buf, len(self.WORK_KEYS))
        return {name: int(buf[i]) for i, name in enumerate(self.WORK_KEYS[:k])}

    def host_wedges(self, threads: int = 0):
        """glt_host_wedges: the wedge pass of the last single-graph count again on `threads`
        host threads (0: every thread this process may use); a dict of the report's fields."""
        r = glt_host_wedge_report()
        rc = self._lib.glt_host_wedges(self._h, threads, ctypes.byref(r))
        if rc != 0:
            raise GltError(rc, self.last_error() or "glt_host_wedges failed")
        return {name: getattr(r, name) for name, _ in glt_host_wedge_report._fields_}

    def count_noalloc(self, row_ptr, col, n: int | None = None, per_edge: bool = False, out=None,
                      stream=None):
        """glt_count_noalloc: as count() with device tensors only; the library allocates no
        device memory during the call (its fixed per-device scratch array serves as the
        workspace; overlapping calls on one device race)."""
        if not (_is_torch(row_ptr) and row_ptr.is_cuda):
            raise ValueError("count_noalloc takes device tensors only")
        return self.count(row_ptr, col, n=n, per_edge=per_edge, out=out, stream=stream, _noalloc=True)

    def count(self, row_ptr, col, n: int | None = None, per_edge: bool = False, out=None,
              stream=None, _noalloc: bool = False):
        """Count graphlets of the CSR graph (row_ptr, col).

        Device inputs: torch CUDA tensors (int32/int64 row_ptr, int32 col); per-edge output
        is a torch int64 tensor [13, m] on the same device (values are exact uint64 counts,
        all below 2^63).  Host inputs: numpy arrays; per-edge output is a numpy uint64 array.
        Returns (X, per_edge_or_None) with X a list of 17 Python ints (X1..X17).
        """
        dev = _is_torch(row_ptr) and row_ptr.is_cuda
        if dev:
            import torch
            if not (_is_torch(col) and col.is_cuda):
                raise ValueError("row_ptr and col must both be device tensors")
            if row_ptr.dtype not in (torch.int32, torch.int64) or col.dtype != torch.int32:
                raise ValueError("row_ptr int32/int64, col int32 expected")
            row_ptr = row_ptr.contiguous()
            col = col.contiguous()
            nn = row_ptr.numel() - 1 if n is None else n
            m = col.numel() // 2
            rp_ptr, col_ptr = row_ptr.data_ptr(), col.data_ptr()
            rp64 = row_ptr.dtype == torch.int64
            if per_edge:
                if out is None:
                    out = torch.empty((13, m), dtype=torch.int64, device=row_ptr.device)
                out_ptr = out.data_ptr()
            else:
                out_ptr = None
            if stream is None:
                stream = torch.cuda.current_stream(row_ptr.device).cuda_stream
        else:
            row_ptr = np.ascontiguousarray(row_ptr)
            col = np.ascontiguousarray(col, dtype=np.int32)
            if row_ptr.dtype not in (np.int32, np.int64):
                row_ptr = row_ptr.astype(np.int64)
            nn = row_ptr.size - 1 if n is None else n
            m = col.size // 2
            rp_ptr, col_ptr = row_ptr.ctypes.data, col.ctypes.data
            rp64 = row_ptr.dtype == np.int64
            if per_edge:
                if out is None:
                    out = np.zeros((13, m), dtype=np.uint64)
                out_ptr = out.ctypes.data
            else:
                out_ptr = None
        g = glt_csr(nn, m, rp_ptr, col_ptr, 1 if rp64 else 0, 1 if dev else 0)
        X = (glt_u128 * 17)()
        flags = GLT_GLOBAL | (GLT_PER_EDGE if per_edge else 0)
        fn = self._lib.glt_count_noalloc if _noalloc else self._lib.glt_count
        rc = fn(self._h, ctypes.byref(g), flags, X, ctypes.c_void_p(out_ptr) if out_ptr else None,
                ctypes.c_void_p(stream) if stream else None)
        if rc != 0:
            raise GltError(rc, self.last_error())
        return [int(x.lo) | (int(x.hi) << 64) for x in X], (out if per_edge else None)


    def schedule(self) -> dict:
        """The handle's work schedule (glt_get_schedule) as a dict."""
        sc = glt_schedule()
        rc = self._lib.glt_get_schedule(self._h, ctypes.byref(sc))
        if rc != 0:
            raise GltError(rc, self.last_error())
        return {k: int(getattr(sc, k)) for k in SCHEDULE_KEYS}

    def set_schedule(self, **fields):
        """Change fields of the work schedule (glt_set_schedule)."""
        cur = self.schedule()
        unknown = set(fields) - set(SCHEDULE_KEYS)
        if unknown:
            raise ValueError(f"unknown schedule fields {sorted(unknown)}")
        cur.update(fields)
        sc = glt_schedule(*[int(cur[k]) for k in SCHEDULE_KEYS])
        rc = self._lib.glt_set_schedule(self._h, ctypes.byref(sc))
        if rc != 0:
            raise GltError(rc, self.last_error())

    def autotune_batch(self, packed, stream=None):
        """Run the batch autotuner (glt_autotune_batch); returns (schedule dict, device ms)."""
        b, _keep, stream = self._batch_struct(packed, stream)
        sc = glt_schedule()
        ms = ctypes.c_float(0)
        rc = self._lib.glt_autotune_batch(self._h, ctypes.byref(b), ctypes.byref(sc), ctypes.byref(ms),
                                          ctypes.c_void_p(stream) if stream else None)
        if rc != 0:
            raise GltError(rc, self.last_error())
        return {k: int(getattr(sc, k)) for k in SCHEDULE_KEYS}, float(ms.value)

    def _batch_struct(self, packed, stream):
        vb = np.ascontiguousarray(packed["vtx_base"], dtype=np.int64)
        sb = np.ascontiguousarray(packed["slot_base"], dtype=np.int64)
        rp, col = packed["row_ptr"], packed["col"]
        B = vb.size - 1
        dev = _is_torch(rp) and rp.is_cuda
        if dev:
            import torch
            rp = rp.contiguous()
            col = col.contiguous()
            if rp.dtype != torch.int32 or col.dtype != torch.int32:
                raise ValueError("int32 row_ptr and col expected")
            rp_ptr, col_ptr = rp.data_ptr(), col.data_ptr()
            if stream is None:
                stream = torch.cuda.current_stream(rp.device).cuda_stream
        else:
            rp = np.ascontiguousarray(rp, dtype=np.int32)
            col = np.ascontiguousarray(col, dtype=np.int32)
            rp_ptr, col_ptr = rp.ctypes.data, col.ctypes.data
        b = glt_batch(B, vb.ctypes.data, sb.ctypes.data, rp_ptr, col_ptr, 1 if dev else 0)
        return b, (vb, sb, rp, col), stream

    def count_batch(self, packed, stream=None, raw: bool = False):
        """Global counts of every graph of a packed batch.

        packed: dict with vtx_base, slot_base (int64 numpy, B+1), row_ptr (int32), col
        (int32); row_ptr/col may be torch CUDA tensors (device) or numpy arrays (host).
        Returns a list of B lists of 17 Python ints, or with raw=True the library's output
        as it is: a numpy uint64 array [B, 17, 2] of (low, high) 64-bit halves (batch_counts()
        turns it into the lists).
        """
        b, _keep, stream = self._batch_struct(packed, stream)
        B = int(b.num_graphs)
        X = np.zeros((max(B, 1), 17, 2), dtype=np.uint64)
        rc = self._lib.glt_count_batch(self._h, ctypes.byref(b), GLT_GLOBAL,
                                       X.ctypes.data_as(ctypes.POINTER(glt_u128)),
                                       ctypes.c_void_p(stream) if stream else None)
        if rc != 0:
            raise GltError(rc, self.last_error())
        return X[:B] if raw else batch_counts(X[:B])


class Server:
    """Continuous-batching request server (glt_server_*)."""

    def __init__(self, device=0, max_batch_graphs=0, max_batch_edges=0, resident_bytes=0,
                 workspace_bytes=0, max_pending=0, large_edges=0):
        self._lib = load_library()
        o = glt_server_opts(device, max_batch_graphs, max_batch_edges, resident_bytes,
                            workspace_bytes, max_pending, large_edges)
        h = ctypes.c_void_p()
        rc = self._lib.glt_server_create(ctypes.byref(o), ctypes.byref(h))
        if rc != 0:
            raise GltError(rc, "glt_server_create failed")
        self._h = h
        self._res = (glt_result * 256)()

    def clock(self) -> float:
        return self._lib.glt_server_clock()

    def submit(self, row_ptr, col, req_id, n=None):
        """Queue a host CSR graph (numpy int32/int64 row_ptr, int32 col).  Returns the
        status (0 = queued)."""
        if not (isinstance(row_ptr, np.ndarray) and row_ptr.dtype in (np.int32, np.int64)
                and row_ptr.flags.c_contiguous):
            row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        if not (isinstance(col, np.ndarray) and col.dtype == np.int32 and col.flags.c_contiguous):
            col = np.ascontiguousarray(col, dtype=np.int32)
        nn = row_ptr.size - 1 if n is None else n
        g = glt_csr(nn, col.size // 2, row_ptr.ctypes.data, col.ctypes.data,
                    1 if row_ptr.dtype == np.int64 else 0, 0)
        return self._lib.glt_server_submit(self._h, ctypes.byref(g), req_id)

    def poll(self, max_results=256, timeout_us=1000):
        """Completed results: list of dicts (req_id, status, X, t_submit, t_admit, t_start,
        t_done, batch_graphs)."""
        k = self._lib.glt_server_poll(self._h, self._res, min(max_results, 256), timeout_us)
        out = []
        for i in range(k):
            r = self._res[i]
            out.append({"req_id": r.req_id, "status": r.status, "batch_graphs": r.batch_graphs,
                        "X": [int(x.lo) | (int(x.hi) << 64) for x in r.X],
                        "t_submit": r.t_submit, "t_admit": r.t_admit, "t_start": r.t_start,
                        "t_done": r.t_done})
        return out

    def inflight(self) -> int:
        return self._lib.glt_server_inflight(self._h)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.glt_server_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


_default = {}


def count(row_ptr, col, n=None, per_edge=False, device=0):
    """Convenience wrapper with a cached per-device Context."""
    ctx = _default.get(device)
    if ctx is None:
        ctx = _default[device] = Context(device)
    return ctx.count(row_ptr, col, n=n, per_edge=per_edge)


PROBE_KINDS = {"atomic_runs": 0, "atomic_scatter": 1, "read": 2, "atomic_runs64": 3, "atomic_scatter64": 4}


def probe(kind: str, nbytes: int, reps: int = 5, device: int = 0):
    """Roofline calibration (glt_probe): (ms per launch, atomics or bytes per launch)."""
    ms = ctypes.c_float(0)
    ops = ctypes.c_uint64(0)
    rc = load_library().glt_probe(device, PROBE_KINDS[kind], nbytes, reps, ctypes.byref(ms), ctypes.byref(ops))
    if rc != 0:
        raise GltError(rc, f"glt_probe({kind}) failed")
    return float(ms.value), int(ops.value)


def version() -> str:
    return load_library().glt_version().decode()
