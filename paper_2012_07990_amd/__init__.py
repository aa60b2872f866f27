"""MI355X (gfx950) frontier-traversal library -- Python binding.

A thin ctypes layer over the C ABI declared in ``include/gg.h`` and built into
``libgg.so`` (HIP kernels for gfx950). The binding only marshals arguments:
graph arrays come in as numpy arrays or torch tensors, outputs are torch
tensors on the current CUDA/HIP device, and every call runs on
``torch.cuda.current_stream()``. Every step of every algorithm runs in the
library's kernels; there is no CPU fallback -- importing this package raises
if the library has not been built.

Low-level functions carry the C names (``gg_bfs``, ``gg_pagerank``, ...);
``Graph`` offers the same calls as methods that allocate the outputs.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libgg.so is not built (%s); run `python -c 'import __graft_entry__ as e; e.build()'` "
        "or `python paper_2012_07990_amd/_build.py`" % LIB_PATH)

# torch first: libgg.so then binds to the HIP runtime torch already loaded
# (same SONAME), so torch's device pointers and streams are valid for it.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

# Library objects still open when the interpreter exits are closed by an
# atexit hook, which runs before torch's own exit handlers (torch was imported
# first, so its handlers were registered first and run last) and before
# module teardown: device memory, streams and worker threads are released
# while the HIP runtime is still up, servers before the graphs they serve.
import atexit  # noqa: E402
import weakref  # noqa: E402

_live_servers = weakref.WeakSet()
_live_graphs = weakref.WeakSet()


@atexit.register
def _close_all():
    for s in list(_live_servers):
        s.close()
    for g in list(_live_graphs):
        g.close()

# ---- enums (mirror include/gg.h) --------------------------------------------------
OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_UNSUPPORTED_SCHEDULE, ERR_OVERFLOW, \
    ERR_ADMISSION, ERR_NOT_FOUND, ERR_NOT_READY = range(9)
ALGO_BFS, ALGO_SSSP, ALGO_CC, ALGO_PR, ALGO_BC = range(5)
LB_VERTEX_BASED, LB_WM, LB_CM, LB_STRICT, LB_TWC, LB_ETWC, LB_EDGE_ONLY = range(7)
LB_NAMES = {"vp": 0, "vertex_based": 0, "wm": 1, "cm": 2, "strict": 3, "twc": 4, "etwc": 5,
            "edge_only": 6}
PUSH, PULL = 0, 1
REP_BOOLMAP, REP_BITMAP = 0, 1
CREATE_FUSED, CREATE_UNFUSED_BOOLMAP, CREATE_UNFUSED_BITMAP = 0, 1, 2
DEDUP_MONOTONIC_COUNTERS, DEDUP_BITMAP, DEDUP_BOOLMAP = 0, 1, 2
PRESET_DEFAULT, PRESET_BFS_HYBRID, PRESET_ROAD_FUSED, PRESET_POWERLAW = 0, 1, 2, 3
INPUT_DEVICE, VALIDATE, SYMMETRIC = 1, 2, 4
PR_NO_DANGLING = 1
PR_NO_LDS_CACHE = 2
STATS_COUNT_EDGES = 1
STATS_TIME_KERNELS = 2
TARGET_GPU, TARGET_CPU = 0, 1
INT32_MAX = 2**31 - 1


class SimpleSchedule(ctypes.Structure):
    _fields_ = [("load_balance", ctypes.c_int32), ("edge_blocking", ctypes.c_int32),
                ("blocking_size", ctypes.c_int32), ("direction", ctypes.c_int32),
                ("pull_rep", ctypes.c_int32), ("frontier_creation", ctypes.c_int32),
                ("dedup_enable", ctypes.c_int32), ("dedup_type", ctypes.c_int32),
                ("delta", ctypes.c_int32), ("kernel_fusion", ctypes.c_int32)]

    def __repr__(self):
        return "SimpleSchedule(%s)" % ", ".join("%s=%s" % (f, getattr(self, f)) for f, _ in self._fields_)


class Schedule(ctypes.Structure):
    _fields_ = [("hybrid", ctypes.c_int32), ("threshold", ctypes.c_float),
                ("s1", SimpleSchedule), ("s2", SimpleSchedule)]

    def __repr__(self):
        return "Schedule(hybrid=%d, threshold=%g, s1=%r, s2=%r)" % (self.hybrid, self.threshold, self.s1, self.s2)

    def copy(self) -> "Schedule":
        c = Schedule()
        ctypes.pointer(c)[0] = self
        return c


class Stats(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("iterations", ctypes.c_int32),
                ("push_iterations", ctypes.c_int32), ("pull_iterations", ctypes.c_int32),
                ("launches", ctypes.c_int32), ("buckets", ctypes.c_int32), ("fused", ctypes.c_int32),
                ("edges_examined", ctypes.c_int64), ("vertices_processed", ctypes.c_int64),
                ("device_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("kernel_launches", ctypes.c_int32), ("kernel_name", ctypes.c_char * 44)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["kernel_name"] = self.kernel_name.decode()
        return d


_P = ctypes.c_void_p
_i32, _i64, _u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
_SP = ctypes.POINTER(Schedule)
_STP = ctypes.POINTER(Stats)


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("gg_status_string", [ctypes.c_int], ctypes.c_char_p)
_sig("gg_last_error", [], ctypes.c_char_p)
_sig("gg_version", [], ctypes.c_char_p)
_sig("gg_graph_create_csr", [_i32, _i64, _P, _P, _P, _u32, _P, ctypes.POINTER(_P)])
_sig("gg_graph_destroy", [_P])
_sig("gg_graph_info", [_P, ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(_i32),
                       ctypes.POINTER(_i32)])
_sig("gg_graph_prepare_edgeblocking", [_P, _i32, _P, ctypes.POINTER(ctypes.c_double)])
_sig("gg_graph_prepare_pull_blocking", [_P, _i32, _P, ctypes.POINTER(ctypes.c_double)])
_sig("gg_graph_edgeblocking_export", [_P, _i32, _P, _P, _P, _P])
_sig("gg_schedule_default", [_SP])
_sig("gg_schedule_preset", [_i32, _i32, _SP])
_sig("gg_schedule_validate", [_P, _i32, _SP])
_sig("gg_bfs", [_P, _i32, _SP, _P, _P, _STP])
_sig("gg_bfs_noalloc", [_P, _i32, _SP, _P, _P])
_sig("gg_sssp", [_P, _i32, _SP, _P, _P, _STP])
_sig("gg_cc", [_P, _SP, _P, _P, _STP])
_sig("gg_pagerank", [_P, _SP, ctypes.c_float, _i32, _u32, _P, _P, _STP])
_sig("gg_bc", [_P, _i32, _SP, _P, _P, _P, _STP])
_sig("gg_bfs_multi", [_P, _P, _i32, _SP, _P, _P, _STP])
_sig("gg_sssp_multi", [_P, _P, _i32, _SP, _P, _P, _STP])
_sig("gg_bc_multi", [_P, _P, _i32, _SP, _P, _P, _P, _STP])
_sig("gg_workspace_bytes", [_P, _i32, _i32, ctypes.POINTER(ctypes.c_size_t)])
_sig("gg_tuned_set", [_P, _i32, _SP, ctypes.c_double])
_sig("gg_tuned_get", [_P, _i32, _SP, ctypes.POINTER(ctypes.c_double)])
_sig("gg_autotune", [_P, _i32, ctypes.c_double, _P, _i32, _P, _SP, ctypes.POINTER(ctypes.c_double)])


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_int64), ("status", ctypes.c_int32), ("graph_id", ctypes.c_int32),
                ("algo", ctypes.c_int32), ("src", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("queue_ms", ctypes.c_double), ("latency_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("collected", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("batches", ctypes.c_int64), ("max_batch", ctypes.c_int32),
                ("bytes_in_use", ctypes.c_size_t), ("bytes_peak", ctypes.c_size_t), ("busy_ms", ctypes.c_double),
                ("bytes_idle", ctypes.c_size_t), ("trims", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


OUT_DEVICE, OUT_HOST, OUT_DISCARD = 0, 1, 2
_RP = ctypes.POINTER(Result)
_sig("gg_server_create", [ctypes.c_size_t, _i32, ctypes.POINTER(_P)])
_sig("gg_server_add_graph", [_P, _P, ctypes.POINTER(_i32)])
_sig("gg_server_set_schedule", [_P, _i32, _i32, _SP])
_sig("gg_server_submit", [_P, _i32, _i32, _i32, ctypes.POINTER(_i64)])
_sig("gg_server_poll", [_P, _i64, _P, _u32, _RP])
_sig("gg_server_wait", [_P, _i64, ctypes.c_double, _P, _u32, _RP])
_sig("gg_server_stats", [_P, ctypes.POINTER(ServeStats)])
_sig("gg_server_destroy", [_P])
_sig("gg_cpu_graph_create", [_i32, ctypes.c_int64, _P, _P, _P, _u32, ctypes.POINTER(ctypes.c_void_p)])
_sig("gg_cpu_graph_destroy", [_P])
_sig("gg_cpu_bfs", [_P, _i32, _i32, _P])
_sig("gg_cpu_sssp", [_P, _i32, _i32, _i32, _P])
_sig("gg_cpu_cc", [_P, _i32, _P])
_sig("gg_cpu_pagerank", [_P, ctypes.c_float, _i32, _u32, _i32, _P])
_sig("gg_cpu_bc", [_P, _i32, _i32, _P, _P])
_sig("gg_place", [_P, _P, _i32, _SP, _i32, _i32, _P, ctypes.POINTER(ctypes.c_int32),
                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)])
_sig("gg_placement_get", [_P, _i32, ctypes.POINTER(ctypes.c_int32)])


class GGError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.gg_last_error().decode()
        super().__init__("%s: %s (%s)" % (where, _lib.gg_status_string(status).decode(), msg))


def _check(status: int, where: str):
    if status != OK:
        raise GGError(status, where)


def version() -> str:
    return _lib.gg_version().decode()


def status_string(s: int) -> str:
    return _lib.gg_status_string(s).decode()


# ---- schedules ----------------------------------------------------------------------
def schedule_default() -> Schedule:
    s = Schedule()
    _check(_lib.gg_schedule_default(ctypes.byref(s)), "gg_schedule_default")
    return s


def schedule_preset(algo: int, preset: int) -> Schedule:
    s = Schedule()
    _check(_lib.gg_schedule_preset(algo, preset, ctypes.byref(s)), "gg_schedule_preset")
    return s


def make_schedule(lb="vp", direction=PUSH, pull_rep=REP_BOOLMAP, creation=CREATE_FUSED, dedup=True,
                  dedup_type=DEDUP_MONOTONIC_COUNTERS, delta=1, fusion=False, edge_blocking=False,
                  blocking_size=1 << 20, hybrid=None, threshold=0.05) -> Schedule:
    """Schedule from keyword choices; `hybrid` is an optional dict of s2
    overrides (e.g. {"direction": PULL, "pull_rep": REP_BITMAP})."""
    s = schedule_default()
    s1 = s.s1
    s1.load_balance = LB_NAMES[lb] if isinstance(lb, str) else int(lb)
    s1.direction, s1.pull_rep, s1.frontier_creation = direction, pull_rep, creation
    s1.dedup_enable, s1.dedup_type, s1.delta = int(dedup), dedup_type, delta
    s1.kernel_fusion, s1.edge_blocking, s1.blocking_size = int(fusion), int(edge_blocking), blocking_size
    s.s2 = s1
    if hybrid is not None:
        s.hybrid = 1
        s.threshold = threshold
        for k, v in hybrid.items():
            if k == "lb":
                k, v = "load_balance", (LB_NAMES[v] if isinstance(v, str) else int(v))
            setattr(s.s2, k, int(v))
    return s


# ---- raw C-name wrappers (tensor arguments are passed by data_ptr) ----------------------
def _torch():
    import torch
    return torch


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(int(t.data_ptr()))


def _sched_ptr(s: Optional[Schedule]):
    return ctypes.byref(s) if s is not None else None


def _stats_ptr(st: Optional[Stats]):
    return ctypes.byref(st) if st is not None else None


def gg_bfs(graph, src, sched, depth, stream=None, stats=None):
    _check(_lib.gg_bfs(graph.handle, int(src), _sched_ptr(sched), _dptr(depth), _stream(stream),
                       _stats_ptr(stats)), "gg_bfs")


def gg_bfs_noalloc(graph, src, sched, depth, stream=None):
    _check(_lib.gg_bfs_noalloc(graph.handle, int(src), _sched_ptr(sched), _dptr(depth), _stream(stream)),
           "gg_bfs_noalloc")


def gg_sssp(graph, src, sched, dist, stream=None, stats=None):
    _check(_lib.gg_sssp(graph.handle, int(src), _sched_ptr(sched), _dptr(dist), _stream(stream),
                        _stats_ptr(stats)), "gg_sssp")


def gg_cc(graph, sched, label, stream=None, stats=None):
    _check(_lib.gg_cc(graph.handle, _sched_ptr(sched), _dptr(label), _stream(stream), _stats_ptr(stats)),
           "gg_cc")


def gg_pagerank(graph, sched, damping, iters, flags, rank, stream=None, stats=None):
    _check(_lib.gg_pagerank(graph.handle, _sched_ptr(sched), float(damping), int(iters), int(flags),
                            _dptr(rank), _stream(stream), _stats_ptr(stats)), "gg_pagerank")


def gg_bc(graph, src, sched, sigma, delta, stream=None, stats=None):
    _check(_lib.gg_bc(graph.handle, int(src), _sched_ptr(sched), _dptr(sigma), _dptr(delta), _stream(stream),
                      _stats_ptr(stats)), "gg_bc")


def gg_bfs_multi(graph, srcs, sched, depth, stream=None, stats=None):
    a = np.ascontiguousarray(np.asarray(srcs, dtype=np.int32))
    _check(_lib.gg_bfs_multi(graph.handle, ctypes.c_void_p(a.ctypes.data), int(a.size), _sched_ptr(sched),
                             _dptr(depth), _stream(stream), _stats_ptr(stats)), "gg_bfs_multi")


def gg_sssp_multi(graph, srcs, sched, dist, stream=None, stats=None):
    a = np.ascontiguousarray(np.asarray(srcs, dtype=np.int32))
    _check(_lib.gg_sssp_multi(graph.handle, ctypes.c_void_p(a.ctypes.data), int(a.size), _sched_ptr(sched),
                              _dptr(dist), _stream(stream), _stats_ptr(stats)), "gg_sssp_multi")


def gg_bc_multi(graph, srcs, sched, sigma, delta, stream=None, stats=None):
    a = np.ascontiguousarray(np.asarray(srcs, dtype=np.int32))
    _check(_lib.gg_bc_multi(graph.handle, ctypes.c_void_p(a.ctypes.data), int(a.size), _sched_ptr(sched),
                            _dptr(sigma), _dptr(delta), _stream(stream), _stats_ptr(stats)), "gg_bc_multi")


# ---- graph object ------------------------------------------------------------------------
class Graph:
    """Device-resident CSR graph (owned by the library; freed on close/del)."""

    def __init__(self, handle: ctypes.c_void_p, n: int, m: int, weighted: bool, symmetric: bool):
        self.handle = handle
        self.n, self.m, self.weighted, self.symmetric = n, m, weighted, symmetric
        _live_graphs.add(self)

    @classmethod
    def from_csr(cls, n, row_ptr, col, w=None, symmetric=True, validate=False, stream=None) -> "Graph":
        """Copy a CSR graph (numpy host arrays or torch device tensors) to the GPU."""
        flags = (SYMMETRIC if symmetric else 0) | (VALIDATE if validate else 0)
        torch = _torch()
        keep = []
        if isinstance(row_ptr, torch.Tensor) and row_ptr.is_cuda:
            flags |= INPUT_DEVICE
            rp, c = row_ptr.to(torch.int32).contiguous(), col.to(torch.int32).contiguous()
            ww = w.to(torch.int32).contiguous() if w is not None else None
            keep = [rp, c, ww]
            p_rp, p_c = _dptr(rp), _dptr(c)
            p_w = _dptr(ww) if ww is not None else None
            m = int(c.numel())
        else:
            rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int32))
            c = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
            ww = np.ascontiguousarray(np.asarray(w, dtype=np.uint32)) if w is not None else None
            keep = [rp, c, ww]
            m = int(c.size)
            p_rp = ctypes.c_void_p(rp.ctypes.data)
            p_c = ctypes.c_void_p(c.ctypes.data) if m else None
            p_w = ctypes.c_void_p(ww.ctypes.data) if (ww is not None and m) else (
                ctypes.c_void_p(np.ones(1, np.uint32).ctypes.data) if ww is not None else None)
        h = ctypes.c_void_p()
        _check(_lib.gg_graph_create_csr(int(n), m, p_rp, p_c, p_w, flags, _stream(stream), ctypes.byref(h)),
               "gg_graph_create_csr")
        del keep
        return cls(h, int(n), m, w is not None, symmetric)

    @classmethod
    def from_graphgen(cls, g, **kw) -> "Graph":
        return cls.from_csr(g.n, g.row_ptr, g.col, g.w, **kw)

    def close(self):
        if self.handle:
            _lib.gg_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- algorithms ------------------------------------------------------------------
    def _empty(self, shape, dtype):
        torch = _torch()
        return torch.empty(shape, dtype=dtype, device="cuda")

    def bfs(self, src, sched=None, stats=None, out=None):
        torch = _torch()
        out = self._empty(self.n, torch.int32) if out is None else out
        gg_bfs(self, src, sched, out, stats=stats)
        return out

    def sssp(self, src, sched=None, stats=None, out=None):
        torch = _torch()
        out = self._empty(self.n, torch.int32) if out is None else out
        gg_sssp(self, src, sched, out, stats=stats)
        return out

    def cc(self, sched=None, stats=None, out=None):
        torch = _torch()
        out = self._empty(self.n, torch.int32) if out is None else out
        gg_cc(self, sched, out, stats=stats)
        return out

    def pagerank(self, sched=None, damping=0.85, iters=20, dangling=True, stats=None, out=None,
                 lds_cache=True):
        torch = _torch()
        out = self._empty(self.n, torch.float32) if out is None else out
        flags = (0 if dangling else PR_NO_DANGLING) | (0 if lds_cache else PR_NO_LDS_CACHE)
        gg_pagerank(self, sched, damping, iters, flags, out, stats=stats)
        return out

    def bc(self, src, sched=None, stats=None):
        torch = _torch()
        sigma = self._empty(self.n, torch.int64)  # uint64 bits
        delta = self._empty(self.n, torch.float32)
        gg_bc(self, src, sched, sigma, delta, stats=stats)
        return sigma, delta

    def bfs_multi(self, srcs: Sequence[int], sched=None, stats=None):
        torch = _torch()
        out = self._empty((len(srcs), self.n), torch.int32)
        gg_bfs_multi(self, srcs, sched, out, stats=stats)
        return out

    def sssp_multi(self, srcs: Sequence[int], sched=None, stats=None):
        torch = _torch()
        out = self._empty((len(srcs), self.n), torch.int32)
        gg_sssp_multi(self, srcs, sched, out, stats=stats)
        return out

    def bc_multi(self, srcs: Sequence[int], sched=None, stats=None):
        torch = _torch()
        sigma = self._empty((len(srcs), self.n), torch.int64)
        delta = self._empty((len(srcs), self.n), torch.float32)
        gg_bc_multi(self, srcs, sched, sigma, delta, stats=stats)
        return sigma, delta

    def prepare_edgeblocking(self, seg_vertices: int, stream=None) -> float:
        ms = ctypes.c_double()
        _check(_lib.gg_graph_prepare_edgeblocking(self.handle, int(seg_vertices), _stream(stream),
                                                  ctypes.byref(ms)), "gg_graph_prepare_edgeblocking")
        return ms.value

    def prepare_pull_blocking(self, seg_vertices: int, stream=None) -> float:
        """Build (or reuse) the PULL EdgeBlocking layout; returns its build time in ms (0 if cached)."""
        ms = ctypes.c_double()
        _check(_lib.gg_graph_prepare_pull_blocking(self.handle, int(seg_vertices), _stream(stream),
                                                   ctypes.byref(ms)), "gg_graph_prepare_pull_blocking")
        return ms.value

    def edgeblocking_export(self, seg_vertices: int):
        torch = _torch()
        S = (self.n + seg_vertices - 1) // seg_vertices
        src = self._empty(max(self.m, 1), torch.int32)
        dst = self._empty(max(self.m, 1), torch.int32)
        seg = np.zeros(S + 1, dtype=np.int64)
        _check(_lib.gg_graph_edgeblocking_export(self.handle, int(seg_vertices), _dptr(src), _dptr(dst),
                                                 ctypes.c_void_p(seg.ctypes.data), _stream(None)),
               "gg_graph_edgeblocking_export")
        return src[:self.m], dst[:self.m], seg

    def autotune(self, algo: int, budget_s: float = 10.0, probes: Sequence[int] = (0,)):
        """Run the library's autotuner; returns (schedule, best_ms)."""
        a = np.ascontiguousarray(np.asarray(probes, dtype=np.int32))
        s = Schedule()
        ms = ctypes.c_double()
        _check(_lib.gg_autotune(self.handle, int(algo), float(budget_s), ctypes.c_void_p(a.ctypes.data),
                                int(a.size), _stream(None), ctypes.byref(s), ctypes.byref(ms)), "gg_autotune")
        return s, ms.value

    def validate(self, algo: int, sched: Schedule) -> None:
        _check(_lib.gg_schedule_validate(self.handle, algo, ctypes.byref(sched)), "gg_schedule_validate")

    def workspace_bytes(self, algo: int, k: int = 1) -> int:
        out = ctypes.c_size_t()
        _check(_lib.gg_workspace_bytes(self.handle, algo, k, ctypes.byref(out)), "gg_workspace_bytes")
        return out.value

    # -- the tuned-schedule cache (gg_tuned_set / gg_tuned_get) -----------------------
    def tuned(self, algo: int):
        """(schedule, ms) cached for `algo` on this graph, or None."""
        s, ms = Schedule(), ctypes.c_double()
        st = _lib.gg_tuned_get(self.handle, int(algo), ctypes.byref(s), ctypes.byref(ms))
        if st == ERR_NOT_FOUND:
            return None
        _check(st, "gg_tuned_get")
        return s, ms.value

    def set_tuned(self, algo: int, sched: Schedule, ms: float = 0.0) -> None:
        _check(_lib.gg_tuned_set(self.handle, int(algo), ctypes.byref(sched), float(ms)), "gg_tuned_set")

    def save_tuned(self, path: str, checksum: str) -> int:
        """Store every cached tuned schedule of this graph in the JSON file at
        `path` under `checksum` (see csr_checksum); returns how many."""
        k = 0
        for algo in ALGO_NAMES:
            t = self.tuned(algo)
            if t is not None:
                save_tuned(path, checksum, algo, t[0], t[1])
                k += 1
        return k

    def load_tuned(self, path: str, checksum: str) -> int:
        """Seed this graph's cache from the schedules stored under `checksum`;
        returns how many."""
        got = load_tuned(path, checksum)
        for algo, (sched, ms) in got.items():
            self.set_tuned(algo, sched, ms)
        return len(got)


# ---- tuned schedules kept across processes: JSON keyed by a graph checksum --------
ALGO_NAMES = {ALGO_BFS: "bfs", ALGO_SSSP: "sssp", ALGO_CC: "cc", ALGO_PR: "pr", ALGO_BC: "bc"}


def csr_checksum(n, row_ptr, col, w=None) -> str:
    """Digest of a host CSR graph (sizes, offsets, columns and weights): the
    key under which its tuned schedules are stored."""
    import hashlib
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int32))
    c = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
    h = hashlib.blake2b(digest_size=16)
    h.update(np.array([int(n), c.size, 0 if w is None else 1], dtype=np.int64).tobytes())
    h.update(rp.tobytes())
    h.update(c.tobytes())
    if w is not None:
        h.update(np.ascontiguousarray(np.asarray(w, dtype=np.uint32)).tobytes())
    return h.hexdigest()


def schedule_to_dict(s: Schedule) -> dict:
    simple = lambda x: {f: int(getattr(x, f)) for f, _ in SimpleSchedule._fields_}  # noqa: E731
    return {"hybrid": int(s.hybrid), "threshold": float(s.threshold), "s1": simple(s.s1), "s2": simple(s.s2)}


def schedule_from_dict(d: dict) -> Schedule:
    s = Schedule()
    s.hybrid = int(d["hybrid"])
    s.threshold = float(d["threshold"])
    for part in ("s1", "s2"):
        for f, _ in SimpleSchedule._fields_:
            setattr(getattr(s, part), f, int(d[part][f]))
    return s


def _read_store(path: str) -> dict:
    import json
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def save_tuned(path: str, checksum: str, algo: int, sched: Schedule, ms: float) -> None:
    """Record (or replace) the tuned schedule of `algo` for the graph with
    `checksum` in the JSON file at `path`, keeping its other entries."""
    import json
    data = _read_store(path)
    data.setdefault(checksum, {})[ALGO_NAMES[int(algo)]] = {"schedule": schedule_to_dict(sched), "ms": float(ms)}
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def load_tuned(path: str, checksum: str) -> dict:
    """{algo: (Schedule, ms)} stored for the graph with `checksum` ({} if none)."""
    ids = {v: k for k, v in ALGO_NAMES.items()}
    entry = _read_store(path).get(checksum, {})
    return {ids[name]: (schedule_from_dict(e["schedule"]), float(e["ms"])) for name, e in entry.items()}


class CpuGraph:
    """Host copy of a CSR graph for the CPU backend (the library's threads;
    numpy in, numpy out)."""

    def __init__(self, n, row_ptr, col, w=None, symmetric=True, validate=False):
        rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int32))
        c = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
        ww = np.ascontiguousarray(np.asarray(w, dtype=np.uint32)) if w is not None else None
        flags = (SYMMETRIC if symmetric else 0) | (VALIDATE if validate else 0)
        h = ctypes.c_void_p()
        _check(_lib.gg_cpu_graph_create(int(n), int(c.size), ctypes.c_void_p(rp.ctypes.data),
                                        ctypes.c_void_p(c.ctypes.data) if c.size else None,
                                        ctypes.c_void_p(ww.ctypes.data) if ww is not None and ww.size else None,
                                        flags, ctypes.byref(h)), "gg_cpu_graph_create")
        self.handle, self.n, self.m, self.symmetric = h, int(n), int(c.size), symmetric

    @classmethod
    def from_graphgen(cls, g, **kw) -> "CpuGraph":
        return cls(g.n, g.row_ptr, g.col, g.w, **kw)

    def bfs(self, src, nthreads=0):
        out = np.empty(self.n, dtype=np.int32)
        _check(_lib.gg_cpu_bfs(self.handle, int(src), int(nthreads), ctypes.c_void_p(out.ctypes.data)),
               "gg_cpu_bfs")
        return out

    def sssp(self, src, delta=64, nthreads=0):
        out = np.empty(self.n, dtype=np.int32)
        _check(_lib.gg_cpu_sssp(self.handle, int(src), int(delta), int(nthreads), ctypes.c_void_p(out.ctypes.data)),
               "gg_cpu_sssp")
        return out

    def cc(self, nthreads=0):
        out = np.empty(self.n, dtype=np.int32)
        _check(_lib.gg_cpu_cc(self.handle, int(nthreads), ctypes.c_void_p(out.ctypes.data)), "gg_cpu_cc")
        return out

    def pagerank(self, damping=0.85, iters=20, dangling=True, nthreads=0):
        out = np.empty(self.n, dtype=np.float32)
        _check(_lib.gg_cpu_pagerank(self.handle, float(damping), int(iters), 0 if dangling else PR_NO_DANGLING,
                                    int(nthreads), ctypes.c_void_p(out.ctypes.data)), "gg_cpu_pagerank")
        return out

    def bc(self, src, nthreads=0):
        sigma = np.empty(self.n, dtype=np.uint64)
        delta = np.empty(self.n, dtype=np.float32)
        _check(_lib.gg_cpu_bc(self.handle, int(src), int(nthreads), ctypes.c_void_p(sigma.ctypes.data),
                              ctypes.c_void_p(delta.ctypes.data)), "gg_cpu_bc")
        return sigma, delta

    def close(self):
        if self.handle:
            _lib.gg_cpu_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def place(graph, cpu_graph, algo, sched=None, src=0, nthreads=0, stream=None):
    """gg_place: time `algo` on both backends; returns (target, gpu_ms, cpu_ms)."""
    t, g_ms, c_ms = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
    _check(_lib.gg_place(graph.handle, cpu_graph.handle, int(algo), _sched_ptr(sched), int(src), int(nthreads),
                         _stream(stream), ctypes.byref(t), ctypes.byref(g_ms), ctypes.byref(c_ms)), "gg_place")
    return t.value, g_ms.value, c_ms.value


class Server:
    """Serving loop (gg_server_*): admission by device-memory footprint and
    continuous batching of queries over registered graphs."""

    def __init__(self, budget_bytes: int, nstreams: int = 4):
        h = ctypes.c_void_p()
        _check(_lib.gg_server_create(int(budget_bytes), int(nstreams), ctypes.byref(h)), "gg_server_create")
        self.handle = h
        self.graphs = []
        _live_servers.add(self)

    def add_graph(self, G: Graph) -> int:
        gid = ctypes.c_int32()
        _check(_lib.gg_server_add_graph(self.handle, G.handle, ctypes.byref(gid)), "gg_server_add_graph")
        self.graphs.append(G)
        return gid.value

    def set_schedule(self, gid: int, algo: int, sched: Schedule):
        _check(_lib.gg_server_set_schedule(self.handle, gid, algo, ctypes.byref(sched)), "gg_server_set_schedule")

    def submit(self, gid: int, algo: int, src: int) -> int:
        t = ctypes.c_int64()
        _check(_lib.gg_server_submit(self.handle, gid, algo, int(src), ctypes.byref(t)), "gg_server_submit")
        return t.value

    def _out(self, out):
        if out is None:
            return None, OUT_DISCARD
        if isinstance(out, np.ndarray):
            return ctypes.c_void_p(out.ctypes.data), OUT_HOST
        return _dptr(out), OUT_DEVICE

    def poll(self, ticket: int, out=None):
        """None while running; else the result record (copying the result into `out`)."""
        p, fl = self._out(out)
        r = Result()
        st = _lib.gg_server_poll(self.handle, int(ticket), p, fl, ctypes.byref(r))
        if st == ERR_NOT_READY:
            return None
        _check(st, "gg_server_poll")
        return r.as_dict()

    def wait(self, ticket: int, timeout: float = -1.0, out=None):
        p, fl = self._out(out)
        r = Result()
        st = _lib.gg_server_wait(self.handle, int(ticket), float(timeout), p, fl, ctypes.byref(r))
        if st == ERR_NOT_READY:
            return None
        _check(st, "gg_server_wait")
        return r.as_dict()

    def stats(self):
        s = ServeStats()
        _check(_lib.gg_server_stats(self.handle, ctypes.byref(s)), "gg_server_stats")
        return s.as_dict()

    def close(self):
        if self.handle:
            _lib.gg_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def header_functions() -> list:
    """Names of the functions include/gg.h declares (for the ABI export test)."""
    import re
    hdr = os.path.join(os.path.dirname(_HERE), "include", "gg.h")
    txt = open(hdr).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|gg_status|void)\s*\**\s*(gg_\w+)\s*\(", txt, re.M)))
