"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct implementations of what the GPU traversal
library computes (BFS depths, SSSP distances, CC labels, PageRank, Brandes
betweenness, EdgeBlocking preprocessing), in single-threaded C with fp64 for
floating point (``oracle.c``), compiled with gcc on first use.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never imports it, and this package never
imports the library: the only code the two sides share is the seeded graph
generator (``graphgen``), which holds none of the method's arithmetic.

Parity pins: every function here is checked by the CPU test suite against
brute force on tiny graphs, closed forms, library routines (scipy) and
invariants -- see tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

INT32_MAX = 2**31 - 1


class OracleOverflow(ArithmeticError):
    pass


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc -O2; plain C, no threads)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def _get():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.oracle_check_csr.restype = ctypes.c_int
        L.oracle_check_csr.argtypes = [i64, P, P]
        L.oracle_bfs.restype = ctypes.c_int
        L.oracle_bfs.argtypes = [i64, P, P, i32, P]
        L.oracle_sssp.restype = ctypes.c_int
        L.oracle_sssp.argtypes = [i64, P, P, P, i32, P]
        L.oracle_cc.restype = None
        L.oracle_cc.argtypes = [i64, P, P, P]
        L.oracle_pagerank.restype = None
        L.oracle_pagerank.argtypes = [i64, P, P, f64, ctypes.c_int, ctypes.c_int, P]
        L.oracle_bc.restype = ctypes.c_int
        L.oracle_bc.argtypes = [i64, P, P, i32, P, P]
        L.oracle_check_digraph.restype = ctypes.c_int
        L.oracle_check_digraph.argtypes = [i64, P, P]
        L.oracle_pagerank_directed.restype = None
        L.oracle_pagerank_directed.argtypes = [i64, P, P, f64, ctypes.c_int, ctypes.c_int, P]
        L.oracle_edgeblock.restype = i64
        L.oracle_edgeblock.argtypes = [i64, i64, P, P, i64, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _csr(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    c = np.ascontiguousarray(col, dtype=np.int32)
    if c.size == 0:
        c = np.zeros(1, dtype=np.int32)
    return rp, c


def check_csr(n, row_ptr, col) -> int:
    """0 when the CSR is sorted, unique, in range, loop-free and symmetric."""
    rp, c = _csr(row_ptr, col)
    return int(_get().oracle_check_csr(n, _p(rp), _p(c)))


def check_digraph(n, row_ptr, col) -> int:
    """0 when the CSR is sorted, unique, in range and loop-free (directed:
    no symmetry required); else check_csr's code for the first violation."""
    rp, c = _csr(row_ptr, col)
    return int(_get().oracle_check_digraph(n, _p(rp), _p(c)))


def bfs(n, row_ptr, col, src) -> np.ndarray:
    """int32 depth per vertex, -1 when unreachable."""
    rp, c = _csr(row_ptr, col)
    out = np.empty(max(n, 1), dtype=np.int32)
    if _get().oracle_bfs(n, _p(rp), _p(c), int(src), _p(out)) != 0:
        raise ValueError("bad source")
    return out[:n]


def sssp(n, row_ptr, col, w, src) -> np.ndarray:
    """int32 distance per vertex (Dijkstra), INT32_MAX when unreachable."""
    rp, c = _csr(row_ptr, col)
    ww = np.ascontiguousarray(w, dtype=np.uint32)
    if ww.size == 0:
        ww = np.zeros(1, dtype=np.uint32)
    out = np.empty(max(n, 1), dtype=np.int32)
    rc = _get().oracle_sssp(n, _p(rp), _p(c), _p(ww), int(src), _p(out))
    if rc == 1:
        raise ValueError("bad source")
    if rc == 2:
        raise OracleOverflow("distance exceeds INT32_MAX-1")
    return out[:n]


def cc(n, row_ptr, col) -> np.ndarray:
    """int32 label per vertex = smallest vertex id in its component."""
    rp, c = _csr(row_ptr, col)
    out = np.empty(max(n, 1), dtype=np.int32)
    _get().oracle_cc(n, _p(rp), _p(c), _p(out))
    return out[:n]


def pagerank(n, row_ptr, col, damping=0.85, iters=20, dangling=True) -> np.ndarray:
    """fp64 ranks after exactly `iters` power-iteration steps from 1/n."""
    rp, c = _csr(row_ptr, col)
    out = np.empty(max(n, 1), dtype=np.float64)
    _get().oracle_pagerank(n, _p(rp), _p(c), float(damping), int(iters),
                           0 if dangling else 1, _p(out))
    return out[:n]


def pagerank_directed(n, row_ptr, col, damping=0.85, iters=20, dangling=True) -> np.ndarray:
    """fp64 ranks on a directed graph (rows are out-edges): each vertex
    passes rank/out-degree along its out-edges; exactly `iters` steps from 1/n."""
    rp, c = _csr(row_ptr, col)
    out = np.empty(max(n, 1), dtype=np.float64)
    _get().oracle_pagerank_directed(n, _p(rp), _p(c), float(damping), int(iters),
                                    0 if dangling else 1, _p(out))
    return out[:n]


def bc(n, row_ptr, col, src, allow_overflow=False):
    """(sigma uint64[n], delta float64[n]) of single-source Brandes."""
    rp, c = _csr(row_ptr, col)
    sigma = np.empty(max(n, 1), dtype=np.uint64)
    delta = np.empty(max(n, 1), dtype=np.float64)
    rc = _get().oracle_bc(n, _p(rp), _p(c), int(src), _p(sigma), _p(delta))
    if rc == 1:
        raise ValueError("bad source")
    if rc == 2 and not allow_overflow:
        raise OracleOverflow("shortest-path count exceeds 2^64-1")
    return sigma[:n], delta[:n]


def edgeblock(n, src, dst, N):
    """EdgeBlocked COO: (src', dst', seg_start int64[S+1])."""
    s = np.ascontiguousarray(src, dtype=np.int32)
    d = np.ascontiguousarray(dst, dtype=np.int32)
    m = s.size
    S = (n + N - 1) // N
    os_ = np.empty(max(m, 1), dtype=np.int32)
    od = np.empty(max(m, 1), dtype=np.int32)
    seg = np.empty(S + 1, dtype=np.int64)
    _get().oracle_edgeblock(n, m, _p(s) if m else _p(os_), _p(d) if m else _p(od), int(N),
                            _p(os_), _p(od), _p(seg))
    return os_[:m], od[:m], seg


def bfs_multi(n, row_ptr, col, srcs) -> np.ndarray:
    """k x n depths: k independent single-source runs."""
    return np.stack([bfs(n, row_ptr, col, s) for s in srcs]) if len(srcs) else \
        np.zeros((0, n), dtype=np.int32)


def bc_multi(n, row_ptr, col, srcs):
    out = [bc(n, row_ptr, col, s) for s in srcs]
    return (np.stack([o[0] for o in out]), np.stack([o[1] for o in out]))
