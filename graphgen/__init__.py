"""Seeded synthetic graph inputs (input preparation only).

Shared by the test oracle and by the GPU library's tests and benchmark. It
holds none of the traversal method's arithmetic: it builds symmetric CSR
graphs (R-MAT power-law graphs, road-like weighted grids, and small closed-form
families) and picks source vertices. The heavy generators are plain C
(``graphgen.c``), compiled with gcc on first use.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_SO = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile graphgen.c into libgraphgen.so (gcc, -O3)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def _get():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64, u64, i32, u32, f64 = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32,
                                   ctypes.c_uint32, ctypes.c_double)
        L.gen_rng.restype = u64
        L.gen_rng.argtypes = [u64, u64]
        L.gen_permutation.argtypes = [i64, u64, P]
        L.gen_rmat_edges.argtypes = [ctypes.c_int, i64, f64, f64, f64, u64, P, P]
        L.gen_build_csr.restype = i64
        L.gen_build_csr.argtypes = [i64, i64, P, P, P, P]
        L.gen_edge_weights.argtypes = [i64, P, P, u64, u32, P]
        L.gen_grid.restype = i64
        L.gen_grid.argtypes = [i32, i32, u64, i64, u32, P, P, P]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class Graph:
    """CSR: row_ptr int32[n+1], col int32[m] (rows sorted, unique, no
    self-loops), optional uint32 weights w[m]. Symmetric unless built by a
    *directed* generator, whose rows are out-edges."""
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: Optional[np.ndarray] = None
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def rng(seed: int, ctr: int) -> int:
    """Counter-based SplitMix64 draw (same stream the C generators use)."""
    return int(_get().gen_rng(int(seed) & 0xFFFFFFFFFFFFFFFF, int(ctr) & 0xFFFFFFFFFFFFFFFF))


def permutation(n: int, seed: int) -> np.ndarray:
    p = np.empty(n, dtype=np.int32)
    _get().gen_permutation(n, seed, _ptr(p))
    return p


def from_edges(n: int, src, dst, name: str = "") -> Graph:
    """Symmetric, self-loop-free, deduplicated CSR from an edge list."""
    src = np.ascontiguousarray(np.asarray(src, dtype=np.int32))
    dst = np.ascontiguousarray(np.asarray(dst, dtype=np.int32))
    assert src.shape == dst.shape
    if src.size:
        assert src.min() >= 0 and dst.min() >= 0 and src.max() < n and dst.max() < n
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col = np.empty(max(2 * src.size, 1), dtype=np.int32)
    m = _get().gen_build_csr(n, src.size, _ptr(src), _ptr(dst), _ptr(row_ptr), _ptr(col))
    return Graph(n, row_ptr, col[:m].copy(), None, name)


def rmat_edges(scale: int, ef: int = 16, a: float = 0.57, b: float = 0.19,
               c: float = 0.19, seed: Optional[int] = None):
    """Raw R-MAT edge list (before cleaning): ef * 2^scale edges."""
    if seed is None:
        seed = 1000 + scale
    m = ef * (1 << scale)
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    _get().gen_rmat_edges(scale, m, a, b, c, seed, _ptr(src), _ptr(dst))
    return src, dst


def rmat(scale: int, ef: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: Optional[int] = None, weights: bool = False,
         weight_seed: Optional[int] = None) -> Graph:
    """R-MAT(scale, ef, a, b, c) -> symmetric CSR with 2^scale vertices."""
    if seed is None:
        seed = 1000 + scale
    src, dst = rmat_edges(scale, ef, a, b, c, seed)
    g = from_edges(1 << scale, src, dst, name="rmat%d" % scale)
    del src, dst
    if weights:
        add_weights(g, seed + 7 if weight_seed is None else weight_seed)
    return g


def from_edges_directed(n: int, src, dst, name: str = "") -> Graph:
    """Directed CSR (rows are out-edges) from an edge list: self-loops
    dropped, repeated edges merged, rows sorted; not symmetrised."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    assert src.shape == dst.shape
    if src.size:
        assert src.min() >= 0 and dst.min() >= 0 and src.max() < n and dst.max() < n
    keep = src != dst
    key = np.unique(src[keep] * n + dst[keep])
    s = key // n
    col = (key % n).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(s, minlength=n), out=row_ptr[1:])
    return Graph(n, row_ptr.astype(np.int32), col, None, name)


def rmat_directed(scale: int, ef: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
                  seed: Optional[int] = None, weights: bool = False,
                  weight_seed: Optional[int] = None) -> Graph:
    """The R-MAT(scale, ef, a, b, c) edge list of rmat() kept directed: each
    generated edge u -> v once, no mirror."""
    if seed is None:
        seed = 1000 + scale
    src, dst = rmat_edges(scale, ef, a, b, c, seed)
    g = from_edges_directed(1 << scale, src, dst, name="rmat%d-directed" % scale)
    del src, dst
    if weights:
        add_weights(g, seed + 7 if weight_seed is None else weight_seed)
    return g


def random_digraph(n: int, p: float, seed: int) -> Graph:
    """Directed G(n, p): each ordered pair u != v kept with probability p
    (counter-based stream)."""
    u, v = np.nonzero(~np.eye(n, dtype=bool))
    keep = np.array([rng(seed, int(i)) >> 11 for i in range(u.size)], dtype=np.float64) \
        * (1.0 / 9007199254740992.0) < p
    return from_edges_directed(n, u[keep], v[keep], name="dgnp%d" % n)


def add_weights(g: Graph, seed: int, wmax: int = 999) -> Graph:
    """Symmetric per-edge weights uniform in 1..wmax (keyed by the unordered pair)."""
    w = np.empty(g.m, dtype=np.uint32)
    _get().gen_edge_weights(g.n, _ptr(g.row_ptr), _ptr(g.col), seed, wmax, _ptr(w))
    g.w = w
    return g


def grid(W: int, H: Optional[int] = None, seed: Optional[int] = None,
         drop_frac: float = 0.1, wmax: int = 999) -> Graph:
    """Road-like W x H grid: spanning tree kept, round(drop_frac*U) of the
    non-tree edges dropped, symmetric weights uniform in 1..wmax."""
    if H is None:
        H = W
    if seed is None:
        seed = W
    U = (W - 1) * H + W * (H - 1)
    ndrop = int(round(drop_frac * U))
    n = W * H
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col = np.empty(max(2 * U, 1), dtype=np.int32)
    w = np.empty(max(2 * U, 1), dtype=np.uint32)
    m = _get().gen_grid(W, H, seed, ndrop, wmax, _ptr(row_ptr), _ptr(col), _ptr(w))
    return Graph(n, row_ptr, col[:m].copy(), w[:m].copy(), name="grid%dx%d" % (W, H))


# ---- small closed-form families -------------------------------------------

def path(n: int) -> Graph:
    i = np.arange(max(n - 1, 0))
    return from_edges(n, i, i + 1, name="path%d" % n)


def cycle(n: int) -> Graph:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, name="cycle%d" % n)


def star(k: int) -> Graph:
    """K_{1,k}: centre 0, leaves 1..k."""
    return from_edges(k + 1, np.zeros(k, dtype=np.int32), np.arange(1, k + 1), name="star%d" % k)


def complete(n: int) -> Graph:
    u, v = np.triu_indices(n, 1)
    return from_edges(n, u, v, name="K%d" % n)


def isolated(n: int) -> Graph:
    e = np.zeros(0, dtype=np.int32)
    return from_edges(n, e, e, name="empty%d" % n)


def full_grid(W: int, H: int) -> Graph:
    """Undropped W x H 4-neighbour grid, id = r*W + c."""
    ids = np.arange(W * H).reshape(H, W)
    s = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    d = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    return from_edges(W * H, s, d, name="fullgrid%dx%d" % (W, H))


def disjoint_cliques(sizes) -> Graph:
    src, dst, off = [], [], 0
    for k in sizes:
        u, v = np.triu_indices(k, 1)
        src.append(u + off)
        dst.append(v + off)
        off += k
    return from_edges(off, np.concatenate(src) if src else [], np.concatenate(dst) if dst else [],
                      name="cliques")


def random_graph(n: int, p: float, seed: int) -> Graph:
    """Erdos-Renyi G(n, p) from the counter-based stream."""
    u, v = np.triu_indices(n, 1)
    keep = np.array([rng(seed, int(i)) >> 11 for i in range(u.size)], dtype=np.float64) \
        * (1.0 / 9007199254740992.0) < p
    return from_edges(n, u[keep], v[keep], name="gnp%d" % n)


# ---- sources ----------------------------------------------------------------

def max_degree_vertex(g: Graph) -> int:
    """Highest-degree vertex, ties to the smallest id."""
    return int(np.argmax(g.degrees()))


def sample_sources(g: Graph, k: int, seed: int) -> np.ndarray:
    """k distinct sources uniform over the non-isolated vertices."""
    cand = np.nonzero(g.degrees() > 0)[0].astype(np.int32)
    if cand.size == 0:
        return np.zeros(0, dtype=np.int32)
    k = min(k, cand.size)
    out, seen, ctr = [], set(), 0
    while len(out) < k:
        j = int((rng(seed, ctr) * cand.size) >> 64)
        ctr += 1
        if j not in seen:
            seen.add(j)
            out.append(int(cand[j]))
    return np.array(out, dtype=np.int32)


def giant_component(g: Graph) -> np.ndarray:
    """Vertex ids of the largest connected component, ascending (ties: the
    component holding the smaller id). Input selection only, by scipy's
    connected_components."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    A = sp.csr_matrix((np.ones(g.m, dtype=np.int8), g.col, g.row_ptr), shape=(g.n, g.n))
    _, lab = connected_components(A, directed=False)
    sizes = np.bincount(lab)
    return np.nonzero(lab == int(np.argmax(sizes)))[0].astype(np.int32)


def sample_giant_sources(g: Graph, k: int, seed: int) -> np.ndarray:
    """k distinct sources uniform over the largest connected component."""
    cand = giant_component(g)
    k = min(k, cand.size)
    out, seen, ctr = [], set(), 0
    while len(out) < k:
        j = int((rng(seed, ctr) * cand.size) >> 64)
        ctr += 1
        if j not in seen:
            seen.add(j)
            out.append(int(cand[j]))
    return np.array(out, dtype=np.int32)

