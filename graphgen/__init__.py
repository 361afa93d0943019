"""Seeded synthetic graph inputs shared by the GPU tests/benchmark and the CPU
oracle.  Holds no BFS/SSSP arithmetic: it only builds CSR graphs and picks
sources.

Seeds: base S = 171100231; stream k of workload family c uses the SplitMix64
seed ``S ^ (c << 32) ^ k`` with k = 0 structure, 1 weights, 2 sources,
3 relabelling permutation (and 4 shortcuts for grids).

Workloads (the synthetic stand-ins for the paper's GTgraph ER/RMAT graphs,
DIMACS road networks and Graph500 graphs, which are not available here):

* ``uniform(14)``: n = 2^14, 8 out-arcs per node to uniform targets,
  self-loops dropped, duplicates kept, weights U[1,100].
* ``rmat(22)``: R-MAT scale 22, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05),
  relabelled, symmetrised, deduplicated, weights U[1,255].
* ``grid(2048)``: 2048x2048 4-neighbour lattice, 10 % of edges dropped,
  shortcuts = 1 % of kept edges with uniform endpoints, symmetrised, weights
  U[1,1000].  ``grid(..., shortcut_frac=0)`` is the high-diameter companion.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgraphgen.so")
BASE_SEED = 171100231

FAMILY_UNIFORM, FAMILY_RMAT, FAMILY_GRID, FAMILY_BATCH, FAMILY_SERVE = 0, 1, 2, 3, 4
STREAM_STRUCT, STREAM_WEIGHT, STREAM_SOURCE, STREAM_PERM, STREAM_SHORTCUT = 0, 1, 2, 3, 4


def stream_seed(family: int, stream: int, salt: int = 0) -> int:
    return (BASE_SEED ^ (family << 32) ^ stream ^ (salt << 40)) & 0xFFFFFFFFFFFFFFFF


def build(out_path: str = LIB_PATH) -> str:
    subprocess.run(["gcc", "-O3", "-std=c11", "-shared", "-fPIC", "-pthread", "-o", out_path,
                    os.path.join(HERE, "graphgen.c")], check=True)
    return out_path


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        u64, i64, i32, u32, dbl = (ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                                   ctypes.c_uint32, ctypes.c_double)
        lib.gg_uniform.restype = vp
        lib.gg_uniform.argtypes = [i64, i32, u64, u64, u32, u32]
        lib.gg_rmat.restype = vp
        lib.gg_rmat.argtypes = [ctypes.c_int, i32, dbl, dbl, dbl, u64, u64, u64, u32, u32]
        lib.gg_grid.restype = vp
        lib.gg_grid.argtypes = [i64, i64, dbl, dbl, u64, u64, u64, u32, u32]
        lib.gg_n.restype = i64
        lib.gg_n.argtypes = [vp]
        lib.gg_m.restype = i64
        lib.gg_m.argtypes = [vp]
        lib.gg_copy.restype = None
        lib.gg_copy.argtypes = [vp, vp, vp, vp]
        lib.gg_free.restype = None
        lib.gg_free.argtypes = [vp]
        lib.gg_sources.restype = i64
        lib.gg_sources.argtypes = [vp, i64, i64, u64, vp]
        lib.gg_splitmix_at.restype = u64
        lib.gg_splitmix_at.argtypes = [u64, u64]
        lib.gg_set_threads.restype = None
        lib.gg_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


@dataclass
class Graph:
    """A CSR graph: offsets int32[n+1], cols int32[m], weights uint32[m]."""

    name: str
    offsets: np.ndarray
    cols: np.ndarray
    weights: np.ndarray

    @property
    def n(self) -> int:
        return int(self.offsets.size - 1)

    @property
    def m(self) -> int:
        return int(self.cols.size)

    @property
    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64))

    def coo_src(self) -> np.ndarray:
        """Source id of every arc (the COO companion of the CSR arrays)."""
        return np.repeat(np.arange(self.n, dtype=np.int32), self.degrees)

    def reached_arcs(self, reached_mask: np.ndarray) -> int:
        """Number of CSR arcs leaving reached nodes (arcs a traversal scans)."""
        return int(self.degrees[reached_mask].sum())


def _take(h, name: str) -> Graph:
    lib = _load()
    if not h:
        raise ValueError(f"generator failed for {name}")
    try:
        n, m = lib.gg_n(h), lib.gg_m(h)
        off = np.empty(n + 1, dtype=np.int32)
        cols = np.empty(m, dtype=np.int32)
        w = np.empty(m, dtype=np.uint32)
        lib.gg_copy(h, off.ctypes.data, cols.ctypes.data, w.ctypes.data)
    finally:
        lib.gg_free(h)
    return Graph(name, off, cols, w)


def uniform(log2n: int = 14, k: int = 8, wlo: int = 1, whi: int = 100, salt: int = 0,
            n: int | None = None) -> Graph:
    nn = (1 << log2n) if n is None else int(n)
    h = _load().gg_uniform(nn, k, stream_seed(FAMILY_UNIFORM, STREAM_STRUCT, salt),
                           stream_seed(FAMILY_UNIFORM, STREAM_WEIGHT, salt), wlo, whi)
    return _take(h, f"uniform-n{nn}-k{k}")


def rmat(scale: int = 22, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, wlo: int = 1, whi: int = 255, salt: int = 0) -> Graph:
    h = _load().gg_rmat(scale, edge_factor, a, b, c,
                        stream_seed(FAMILY_RMAT, STREAM_STRUCT, salt),
                        stream_seed(FAMILY_RMAT, STREAM_PERM, salt),
                        stream_seed(FAMILY_RMAT, STREAM_WEIGHT, salt), wlo, whi)
    return _take(h, f"rmat-s{scale}-ef{edge_factor}")


def grid(width: int = 2048, height: int | None = None, drop_prob: float = 0.10,
         shortcut_frac: float = 0.01, wlo: int = 1, whi: int = 1000, salt: int = 0) -> Graph:
    hh = width if height is None else height
    h = _load().gg_grid(width, hh, drop_prob, shortcut_frac,
                        stream_seed(FAMILY_GRID, STREAM_STRUCT, salt),
                        stream_seed(FAMILY_GRID, STREAM_SHORTCUT, salt),
                        stream_seed(FAMILY_GRID, STREAM_WEIGHT, salt), wlo, whi)
    tag = "" if shortcut_frac > 0 else "-noshortcut"
    return _take(h, f"grid-{width}x{hh}{tag}")


def sources(g: Graph, count: int, family: int, salt: int = 0) -> np.ndarray:
    """``count`` distinct seeded sources with out-degree > 0."""
    out = np.empty(count, dtype=np.int32)
    off = np.ascontiguousarray(g.offsets, dtype=np.int32)
    k = _load().gg_sources(off.ctypes.data, g.n, count, stream_seed(family, STREAM_SOURCE, salt),
                           out.ctypes.data)
    return out[:k]


def from_edges(n: int, src, dst, weights=None, name: str = "edges") -> Graph:
    """CSR from an explicit arc list (kept in the given order per row)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    w = np.ones(src.size, dtype=np.uint32) if weights is None else np.asarray(weights, np.uint32)
    order = np.argsort(src, kind="stable")
    deg = np.bincount(src, minlength=n) if src.size else np.zeros(n, dtype=np.int64)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=off[1:])
    return Graph(name, off.astype(np.int32), dst[order].astype(np.int32), w[order])


def pack(graphs) -> tuple:
    """Disjoint union of several graphs in one CSR with global node ids.
    Returns (union Graph, node_base int64[k+1], edge_base int64[k+1]);
    instance i owns nodes [node_base[i], node_base[i+1])."""
    nb = np.zeros(len(graphs) + 1, dtype=np.int64)
    eb = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        nb[i + 1] = nb[i] + g.n
        eb[i + 1] = eb[i] + g.m
    if nb[-1] >= 2**31 or eb[-1] >= 2**31:
        raise ValueError("packed graph exceeds int32 ids")
    off = np.empty(nb[-1] + 1, dtype=np.int64)
    off[-1] = eb[-1]
    cols = np.empty(eb[-1], dtype=np.int32)
    w = np.empty(eb[-1], dtype=np.uint32)
    for i, g in enumerate(graphs):
        off[nb[i]: nb[i + 1]] = g.offsets[:-1].astype(np.int64) + eb[i]
        cols[eb[i]: eb[i + 1]] = g.cols.astype(np.int64) + nb[i]
        w[eb[i]: eb[i + 1]] = g.weights
    return Graph("packed", off.astype(np.int32), cols, w), nb, eb


def batch_instances(count: int = 256, salt: int = 0, lo_exp: int = 10, hi_exp: int = 18):
    """The batched workload: `count` instances of uneven size, half R-MAT
    (scale uniform in [lo_exp, hi_exp], edge factor 16, symmetrised) and half
    uniform (n = floor(2^U(lo_exp, hi_exp)), 8 out-arcs per node), weights
    U[1,255]; instance sizes come from stream 0 of the batched family."""
    seed = stream_seed(FAMILY_BATCH, STREAM_STRUCT, salt)
    graphs = []
    for i in range(count):
        x = splitmix_at(seed, i)
        if i % 2 == 0:
            scale = lo_exp + (x % (hi_exp - lo_exp + 1))
            graphs.append(rmat(scale, edge_factor=16, wlo=1, whi=255, salt=salt * 1000 + i + 1))
        else:
            u = (x >> 11) / float(1 << 53)
            n = int(2.0 ** (lo_exp + u * (hi_exp - lo_exp)))
            graphs.append(uniform(k=8, wlo=1, whi=255, salt=salt * 1000 + i + 1, n=n))
    return graphs


def splitmix_at(seed: int, i: int) -> int:
    return int(_load().gg_splitmix_at(seed, i))


def set_threads(t: int) -> None:
    _load().gg_set_threads(int(t))
