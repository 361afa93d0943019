"""CPU oracle for BFS levels and SSSP distances -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  It wraps ``oracle.c`` (plain
C, built with gcc) through ctypes and shares no code with the HIP library.

Definitions followed (paper: "Dynamic Load Balancing Strategies for Graph
Applications on GPUs"):

* ``bfs``: hop distance from the source along out-edges (Section IV, BFS
  application; Section II-B distributivity remark).
* ``dijkstra``: minimum path weight, the fixed point the data-driven SSSP of
  Sections II-B and III-A converges to.
* ``bellman_ford`` / ``floyd_warshall``: brute-force references for tiny
  graphs.
* ``certificate``: exactness certificate usable at any size.
* ``mdt``: histogram threshold of Section III-B.
* ``wd_offsets``: workload-decomposition split of Section III-A.
* ``hp_schedule``: sub-iteration sublist sizes of Section III-C.
* ``ns_pieces``: node-splitting piece sizes of Section III-B.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
BFS_INF = np.int32(2**31 - 1)
SSSP_INF = np.uint32(2**32 - 1)

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def build(out_path: str = LIB_PATH, mutant: int = 0) -> str:
    """Compile oracle.c with gcc.  ``mutant`` > 0 plants a deliberate mistake
    (used only by the tests that prove the pins catch mistakes)."""
    cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", out_path,
           os.path.join(HERE, "oracle.c")]
    if mutant:
        cmd.insert(1, f"-DORACLE_MUTANT={int(mutant)}")
    subprocess.run(cmd, check=True)
    return out_path


class Oracle:
    """ctypes view of one built oracle library."""

    def __init__(self, path: str = LIB_PATH):
        if not os.path.exists(path):
            build(path)
        lib = ctypes.CDLL(path)
        lib.oracle_bfs.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int64, _i32p]
        lib.oracle_dijkstra.argtypes = [ctypes.c_int64, _i64p, _i32p, _u32p, ctypes.c_int64, _u32p]
        lib.oracle_bellman_ford.argtypes = [ctypes.c_int64, _i64p, _i32p, _u32p, ctypes.c_int64, _u32p]
        lib.oracle_floyd_warshall.argtypes = [ctypes.c_int64, _i64p, _i32p, _u32p, _u32p]
        lib.oracle_certificate.argtypes = [ctypes.c_int64, _i64p, _i32p, _u32p, ctypes.c_int64,
                                           ctypes.c_void_p, _i64p]
        lib.oracle_mdt.argtypes = [ctypes.c_int64, _i64p, ctypes.c_int32, _i64p, _i64p]
        lib.oracle_wd_offsets.argtypes = [ctypes.c_int64, _i64p, ctypes.c_int64, _i64p, _i64p, _i64p]
        lib.oracle_hp_schedule.argtypes = [ctypes.c_int64, _i64p, ctypes.c_int64, ctypes.c_int64,
                                           _i64p, _i64p]
        lib.oracle_ns_pieces.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _i64p, _i64p]
        for f in ("oracle_bfs", "oracle_dijkstra", "oracle_bellman_ford", "oracle_floyd_warshall",
                  "oracle_certificate", "oracle_mdt", "oracle_wd_offsets", "oracle_hp_schedule",
                  "oracle_ns_pieces"):
            getattr(lib, f).restype = ctypes.c_int
        self.lib = lib

    # -- helpers -----------------------------------------------------------
    @staticmethod
    def _graph(offsets, cols, weights=None):
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        c = np.ascontiguousarray(cols, dtype=np.int32)
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.uint32)
        if c.size == 0:
            c = np.zeros(1, dtype=np.int32)
            if w is not None and w.size == 0:
                w = np.zeros(1, dtype=np.uint32)
        return off, c, w

    @staticmethod
    def _p(a, t):
        return None if a is None else a.ctypes.data_as(t)

    # -- distances ---------------------------------------------------------
    def bfs(self, offsets, cols, src):
        off, c, _ = self._graph(offsets, cols)
        n = off.size - 1
        out = np.empty(n, dtype=np.int32)
        rc = self.lib.oracle_bfs(n, self._p(off, _i64p), self._p(c, _i32p), int(src),
                                 self._p(out, _i32p))
        if rc:
            raise ValueError(f"oracle_bfs failed: {rc}")
        return out

    def dijkstra(self, offsets, cols, weights, src):
        off, c, w = self._graph(offsets, cols, weights)
        n = off.size - 1
        out = np.empty(n, dtype=np.uint32)
        rc = self.lib.oracle_dijkstra(n, self._p(off, _i64p), self._p(c, _i32p), self._p(w, _u32p),
                                      int(src), self._p(out, _u32p))
        if rc:
            raise ValueError(f"oracle_dijkstra failed: {rc}")
        return out

    def bellman_ford(self, offsets, cols, weights, src):
        off, c, w = self._graph(offsets, cols, weights)
        n = off.size - 1
        out = np.empty(n, dtype=np.uint32)
        rc = self.lib.oracle_bellman_ford(n, self._p(off, _i64p), self._p(c, _i32p),
                                          self._p(w, _u32p), int(src), self._p(out, _u32p))
        if rc:
            raise ValueError(f"oracle_bellman_ford failed: {rc}")
        return out

    def floyd_warshall(self, offsets, cols, weights):
        off, c, w = self._graph(offsets, cols, weights)
        n = off.size - 1
        out = np.empty((n, n), dtype=np.uint32)
        rc = self.lib.oracle_floyd_warshall(n, self._p(off, _i64p), self._p(c, _i32p),
                                            self._p(w, _u32p), self._p(out, _u32p))
        if rc:
            raise ValueError(f"oracle_floyd_warshall failed: {rc}")
        return out

    def certificate(self, offsets, cols, weights, src, d):
        """Returns (code, bad_index); code 0 means d is the exact distance
        vector.  ``weights=None`` certifies BFS levels (int32)."""
        off, c, w = self._graph(offsets, cols, weights)
        n = off.size - 1
        dd = np.ascontiguousarray(d, dtype=np.int32 if weights is None else np.uint32)
        if dd.size != n:
            raise ValueError("distance vector has the wrong length")
        bad = ctypes.c_int64(-1)
        rc = self.lib.oracle_certificate(n, self._p(off, _i64p), self._p(c, _i32p),
                                         self._p(w, _u32p), int(src),
                                         dd.ctypes.data_as(ctypes.c_void_p), ctypes.byref(bad))
        if rc < 0:
            raise ValueError(f"oracle_certificate failed: {rc}")
        return rc, bad.value

    # -- decomposition arithmetic -----------------------------------------
    def mdt(self, offsets, bins=10):
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        n = off.size - 1
        out = ctypes.c_int64(0)
        hist = np.zeros(bins, dtype=np.int64)
        rc = self.lib.oracle_mdt(n, self._p(off, _i64p), int(bins), ctypes.byref(out),
                                 self._p(hist, _i64p))
        if rc:
            raise ValueError(f"oracle_mdt failed: {rc}")
        return out.value, hist

    def wd_offsets(self, deg, num_threads):
        d = np.ascontiguousarray(deg, dtype=np.int64)
        ept = ctypes.c_int64(0)
        node = np.zeros(num_threads, dtype=np.int64)
        edge = np.zeros(num_threads, dtype=np.int64)
        rc = self.lib.oracle_wd_offsets(d.size, self._p(d, _i64p) if d.size else None,
                                        int(num_threads), ctypes.byref(ept),
                                        self._p(node, _i64p), self._p(edge, _i64p))
        if rc:
            raise ValueError(f"oracle_wd_offsets failed: {rc}")
        return ept.value, node, edge

    def hp_schedule(self, deg, mdt, max_sub=1 << 16):
        d = np.ascontiguousarray(deg, dtype=np.int64)
        sizes = np.zeros(max_sub, dtype=np.int64)
        ns = ctypes.c_int64(0)
        rc = self.lib.oracle_hp_schedule(d.size, self._p(d, _i64p) if d.size else None, int(mdt),
                                         max_sub, self._p(sizes, _i64p), ctypes.byref(ns))
        if rc:
            raise ValueError(f"oracle_hp_schedule failed: {rc}")
        return sizes[: min(ns.value, max_sub)]

    def ns_pieces(self, deg, mdt, max_pieces=1 << 16):
        sizes = np.zeros(max_pieces, dtype=np.int64)
        npc = ctypes.c_int64(0)
        rc = self.lib.oracle_ns_pieces(int(deg), int(mdt), max_pieces, self._p(sizes, _i64p),
                                       ctypes.byref(npc))
        if rc:
            raise ValueError(f"oracle_ns_pieces failed: {rc}")
        return sizes[: min(npc.value, max_pieces)]


_default = None


def get() -> Oracle:
    """The production oracle (built on first use if needed)."""
    global _default
    if _default is None:
        _default = Oracle(LIB_PATH)
    return _default


def mutant(k: int) -> Oracle:
    """An oracle with planted mistake number ``k`` (tests only)."""
    d = tempfile.mkdtemp(prefix="oracle_mutant_")
    return Oracle(build(os.path.join(d, f"liboracle_m{k}.so"), mutant=k))
