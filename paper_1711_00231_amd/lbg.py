"""Thin Python binding of the lbg C ABI (include/lbg.h).

Argument marshalling only: every step of BFS/SSSP runs in the HIP kernels of
liblbg.so.  torch provides device memory and the current HIP stream.  If the
library is not built, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbg.so")

OK, EINVAL, ERANGE, ENOMEM, EHIP, EOVERFLOW, EINTERNAL, EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
AUTO, NODE, EDGE, BALANCED, BINNED, EDGE_NOCHUNK, HIER, SLICED, SPLIT = 0, 1, 2, 3, 4, 5, 6, 7, 8
STRATEGIES = {"auto": AUTO, "node": NODE, "edge": EDGE, "balanced": BALANCED, "binned": BINNED,
              "edge_nochunk": EDGE_NOCHUNK, "hier": HIER, "sliced": SLICED,
              "split": SPLIT}
BFS_INF = 2**31 - 1
SSSP_INF = 2**32 - 1
NOALLOC_SCRATCH_BYTES = 64 << 20  # LBG_NOALLOC_SCRATCH_BYTES


class LbgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbg error {code}: {msg}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("frontier_entries", ctypes.c_int64), ("edges_scanned", ctypes.c_int64),
                ("updates", ctypes.c_int64), ("atomics", ctypes.c_int64),
                ("edges_skipped", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


KIND_BFS, KIND_SSSP = 0, 1


class Query(ctypes.Structure):
    _fields_ = [("src", ctypes.c_int32), ("lo", ctypes.c_int32), ("hi", ctypes.c_int32),
                ("kind", ctypes.c_int32), ("out_off", ctypes.c_int64)]


class Bins(ctypes.Structure):
    _fields_ = [("mdt", ctypes.c_int32), ("t_wave", ctypes.c_int32), ("t_block", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("empty_launches", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double), ("empty_ms", ctypes.c_double),
                ("frontier_entries", ctypes.c_int64),
                ("edges_scanned", ctypes.c_int64), ("updates", ctypes.c_int64),
                ("atomics", ctypes.c_int64), ("edges_skipped", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.lbg_workspace_bytes.restype = sz
    lib.lbg_workspace_bytes.argtypes = [i32, i64, i32, i32]
    lib.lbg_bfs.restype = ctypes.c_int
    lib.lbg_bfs.argtypes = [vp, vp, i32, i64, i32, vp, vp, sz, i32, vp, ctypes.POINTER(Stats), vp]
    lib.lbg_sssp.restype = ctypes.c_int
    lib.lbg_sssp.argtypes = [vp, vp, vp, i32, i64, i32, vp, vp, sz, i32, vp,
                             ctypes.POINTER(Stats), vp]
    lib.lbg_sssp_noalloc.restype = ctypes.c_int
    lib.lbg_sssp_noalloc.argtypes = [vp, vp, vp, i32, i64, i32, vp, i32, ctypes.POINTER(Stats), vp]
    lib.lbg_coo_sources.restype = ctypes.c_int
    lib.lbg_coo_sources.argtypes = [vp, i32, i64, vp, vp]
    lib.lbg_set_hier_mdt.restype = ctypes.c_int
    lib.lbg_set_hier_mdt.argtypes = [i32]
    lib.lbg_get_hier_mdt.restype = i32
    lib.lbg_get_hier_mdt.argtypes = []
    lib.lbg_hier_last_schedule.restype = i32
    lib.lbg_hier_last_schedule.argtypes = [ctypes.POINTER(i32), i32, i32, ctypes.POINTER(i32)]
    lib.lbg_pack_arcs.restype = ctypes.c_int
    lib.lbg_pack_arcs.argtypes = [vp, vp, i32, i64, vp, ctypes.POINTER(i32), vp, sz, vp]
    lib.lbg_sssp_packed.restype = ctypes.c_int
    lib.lbg_sssp_packed.argtypes = [vp, vp, i32, i32, i64, i32, vp, vp, sz, ctypes.POINTER(Stats), vp]
    lib.lbg_slice_nodes.restype = i32
    lib.lbg_slice_nodes.argtypes = [i32]
    lib.lbg_set_slice_min.restype = ctypes.c_int
    lib.lbg_set_slice_min.argtypes = [i32]
    lib.lbg_set_addressing.restype = ctypes.c_int
    lib.lbg_set_addressing.argtypes = [i32]
    lib.lbg_get_addressing.restype = i32
    lib.lbg_get_addressing.argtypes = []
    lib.lbg_set_bfs_scan_min.restype = ctypes.c_int
    lib.lbg_set_bfs_scan_min.argtypes = [i64]
    lib.lbg_get_bfs_scan_min.restype = i64
    lib.lbg_get_bfs_scan_min.argtypes = []
    lib.lbg_get_slice_min.restype = i32
    lib.lbg_get_slice_min.argtypes = []
    lib.lbg_slice_graph.restype = ctypes.c_int
    lib.lbg_slice_graph.argtypes = [vp, vp, vp, i32, i64, vp, vp, vp, vp]
    lib.lbg_bfs_sliced.restype = ctypes.c_int
    lib.lbg_bfs_sliced.argtypes = [vp, vp, vp, i32, i64, i32, vp, vp, sz, ctypes.POINTER(Stats), vp]
    lib.lbg_sssp_sliced.restype = ctypes.c_int
    lib.lbg_sssp_sliced.argtypes = [vp, vp, vp, vp, i32, i64, i32, vp, vp, sz, ctypes.POINTER(Stats), vp]
    lib.lbg_split_scratch_bytes.restype = sz
    lib.lbg_split_scratch_bytes.argtypes = [i32]
    lib.lbg_split_count.restype = ctypes.c_int
    lib.lbg_split_count.argtypes = [vp, i32, i64, i32, ctypes.POINTER(i64), vp, sz, vp]
    lib.lbg_split_graph.restype = ctypes.c_int
    lib.lbg_split_graph.argtypes = [vp, vp, vp, i32, i64, i32, i64, vp, vp, vp, vp, vp, sz, vp]
    lib.lbg_split_workspace_bytes.restype = sz
    lib.lbg_split_workspace_bytes.argtypes = [i32, i64, i64, i32]
    lib.lbg_bfs_split.restype = ctypes.c_int
    lib.lbg_bfs_split.argtypes = [vp, vp, vp, i32, i64, i64, i32, vp, vp, sz, ctypes.POINTER(Stats), vp]
    lib.lbg_sssp_split.restype = ctypes.c_int
    lib.lbg_sssp_split.argtypes = [vp, vp, vp, vp, i32, i64, i64, i32, vp, vp, sz, ctypes.POINTER(Stats), vp]
    lib.lbg_order_scratch_bytes.restype = sz
    lib.lbg_order_scratch_bytes.argtypes = [i32]
    lib.lbg_order_graph.restype = ctypes.c_int
    lib.lbg_order_graph.argtypes = [vp, vp, vp, i32, i64, vp, vp, vp, vp, vp, sz, vp]
    lib.lbg_sssp_ordered.restype = ctypes.c_int
    lib.lbg_sssp_ordered.argtypes = [vp, vp, vp, vp, i32, i64, i32, vp, vp, sz, ctypes.POINTER(Stats), vp]
    lib.lbg_validate_csr.restype = ctypes.c_int
    lib.lbg_validate_csr.argtypes = [vp, vp, i32, i64, vp, sz, vp]
    lib.lbg_last_error.restype = ctypes.c_char_p
    lib.lbg_last_error.argtypes = []
    lib.lbg_profile_enable.restype = None
    lib.lbg_profile_enable.argtypes = [i32, i32]
    lib.lbg_profile_read.restype = None
    lib.lbg_profile_read.argtypes = [i32, ctypes.POINTER(Profile)]
    lib.lbg_batch_workspace_bytes.restype = sz
    lib.lbg_batch_workspace_bytes.argtypes = [i32, i64, i64]
    lib.lbg_batch_solve.restype = ctypes.c_int
    lib.lbg_batch_solve.argtypes = [vp, vp, vp, i32, i64, ctypes.POINTER(Query), i32, vp, i64, i64,
                                    vp, sz, ctypes.POINTER(Stats), vp]
    lib.lbg_batch_solve_graph.restype = ctypes.c_int
    lib.lbg_batch_solve_graph.argtypes = lib.lbg_batch_solve.argtypes
    lib.lbg_engine_workspace_bytes.restype = sz
    lib.lbg_engine_workspace_bytes.argtypes = [i32, i64, i64]
    lib.lbg_engine_create.restype = ctypes.c_int
    lib.lbg_engine_create.argtypes = [vp, vp, vp, i32, i64, i32, i64, i64, vp, vp, sz, vp,
                                      ctypes.POINTER(vp)]
    lib.lbg_engine_submit.restype = ctypes.c_int
    lib.lbg_engine_submit.argtypes = [vp, ctypes.POINTER(Query), ctypes.POINTER(i32)]
    lib.lbg_engine_step.restype = ctypes.c_int
    lib.lbg_engine_step.argtypes = [vp, i32, ctypes.POINTER(i32)]
    lib.lbg_engine_finished.restype = i32
    lib.lbg_engine_finished.argtypes = [vp, ctypes.POINTER(i32), i32]
    lib.lbg_engine_release.restype = ctypes.c_int
    lib.lbg_engine_release.argtypes = [vp, i32]
    lib.lbg_engine_info.restype = ctypes.c_int
    lib.lbg_engine_info.argtypes = [vp, ctypes.POINTER(Stats), ctypes.POINTER(i32),
                                    ctypes.POINTER(ctypes.c_uint32)]
    lib.lbg_engine_destroy.restype = None
    lib.lbg_engine_destroy.argtypes = [vp]
    lib.lbg_set_bins.restype = ctypes.c_int
    lib.lbg_set_bins.argtypes = [ctypes.POINTER(Bins)]
    lib.lbg_get_bins.restype = None
    lib.lbg_get_bins.argtypes = [ctypes.POINTER(Bins)]
    lib.lbg_degree_mdt.restype = ctypes.c_int
    lib.lbg_degree_mdt.argtypes = [vp, i32, i64, vp, sz, ctypes.POINTER(i32), ctypes.POINTER(i32), vp]
    lib.lbg_autotune_bins.restype = ctypes.c_int
    lib.lbg_autotune_bins.argtypes = [vp, vp, vp, i32, i64, ctypes.POINTER(i32), i32, vp, vp, sz,
                                      ctypes.POINTER(Bins), vp]
    lib.lbg_tile_edges.restype = i32
    lib.lbg_tile_edges.argtypes = []
    lib.lbg_grid_blocks.restype = i32
    lib.lbg_grid_blocks.argtypes = []
    return lib


lib = _load()


def _check(rc: int):
    if rc != OK:
        raise LbgError(rc, lib.lbg_last_error().decode())


def _strategy(s) -> int:
    if isinstance(s, str):
        return STRATEGIES[s]
    return int(s)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _out(out, n: int, device, what: str = "out"):
    """The caller's result tensor, checked (the library writes n 4-byte
    words through its pointer and cannot see its size), or a new one."""
    if out is None:
        return torch.empty(n, dtype=torch.int32, device=device)
    if (out.dtype not in (torch.int32, torch.uint32) or out.dim() != 1 or not out.is_contiguous()
            or out.device != device or out.numel() < n):
        raise ValueError(f"{what} must be a contiguous 1-D int32 tensor of at least {n} elements on "
                         f"{device} (got shape {tuple(out.shape)}, {out.dtype}, on {out.device})")
    return out


def workspace_bytes(n: int, m: int, strategy="balanced", sssp: bool = False) -> int:
    return int(lib.lbg_workspace_bytes(n, m, _strategy(strategy), int(sssp)))


@dataclass
class DeviceGraph:
    """A CSR graph resident in device memory (int32 offsets/cols, uint32
    weights stored in an int32 tensor).  ``coo_src`` (edge-based strategy)
    and ``sliced`` (destination-sliced strategy) are built only on demand."""

    offsets: torch.Tensor
    cols: torch.Tensor
    weights: torch.Tensor | None
    coo_src: torch.Tensor | None = None
    host_offsets: object = None  # numpy copy, used to size batched solves
    sliced: "SlicedGraph | None" = None
    packed: "tuple | None" = None  # (arcs tensor, wbits) from lbg_pack_arcs
    split: "SplitGraph | None" = None
    ordered: "OrderedGraph | None" = None

    def __post_init__(self):
        dev = self.offsets.device
        for name, t, types in (("offsets", self.offsets, (torch.int32,)), ("cols", self.cols, (torch.int32,)),
                               ("weights", self.weights, (torch.int32, torch.uint32))):
            if t is not None and (t.dtype not in types or t.dim() != 1 or not t.is_contiguous()
                                  or t.device != dev):
                raise ValueError(f"{name} must be a contiguous 1-D 32-bit integer tensor on {dev} "
                                 f"(got shape {tuple(t.shape)}, {t.dtype}, on {t.device})")
        if self.offsets.numel() < 1:
            raise ValueError("offsets needs n + 1 >= 1 entries")
        if self.weights is not None and self.weights.numel() != self.cols.numel():
            raise ValueError(f"weights has {self.weights.numel()} entries for {self.cols.numel()} arcs")

    @property
    def n(self) -> int:
        return int(self.offsets.numel() - 1)

    @property
    def m(self) -> int:
        return int(self.cols.numel())

    @classmethod
    def from_numpy(cls, offsets, cols, weights=None, device="cuda", with_coo=False, with_slices=False,
                   with_packed=False):
        import numpy as np

        off = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int32)).to(device)
        c = torch.from_numpy(np.ascontiguousarray(cols, dtype=np.int32)).to(device)
        w = None
        if weights is not None:
            w = torch.from_numpy(np.ascontiguousarray(weights, dtype=np.uint32).view(np.int32)).to(device)
        g = cls(off, c, w, None, np.ascontiguousarray(offsets, dtype=np.int64))
        if with_coo:
            g.ensure_coo()
        if with_slices:
            g.ensure_sliced()
        if with_packed:
            g.ensure_packed()
        return g

    def ensure_packed(self, stream=None) -> tuple:
        """(arcs, wbits): arc e as one word (cols[e] << wbits) | weights[e]
        (lbg_pack_arcs); raises LbgError(ERANGE) if ids and weights do not
        fit in 32 bits."""
        if self.packed is None:
            if self.weights is None:
                raise ValueError("packing needs weights")
            dev = self.offsets.device
            arcs = torch.empty(max(self.m, 1), dtype=torch.int32, device=dev)
            scratch = _ws(None, 4096, dev)
            wb = ctypes.c_int32(0)
            _check(lib.lbg_pack_arcs(_ptr(self.cols), _ptr(self.weights), self.n, self.m, _ptr(arcs),
                                     ctypes.byref(wb), _ptr(scratch), scratch.numel(), _stream(stream)))
            self.packed = (arcs, int(wb.value))
        return self.packed

    def ensure_sliced(self, stream=None) -> "SlicedGraph":
        if self.sliced is None:
            self.sliced = slice_graph(self, stream=stream)
        return self.sliced

    def ensure_split(self, mdt: int | None = None, stream=None) -> "SplitGraph":
        """The split graph for split size ``mdt`` (None: the histogram rule
        of lbg_degree_mdt), rebuilt when a different size is asked for."""
        if mdt is None:
            if self.split is not None and self.split.auto:
                return self.split
            mdt_v, auto = degree_mdt(self, stream=stream)[0], True
        else:
            mdt_v, auto = int(mdt), False
        if self.split is None or self.split.mdt != mdt_v:
            self.split = split_graph(self, mdt_v, stream=stream)
        self.split.auto = auto
        return self.split

    def ensure_ordered(self, stream=None) -> "OrderedGraph":
        """The degree-class ordered copy (lbg_order_graph), built once."""
        if self.ordered is None:
            self.ordered = order_graph(self, stream=stream)
        return self.ordered

    def ensure_coo(self, stream=None) -> torch.Tensor:
        """The COO source array of the edge-based strategy, built by the
        library (lbg_coo_sources) once per graph."""
        if self.coo_src is None:
            coo = torch.empty(max(self.m, 1), dtype=torch.int32, device=self.offsets.device)
            _check(lib.lbg_coo_sources(_ptr(self.offsets), self.n, self.m, _ptr(coo), _stream(stream)))
            self.coo_src = coo
        return self.coo_src


@dataclass
class SlicedGraph:
    """The same graph with every adjacency list grouped by destination slice
    (lbg_slice_graph): slice_offsets[8n + 1], cols, weights."""

    slice_offsets: torch.Tensor
    cols: torch.Tensor
    weights: torch.Tensor | None
    n: int
    m: int


def slice_nodes(n: int) -> int:
    return int(lib.lbg_slice_nodes(int(n)))


def set_slice_min(min_degree: int) -> None:
    """Degree from which the sliced strategy splits a node by destination
    slice (see lbg_set_slice_min)."""
    _check(lib.lbg_set_slice_min(int(min_degree)))


def get_slice_min() -> int:
    return int(lib.lbg_get_slice_min())


def set_bfs_scan_min(arcs: int) -> None:
    """Frontier arcs from which a balanced BFS level runs in scan mode
    (< 0: n / 4, 0: every level, >= 2**32: never; see lbg_set_bfs_scan_min)."""
    _check(lib.lbg_set_bfs_scan_min(int(arcs)))


def get_bfs_scan_min() -> int:
    return int(lib.lbg_get_bfs_scan_min())


def set_addressing(mode: int) -> None:
    """0: 32-bit element offsets whenever the arrays fit (default), 1: 64-bit
    addresses always (see lbg_set_addressing)."""
    _check(lib.lbg_set_addressing(int(mode)))


def get_addressing() -> int:
    return int(lib.lbg_get_addressing())


def slice_graph(g: DeviceGraph, stream=None) -> SlicedGraph:
    dev = g.offsets.device
    so = torch.empty(8 * g.n + 1, dtype=torch.int32, device=dev)
    cols = torch.empty(max(g.m, 1), dtype=torch.int32, device=dev)
    w = None if g.weights is None else torch.empty(max(g.m, 1), dtype=torch.int32, device=dev)
    _check(lib.lbg_slice_graph(_ptr(g.offsets), _ptr(g.cols), _ptr(g.weights), g.n, g.m, _ptr(so),
                               _ptr(cols), _ptr(w), _stream(stream)))
    return SlicedGraph(so, cols, w, g.n, g.m)


@dataclass
class SplitGraph:
    """The graph with every node of more than ``mdt`` out-arcs cut into
    pieces held by child nodes (lbg_split_graph): split_offsets[n + children
    + 1], child_base[n + 1], cols, weights."""

    split_offsets: torch.Tensor
    child_base: torch.Tensor
    cols: torch.Tensor
    weights: torch.Tensor | None
    n: int
    m: int
    mdt: int
    children: int
    auto: bool = False


def split_count(g: DeviceGraph, mdt: int, stream=None) -> int:
    """Number of child nodes node splitting with split size ``mdt`` makes."""
    dev = g.offsets.device
    scratch = _ws(None, int(lib.lbg_split_scratch_bytes(g.n)), dev)
    c = ctypes.c_int64(0)
    _check(lib.lbg_split_count(_ptr(g.offsets), g.n, g.m, int(mdt), ctypes.byref(c), _ptr(scratch),
                               scratch.numel(), _stream(stream)))
    return int(c.value)


def split_graph(g: DeviceGraph, mdt: int, stream=None) -> SplitGraph:
    dev = g.offsets.device
    children = split_count(g, mdt, stream)
    scratch = _ws(None, int(lib.lbg_split_scratch_bytes(g.n)), dev)
    so = torch.empty(g.n + children + 1, dtype=torch.int32, device=dev)
    cb = torch.empty(g.n + 1, dtype=torch.int32, device=dev)
    cols = torch.empty(max(g.m, 1), dtype=torch.int32, device=dev)
    w = None if g.weights is None else torch.empty(max(g.m, 1), dtype=torch.int32, device=dev)
    _check(lib.lbg_split_graph(_ptr(g.offsets), _ptr(g.cols), _ptr(g.weights), g.n, g.m, int(mdt), children,
                               _ptr(so), _ptr(cb), _ptr(cols), _ptr(w), _ptr(scratch), scratch.numel(),
                               _stream(stream)))
    return SplitGraph(so, cb, cols, w, g.n, g.m, int(mdt), children)


@dataclass
class OrderedGraph:
    """The graph renumbered by degree class, largest first (lbg_order_graph):
    offsets, cols, weights in new ids and new_id[v] of every original node."""

    offsets: torch.Tensor
    cols: torch.Tensor
    weights: torch.Tensor | None
    new_id: torch.Tensor
    n: int
    m: int


def order_graph(g: DeviceGraph, stream=None) -> OrderedGraph:
    dev = g.offsets.device
    scratch = torch.empty(max(int(lib.lbg_order_scratch_bytes(g.n)), 256), dtype=torch.uint8, device=dev)
    off = torch.empty(g.n + 1, dtype=torch.int32, device=dev)
    nid = torch.empty(g.n, dtype=torch.int32, device=dev)
    cols = torch.empty(max(g.m, 1), dtype=torch.int32, device=dev)
    w = None if g.weights is None else torch.empty(max(g.m, 1), dtype=torch.int32, device=dev)
    _check(lib.lbg_order_graph(_ptr(g.offsets), _ptr(g.cols), _ptr(g.weights), g.n, g.m, _ptr(off), _ptr(cols),
                               _ptr(w), _ptr(nid), _ptr(scratch), scratch.numel(), _stream(stream)))
    return OrderedGraph(off, cols, w, nid, g.n, g.m)


def split_workspace_bytes(n: int, m: int, children: int, sssp: bool = False) -> int:
    return int(lib.lbg_split_workspace_bytes(n, m, children, int(sssp)))


class Workspace:
    """Caller-owned device workspace, grown on demand and reused."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self.buf


_default_ws: dict = {}


def _ws(workspace, nbytes, device):
    if workspace is None:
        key = str(device)
        workspace = _default_ws.setdefault(key, Workspace(device))
    return workspace.get(nbytes)


def bfs(g: DeviceGraph, src: int, strategy="balanced", out: torch.Tensor | None = None,
        workspace: Workspace | None = None, stats: bool = False, stream=None, mdt: int | None = None):
    """Levels from ``src`` (int32, INT32_MAX = unreachable).  Returns the
    tensor, or (tensor, stats dict) if ``stats``.  ``mdt``: split size of
    the 'split' strategy (None: the histogram rule)."""
    s = _strategy(strategy)
    out = _out(out, g.n, g.offsets.device)
    need = workspace_bytes(g.n, g.m, s, False) if s != SPLIT else 0  # sized below
    ws = _ws(workspace, need, g.offsets.device)
    coo = g.ensure_coo() if s in (EDGE, EDGE_NOCHUNK) else None
    st = Stats()
    if s == SPLIT:
        sp = g.ensure_split(mdt, stream=stream)
        ws = _ws(workspace, split_workspace_bytes(g.n, g.m, sp.children, False), g.offsets.device)
        rc = lib.lbg_bfs_split(_ptr(sp.split_offsets), _ptr(sp.child_base), _ptr(sp.cols), g.n, sp.children,
                               g.m, int(src), _ptr(out), _ptr(ws), ws.numel(),
                               ctypes.byref(st) if stats else None, _stream(stream))
    elif s == SLICED:
        sg = g.ensure_sliced(stream)
        rc = lib.lbg_bfs_sliced(_ptr(g.offsets), _ptr(sg.slice_offsets), _ptr(sg.cols), g.n, g.m, int(src),
                                _ptr(out), _ptr(ws), ws.numel(), ctypes.byref(st) if stats else None,
                                _stream(stream))
    else:
        rc = lib.lbg_bfs(_ptr(g.offsets), _ptr(g.cols), g.n, g.m, int(src), _ptr(out), _ptr(ws),
                         ws.numel(), s, _ptr(coo), ctypes.byref(st) if stats else None, _stream(stream))
    _check(rc)
    return (out, st.as_dict()) if stats else out


def sssp(g: DeviceGraph, src: int, strategy="balanced", out: torch.Tensor | None = None,
         workspace: Workspace | None = None, stats: bool = False, stream=None, packed: bool = False,
         mdt: int | None = None, ordered: bool = False):
    """Distances from ``src`` as an int32 tensor holding uint32 bit patterns
    (use ``.view(torch.uint32)``; UINT32_MAX = unreachable).  ``packed``:
    balanced strategy on the packed arc words (lbg_sssp_packed).  ``mdt``:
    split size of the 'split' strategy (None: the histogram rule).
    ``ordered``: balanced strategy on the degree-class ordered copy
    (lbg_sssp_ordered); source and result stay in original ids."""
    s = _strategy(strategy)
    if (packed or ordered) and s not in (AUTO, BALANCED):
        raise ValueError("packed arcs and the ordered copy run the balanced strategy")
    if packed and ordered:
        raise ValueError("packed arcs and the ordered copy are separate layouts")
    if g.weights is None:
        raise ValueError("sssp needs weights")
    out = _out(out, g.n, g.offsets.device)
    need = workspace_bytes(g.n, g.m, s, True) if s != SPLIT else 0  # sized below
    ws = _ws(workspace, need, g.offsets.device)
    coo = g.ensure_coo() if s in (EDGE, EDGE_NOCHUNK) else None
    st = Stats()
    if ordered:
        og = g.ensure_ordered(stream)
        rc = lib.lbg_sssp_ordered(_ptr(og.offsets), _ptr(og.cols), _ptr(og.weights), _ptr(og.new_id), g.n, g.m,
                                  int(src), _ptr(out), _ptr(ws), ws.numel(), ctypes.byref(st) if stats else None,
                                  _stream(stream))
    elif packed:
        arcs, wbits = g.ensure_packed(stream)
        rc = lib.lbg_sssp_packed(_ptr(g.offsets), _ptr(arcs), wbits, g.n, g.m, int(src), _ptr(out), _ptr(ws),
                                 ws.numel(), ctypes.byref(st) if stats else None, _stream(stream))
    elif s == SPLIT:
        sp = g.ensure_split(mdt, stream=stream)
        if sp.weights is None:
            raise ValueError("the split graph was built without weights")
        ws = _ws(workspace, split_workspace_bytes(g.n, g.m, sp.children, True), g.offsets.device)
        rc = lib.lbg_sssp_split(_ptr(sp.split_offsets), _ptr(sp.child_base), _ptr(sp.cols), _ptr(sp.weights),
                                g.n, sp.children, g.m, int(src), _ptr(out), _ptr(ws), ws.numel(),
                                ctypes.byref(st) if stats else None, _stream(stream))
    elif s == SLICED:
        sg = g.ensure_sliced(stream)
        if sg.weights is None:
            raise ValueError("the sliced graph was built without weights")
        rc = lib.lbg_sssp_sliced(_ptr(g.offsets), _ptr(sg.slice_offsets), _ptr(sg.cols), _ptr(sg.weights),
                                 g.n, g.m, int(src), _ptr(out), _ptr(ws), ws.numel(),
                                 ctypes.byref(st) if stats else None, _stream(stream))
    else:
        rc = lib.lbg_sssp(_ptr(g.offsets), _ptr(g.cols), _ptr(g.weights), g.n, g.m, int(src),
                          _ptr(out), _ptr(ws), ws.numel(), s, _ptr(coo),
                          ctypes.byref(st) if stats else None, _stream(stream))
    _check(rc)
    return (out, st.as_dict()) if stats else out


def sssp_noalloc(g: DeviceGraph, src: int, strategy="balanced", out: torch.Tensor | None = None,
                 stats: bool = False, stream=None):
    """lbg_sssp_noalloc: SSSP whose workspace is the library's own static
    device array (no allocation in the call; sizes up to
    NOALLOC_SCRATCH_BYTES of workspace).  ``out`` must be given by callers
    that cannot allocate; calls that overlap on one GPU race."""
    if g.weights is None:
        raise ValueError("sssp needs weights")
    out = _out(out, g.n, g.offsets.device)
    st = Stats()
    rc = lib.lbg_sssp_noalloc(_ptr(g.offsets), _ptr(g.cols), _ptr(g.weights), g.n, g.m, int(src), _ptr(out),
                              _strategy(strategy), ctypes.byref(st) if stats else None, _stream(stream))
    _check(rc)
    return (out, st.as_dict()) if stats else out


_QUERY_DTYPE = None


def _query_dtype():
    global _QUERY_DTYPE
    if _QUERY_DTYPE is None:
        import numpy as np

        _QUERY_DTYPE = np.dtype({"names": [f for f, _ in Query._fields_],
                                 "formats": ["<i4", "<i4", "<i4", "<i4", "<i8"],
                                 "offsets": [getattr(Query, f).offset for f, _ in Query._fields_],
                                 "itemsize": ctypes.sizeof(Query)})
    return _QUERY_DTYPE


def batch_queries(queries):
    """Query array from (src, lo, hi, kind[, out_off]) tuples; missing row
    offsets are assigned back to back.  Returns (Query array, total_rows).
    The array is a ctypes view of a numpy record array (attribute ``rec``)."""
    import numpy as np

    k = len(queries)
    rec = np.zeros(k, dtype=_query_dtype())
    widths = {len(q) for q in queries}
    if k and widths <= {4, 5} and len(widths) == 1:
        a = np.array(queries, dtype=np.int64).reshape(k, -1)
        for j, f in enumerate(("src", "lo", "hi", "kind")):
            rec[f] = a[:, j]
        size = a[:, 2] - a[:, 1]
        if a.shape[1] == 5:
            rec["out_off"] = a[:, 4]
            off = int(max(0, (a[:, 4] + size).max()))
        else:
            ends = np.cumsum(size)
            rec["out_off"] = ends - size
            off = int(max(0, ends[-1]))
    else:  # mixed tuple lengths: offsets follow the sequence
        off = 0
        for i, q in enumerate(queries):
            src, lo, hi, kind = (int(x) for x in q[:4])
            o = int(q[4]) if len(q) > 4 else off
            rec[i] = (src, lo, hi, kind, o)
            off = max(off, o + hi - lo)
    arr = (Query * k).from_buffer(rec)
    arr.rec = rec
    return arr, off


def batch_workspace_bytes(num_queries: int, total_rows: int, total_arcs: int) -> int:
    return int(lib.lbg_batch_workspace_bytes(num_queries, total_rows, total_arcs))


def batch_solve(g: DeviceGraph, queries, out: torch.Tensor | None = None, total_arcs=None,
                workspace: Workspace | None = None, stats: bool = False, stream=None,
                graph: bool = False):
    """Solve many BFS (kind 0) / SSSP (kind 1) queries over a packed graph in
    one level-synchronous batch (see lbg_batch_solve; graph=True replays a
    cached HIP graph of 64 levels, lbg_batch_solve_graph).  ``queries``: sequence
    of (src, lo, hi, kind[, out_off]) with global node ids.  Returns the int32
    result tensor (BFS rows: levels; SSSP rows: uint32 bit patterns) or
    (tensor, stats)."""
    if g.weights is None:
        raise ValueError("batched solves need weights (BFS queries ignore them)")
    qarr, rows = batch_queries(queries)
    if total_arcs is None:
        if g.host_offsets is None:
            raise ValueError("total_arcs is required when the graph has no host offsets")
        ho = g.host_offsets
        total_arcs = int((ho[qarr.rec["hi"]] - ho[qarr.rec["lo"]]).sum()) if len(qarr) else 0
    out = _out(out, max(rows, 1), g.offsets.device)
    need = batch_workspace_bytes(len(qarr), out.numel(), total_arcs)
    if need == 0:
        raise LbgError(EINVAL, "invalid batch sizes")
    ws = _ws(workspace, need, g.offsets.device)
    st = Stats()
    fn = lib.lbg_batch_solve_graph if graph else lib.lbg_batch_solve
    rc = fn(_ptr(g.offsets), _ptr(g.cols), _ptr(g.weights), g.n, g.m, qarr,
                             len(qarr), _ptr(out), out.numel(), total_arcs, _ptr(ws), ws.numel(),
                             ctypes.byref(st) if stats else None, _stream(stream))
    _check(rc)
    return (out, st.as_dict()) if stats else out


class Engine:
    """Continuous-batching engine over one packed graph (lbg_engine_*).
    Rows of results live in ``self.rows`` (int32 tensor of max_rows); the
    caller assigns each query's row offset (admission is the caller's)."""

    def __init__(self, g: DeviceGraph, max_queries: int, max_rows: int, max_level_arcs: int,
                 stream=None):
        if g.weights is None:
            raise ValueError("the engine needs weights (BFS queries ignore them)")
        self.g = g
        self.max_queries = int(max_queries)
        self.max_rows = int(max_rows)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        need = int(lib.lbg_engine_workspace_bytes(max_queries, max_rows, max_level_arcs))
        if need == 0:
            raise LbgError(EINVAL, "invalid engine capacities")
        self.ws = torch.empty(need, dtype=torch.uint8, device=g.offsets.device)
        self.rows = torch.empty(max_rows, dtype=torch.int32, device=g.offsets.device)
        h = ctypes.c_void_p()
        _check(lib.lbg_engine_create(_ptr(g.offsets), _ptr(g.cols), _ptr(g.weights), g.n, g.m,
                                     max_queries, max_rows, max_level_arcs, _ptr(self.rows),
                                     _ptr(self.ws), need, _stream(self.stream), ctypes.byref(h)))
        self.h = h
        self._done = (ctypes.c_int32 * self.max_queries)()

    def submit(self, src: int, lo: int, hi: int, kind: int, out_off: int) -> int:
        q = Query(int(src), int(lo), int(hi), int(kind), int(out_off))
        slot = ctypes.c_int32(-1)
        rc = lib.lbg_engine_submit(self.h, ctypes.byref(q), ctypes.byref(slot))
        if rc == EBUSY:
            return -1
        _check(rc)
        return slot.value

    def step(self, levels: int = 1) -> list:
        """Run `levels` levels; returns the slots that finished."""
        n = ctypes.c_int32(0)
        _check(lib.lbg_engine_step(self.h, int(levels), ctypes.byref(n)))
        k = lib.lbg_engine_finished(self.h, self._done, self.max_queries)
        return [self._done[i] for i in range(k)]

    def release(self, slot: int) -> None:
        _check(lib.lbg_engine_release(self.h, int(slot)))

    def info(self) -> dict:
        st = Stats()
        running = ctypes.c_int32(0)
        level = ctypes.c_uint32(0)
        _check(lib.lbg_engine_info(self.h, ctypes.byref(st), ctypes.byref(running),
                                   ctypes.byref(level)))
        d = st.as_dict()
        d["running"] = running.value
        d["level"] = level.value
        return d

    def close(self) -> None:
        if getattr(self, "h", None):
            lib.lbg_engine_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def validate_csr(g: DeviceGraph, workspace: Workspace | None = None, stream=None) -> None:
    need = workspace_bytes(g.n, g.m, NODE, False)
    ws = _ws(workspace, need, g.offsets.device)
    _check(lib.lbg_validate_csr(_ptr(g.offsets), _ptr(g.cols), g.n, g.m, _ptr(ws), ws.numel(),
                                _stream(stream)))


def profile_enable(enable: bool = True, reset: bool = True) -> None:
    lib.lbg_profile_enable(int(enable), int(reset))


def profile_read(which) -> dict:
    """Expansion-kernel totals since the last reset: which = "bfs", "sssp",
    "batch" (one-level launches), "bfs_small" or "sssp_small" (launches of
    the single-workgroup small-frontier level loop); booleans select
    sssp/bfs."""
    idx = ({"bfs": 0, "sssp": 1, "batch": 2, "bfs_small": 3, "sssp_small": 4}[which]
           if isinstance(which, str) else int(bool(which)))
    p = Profile()
    lib.lbg_profile_read(idx, ctypes.byref(p))
    return p.as_dict()


def set_hier_mdt(mdt: int) -> None:
    """Fixed MDT of later LBG_HIER solves (0 = the histogram rule)."""
    _check(lib.lbg_set_hier_mdt(int(mdt)))


def get_hier_mdt() -> int:
    return int(lib.lbg_get_hier_mdt())


def hier_last_schedule(max_levels: int = 64, max_subs: int = 256):
    """(sizes, mdt) of this thread's last LBG_HIER solve: sizes[l][s] = the
    sublist size of sub-iteration s of level l (0 past the last), as a numpy
    int32 array of shape (levels, max_subs)."""
    import numpy as np

    buf = (ctypes.c_int32 * (max_levels * max_subs))()
    mdt = ctypes.c_int32(0)
    nl = int(lib.lbg_hier_last_schedule(buf, max_levels, max_subs, ctypes.byref(mdt)))
    arr = np.frombuffer(buf, dtype=np.int32).reshape(max_levels, max_subs)[:nl].copy()
    return arr, int(mdt.value)


def set_bins(mdt: int, t_wave: int, t_block: int) -> None:
    """Degree-bin parameters of 'binned' solves (see lbg_set_bins)."""
    _check(lib.lbg_set_bins(ctypes.byref(Bins(int(mdt), int(t_wave), int(t_block)))))


def get_bins() -> dict:
    b = Bins()
    lib.lbg_get_bins(ctypes.byref(b))
    return b.as_dict()


def degree_mdt(g: DeviceGraph, workspace: Workspace | None = None, stream=None) -> tuple:
    """(MDT, max out-degree) of the graph by the histogram rule of Section
    III-B, computed on the device (see lbg_degree_mdt)."""
    ws = _ws(workspace, workspace_bytes(g.n, g.m, NODE, False), g.offsets.device)
    mdt, mx = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib.lbg_degree_mdt(_ptr(g.offsets), g.n, g.m, _ptr(ws), ws.numel(), ctypes.byref(mdt),
                              ctypes.byref(mx), _stream(stream)))
    return mdt.value, mx.value


def autotune_bins(g: DeviceGraph, sources, workspace: Workspace | None = None, stream=None) -> dict:
    """Time 'binned' BFS (and SSSP if the graph has weights) from `sources`
    over candidate bin parameters and keep the fastest (lbg_autotune_bins)."""
    need = max(workspace_bytes(g.n, g.m, BINNED, False), workspace_bytes(g.n, g.m, BINNED, True))
    ws = _ws(workspace, need, g.offsets.device)
    src = (ctypes.c_int32 * len(sources))(*[int(x) for x in sources])
    out = torch.empty(g.n, dtype=torch.int32, device=g.offsets.device)
    best = Bins()
    _check(lib.lbg_autotune_bins(_ptr(g.offsets), _ptr(g.cols), _ptr(g.weights), g.n, g.m, src,
                                 len(sources), _ptr(out), _ptr(ws), ws.numel(), ctypes.byref(best),
                                 _stream(stream)))
    return best.as_dict()


def tile_edges() -> int:
    return int(lib.lbg_tile_edges())


def grid_blocks() -> int:
    return int(lib.lbg_grid_blocks())
