"""Bounds-checked host emulation of the balanced one-level kernel's index
arithmetic (tests/c/expand_emul.cpp): tile marks and their look-ahead,
staging of a tile's entries, the slot-to-entry map, per-XCD filter words,
the push path and the worklist/tile-mark capacities, for BFS and SSSP with
tiles of 8 and 16 arcs per lane (the shipped BFS tile is 16, SSSP 8; BFS at 8
is a size the library does not ship).  Each run must touch no array outside
its allocated size, never read an LDS slot staged for another tile, raise no
device guard, and give the oracle's result."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import graphgen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
O = oracle.get()
MIN_TILE = 512  # the single-solve tile marks are sized by the SSSP tile (64 x 8 arcs)
NEVER = 0xFFFFFFFF  # BFS scan mode off


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    so = str(tmp_path_factory.mktemp("emu") / "libexpand_emul.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-Wall", "-Wextra", "-Werror",
                    os.path.join(ROOT, "tests", "c", "expand_emul.cpp"), "-o", so], check=True)
    lib = ctypes.CDLL(so)
    vp = ctypes.c_void_p
    u32 = ctypes.c_uint32
    lib.emu_solve.argtypes = [vp, vp, vp, u32, u32, ctypes.c_int32, ctypes.c_int, u32, u32, u32, u32, vp, vp,
                              ctypes.c_char_p, ctypes.c_int]

    def run(g, src, sssp, items, grid, scan_min=NEVER):
        out = np.empty(g.n, dtype=np.uint32 if sssp else np.int32)
        st = np.zeros(7, dtype=np.int64)
        msg = ctypes.create_string_buffer(512)
        off = np.ascontiguousarray(g.offsets, dtype=np.int32)
        cols = np.ascontiguousarray(g.cols, dtype=np.int32)
        w = np.ascontiguousarray(g.weights if g.weights is not None else np.ones(g.m), dtype=np.uint32)
        lib.emu_solve(off.ctypes.data, cols.ctypes.data, w.ctypes.data, g.n, g.m, int(src), int(sssp), items,
                      MIN_TILE, grid, scan_min, out.ctypes.data, st.ctypes.data, msg, 512)
        return out, st, msg.value.decode()

    return run


def _check(emu, g, src, sssp, items, grid, scan_min=NEVER):
    out, st, msg = emu(g, src, sssp, items, grid, scan_min)
    assert st[0] == 0, f"out-of-bounds access: {msg}"
    assert st[1] == 0, "an LDS slot staged for another tile was read"
    assert st[2] == 0, f"device guard flags 0x{st[2]:x} (0x100: a tile dealt twice or never)"
    exp = O.dijkstra(g.offsets, g.cols, g.weights, src) if sssp else O.bfs(g.offsets, g.cols, src)
    assert np.array_equal(out, exp)
    return st


def _hub_graph():
    """Level 1 holds three hubs (degrees 300,000, exactly 8 x 1024 and
    1024 x 7 + 1) among 5,000 nodes of degree 1..40, so hub entries span many
    tiles of either size and tile boundaries fall on, just before and just
    after entry boundaries."""
    rng = np.random.default_rng(11)
    n = 400_000
    hubs = [1, 2, 3]
    hub_deg = [300_000, 8 * 1024, 7 * 1024 + 1]
    small = np.arange(4, 5004)
    src = [np.zeros(len(hubs) + small.size, dtype=np.int64)]
    dst = [np.r_[hubs, small]]
    for h, d in zip(hubs, hub_deg):
        src.append(np.full(d, h))
        dst.append(rng.integers(5004, n, d))
    for u in small:
        d = int(rng.integers(1, 41))
        src.append(np.full(d, u))
        dst.append(rng.integers(5004, n, d))
    src, dst = np.concatenate(src), np.concatenate(dst)
    w = rng.integers(1, 256, src.size)
    return graphgen.from_edges(n, src, dst, w, "hubs")


@pytest.mark.parametrize("items", [8, 16])
@pytest.mark.parametrize("sssp", [False, True])
def test_small_graphs(emu, items, sssp):
    for g in (graphgen.uniform(14), graphgen.rmat(16), graphgen.grid(96)):
        s = int(graphgen.sources(g, 1, graphgen.FAMILY_RMAT)[0])
        # one workgroup, an odd grid, the smallest grids that take the last
        # eighth of a level's tiles from the per-XCD counters, a resident grid
        for grid in (1, 7, 8, 9, 512):
            _check(emu, g, s, sssp, items, grid)


@pytest.mark.parametrize("items", [8, 16])
@pytest.mark.parametrize("sssp", [False, True])
def test_hub_heavy_frontier(emu, items, sssp):
    g = _hub_graph()
    for grid in (3, 8, 768):
        st = _check(emu, g, 0, sssp, items, grid)
        assert st[5] >= 300_000  # the hubs' level was expanded in tiles


def test_degenerate_graphs(emu):
    one = graphgen.from_edges(1, np.zeros(0), np.zeros(0), None, "single")
    star = graphgen.from_edges(1025, np.zeros(1024), np.arange(1, 1025), None, "star-1024")
    for g in (one, star):
        for items in (8, 16):
            _check(emu, g, 0, False, items, 5)


@pytest.fixture(scope="module")
def rmat22():
    g = graphgen.rmat(22)
    return g, graphgen.sources(g, 64, graphgen.FAMILY_RMAT)


@pytest.mark.parametrize("sssp, items", [(False, 8), (False, 16), (True, 8)])
def test_rmat22_levels(emu, rmat22, sssp, items):
    """R-MAT scale 22 at its real level sizes (BFS: 8 levels, the largest
    with 1.7 M entries and 113 M edges), in a resident-size grid."""
    g, srcs = rmat22
    st = _check(emu, g, int(srcs[0]), sssp, items, 768)
    assert st[5] > 100_000_000


@pytest.mark.parametrize("rule", ["every", "quarter_n"])
def test_bfs_scan_levels(emu, rule):
    """BFS levels expanded in scan mode (plain level stores, no claims or
    pushes) and the compaction that builds the next worklist in node order:
    every level (threshold 0) or the library's default, levels of at least
    n / 4 arcs, mixed with push-mode levels; on the three families, the hub
    frontier and one-node / star graphs, grids from one workgroup to a
    resident one (the compaction's grid is one workgroup per 4096 nodes, at
    most the expansion's)."""
    graphs = [graphgen.uniform(14), graphgen.rmat(16), graphgen.grid(96), _hub_graph(),
              graphgen.from_edges(1, np.zeros(0), np.zeros(0), None, "single"),
              graphgen.from_edges(1025, np.zeros(1024), np.arange(1, 1025), None, "star-1024")]
    for g in graphs:
        s = 0 if g.n <= 1025 or g.name == "hubs" else int(graphgen.sources(g, 1, graphgen.FAMILY_RMAT)[0])
        scan_min = 0 if rule == "every" else max(1, g.n // 4)
        for grid in (1, 9, 768):
            st = _check(emu, g, s, False, 16, grid, scan_min)
            if rule == "every" and g.m:
                assert st[6] == st[3]  # every level ran in scan mode
            if rule == "quarter_n" and g.name == "hubs":
                assert 0 < st[6] < st[3]  # the hubs' level scanned, the others pushed


def test_rmat22_scan_levels(emu, rmat22):
    """R-MAT scale 22 with the default threshold (levels of >= n / 4 arcs
    scan)."""
    g, srcs = rmat22
    st = _check(emu, g, int(srcs[0]), False, 16, 768, g.n // 4)
    assert st[6] >= 2
