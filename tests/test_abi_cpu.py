"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, sizes workspaces by the documented formulas and rejects bad
arguments on the host before any launch."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbg.h")

lbgmod = pytest.importorskip("paper_1711_00231_amd.lbg",
                             reason="liblbg.so not built (run __graft_entry__.build())")
lib = lbgmod.lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbg_\w+)\s*\(", text)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert "lbg_bfs" in names and "lbg_sssp" in names
    raw = ctypes.CDLL(lbgmod.LIB_PATH)
    missing = [f for f in names if not hasattr(raw, f)]
    assert not missing, missing


def test_workspace_formulas():
    T = lbgmod.tile_edges()
    assert T > 0 and T % 256 == 0
    al = lambda x: (x + 255) // 256 * 256
    n, m = 1000, 123457
    ctl = al(128 + 8 * 128)
    words = (n + 31) // 32
    bfs_state = 3 * al(4 * words) + al(4 * words * 8)   # visited + 2 snapshots + per-XCD filters
    sssp_state = al(8 * n) + al(2 * n)              # packed (distance, iteration) + 16-bit filter
    # BFS, node-based / balanced: node state + 2 x (3 node arrays + tile marks)
    tiles = (m + T - 1) // T + 2
    exp_bfs = ctl + bfs_state + 2 * (3 * al(4 * n) + al(4 * tiles))
    assert lbgmod.workspace_bytes(n, m, "balanced", False) == exp_bfs
    assert lbgmod.workspace_bytes(n, m, "node", False) == exp_bfs
    assert lbgmod.workspace_bytes(n, m, "auto", False) == exp_bfs
    exp_sssp = ctl + sssp_state + 2 * (3 * al(4 * n) + al(4 * tiles))
    assert lbgmod.workspace_bytes(n, m, "balanced", True) == exp_sssp
    # edge-based: two worklists of m arc ids (the COO-scale cost, Section II-B)
    assert lbgmod.workspace_bytes(n, m, "edge", False) == ctl + bfs_state + 2 * al(4 * m)
    assert lbgmod.workspace_bytes(n, m, "edge", True) == ctl + sssp_state + 2 * al(4 * m)
    assert lbgmod.workspace_bytes(n, m, "edge_nochunk", True) == ctl + sssp_state + 2 * al(4 * m)
    # binned: split hubs add at most m / 64 entries per level
    cap = n + m // 64 + 1
    exp_binned = ctl + bfs_state + 2 * (3 * al(4 * cap) + al(4 * tiles))
    assert lbgmod.workspace_bytes(n, m, "binned", False) == exp_binned
    # hierarchical: two sublists of n worklist indices
    # (plus the sub-iteration trace: 64 levels x 256 sub-iterations)
    assert lbgmod.workspace_bytes(n, m, "hier", False) == exp_bfs + 2 * al(4 * n) + al(4 * 64 * 256)
    # destination-sliced: per buffer, 8 slice lists + the mixed list, each of
    # min(n, m) entries and its tile marks
    cap = min(n, m)
    exp_sliced = lambda state: ctl + state + 2 * (3 * al(4 * 9 * cap) + al(4 * 9 * tiles))
    assert lbgmod.workspace_bytes(n, m, "sliced", False) == exp_sliced(bfs_state)
    assert lbgmod.workspace_bytes(n, m, "sliced", True) == exp_sliced(sssp_state)
    assert lbgmod.workspace_bytes(n, 0, "sliced", True) == ctl + sssp_state + 2 * (3 * al(4 * 9) + al(4 * 9 * 2))
    # split graph: worklists of n + children entries (the bound C = m when
    # the child count is not given)
    exp_split = lambda c, state: ctl + state + 2 * (3 * al(4 * (n + c)) + al(4 * tiles))
    assert lbgmod.workspace_bytes(n, m, "split", False) == exp_split(m, bfs_state)
    for c in (0, 17, 5000, m):
        assert lbgmod.split_workspace_bytes(n, m, c, False) == exp_split(c, bfs_state)
        assert lbgmod.split_workspace_bytes(n, m, c, True) == exp_split(c, sssp_state)
    assert lbgmod.split_workspace_bytes(n, m, m + 1, False) == 0
    assert lbgmod.split_workspace_bytes(n, m, -1, False) == 0
    assert lbgmod.split_workspace_bytes(0, m, 0, False) == 0
    # CSR strategies stay O(n + m / tile); the edge one grows with m
    assert lbgmod.workspace_bytes(n, 50 * m, "balanced", False) < lbgmod.workspace_bytes(n, 50 * m, "edge", False) / 10
    # invalid arguments
    assert lbgmod.workspace_bytes(0, 10, "balanced", False) == 0
    assert lbgmod.workspace_bytes(10, -1, "balanced", False) == 0
    assert lbgmod.workspace_bytes(10, 2**31, "balanced", False) == 0
    assert lib.lbg_workspace_bytes(10, 10, 99, 0) == 0


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails a host check
WS = ctypes.c_void_p(0x10000)   # 256-byte aligned fake device address


def _bfs(n=10, m=20, src=0, offsets=FAKE, cols=FAKE, out=FAKE, ws=WS, ws_bytes=1 << 40,
         strategy=lbgmod.BALANCED, coo=None):
    return lib.lbg_bfs(offsets, cols, n, m, src, out, ws, ws_bytes, strategy, coo, None, None)


def _sssp(n=10, m=20, src=0, weights=FAKE, strategy=lbgmod.BALANCED, coo=None, ws_bytes=1 << 40):
    return lib.lbg_sssp(FAKE, FAKE, weights, n, m, src, FAKE, WS, ws_bytes, strategy, coo, None, None)


@pytest.mark.parametrize("kwargs, code", [
    (dict(n=0), lbgmod.EINVAL),
    (dict(n=-5), lbgmod.EINVAL),
    (dict(m=-1), lbgmod.ERANGE),
    (dict(m=2**31), lbgmod.ERANGE),
    (dict(src=10), lbgmod.ERANGE),
    (dict(src=-1), lbgmod.ERANGE),
    (dict(offsets=None), lbgmod.EINVAL),
    (dict(out=None), lbgmod.EINVAL),
    (dict(ws=None), lbgmod.EINVAL),
    (dict(cols=None), lbgmod.EINVAL),
    (dict(strategy=9), lbgmod.EINVAL),
    (dict(strategy=lbgmod.SLICED), lbgmod.EINVAL),        # only through lbg_bfs_sliced
    (dict(strategy=lbgmod.SPLIT), lbgmod.EINVAL),         # only through lbg_bfs_split
    (dict(strategy=-2), lbgmod.EINVAL),
    (dict(strategy=lbgmod.EDGE_NOCHUNK), lbgmod.EINVAL),  # no coo_src
    (dict(strategy=lbgmod.EDGE), lbgmod.EINVAL),          # no coo_src
    (dict(ws=ctypes.c_void_p(0x10010)), lbgmod.EINVAL),  # misaligned workspace
    (dict(ws_bytes=100), lbgmod.ENOMEM),
])
def test_bfs_argument_errors(kwargs, code):
    assert _bfs(**kwargs) == code
    assert lib.lbg_last_error().decode()


def test_sssp_argument_errors():
    assert _sssp(weights=None) == lbgmod.EINVAL
    assert _sssp(strategy=lbgmod.EDGE) == lbgmod.EINVAL
    assert _sssp(ws_bytes=16) == lbgmod.ENOMEM
    assert _sssp(src=99) == lbgmod.ERANGE
    assert "src" in lib.lbg_last_error().decode()


def test_sssp_noalloc_limits_on_the_host():
    """The no-allocation SSSP refuses, before touching a device, what its
    static scratch cannot hold and the strategies that need other inputs."""
    cap = lbgmod.NOALLOC_SCRATCH_BYTES

    def call(n, m, strategy=lbgmod.BALANCED):
        return lib.lbg_sssp_noalloc(FAKE, FAKE, FAKE, n, m, 0, FAKE, strategy, None, None)

    # R-MAT scale 20 fits, scale 22 does not
    assert lbgmod.workspace_bytes(1 << 20, 31_400_000, "balanced", True) <= cap
    assert lbgmod.workspace_bytes(1 << 22, 128_307_136, "balanced", True) > cap
    assert call(1 << 22, 128_307_136) == lbgmod.ENOMEM
    assert "maximum" in lib.lbg_last_error().decode()
    for s in (lbgmod.EDGE, lbgmod.EDGE_NOCHUNK, lbgmod.SLICED, lbgmod.SPLIT, 9, -1):
        assert call(100, 200, s) == lbgmod.EINVAL


def test_validate_csr_argument_errors():
    assert lib.lbg_validate_csr(FAKE, FAKE, 0, 5, WS, 1 << 20, None) == lbgmod.EINVAL
    assert lib.lbg_validate_csr(FAKE, FAKE, 5, -2, WS, 1 << 20, None) == lbgmod.ERANGE
    assert lib.lbg_validate_csr(None, FAKE, 5, 5, WS, 1 << 20, None) == lbgmod.EINVAL
    assert lib.lbg_validate_csr(FAKE, FAKE, 5, 5, WS, 8, None) == lbgmod.ENOMEM


def test_batch_workspace_and_argument_errors():
    T = 256  # batched tile
    al = lambda x: (x + 255) // 256 * 256
    Q, rows, arcs = 7, 5000, 123457
    tiles = (arcs + T - 1) // T + 2
    exp = (al(128 + 8 * 128) + al(32 * Q) + al(8 * rows) + al(4 * ((rows + 31) // 32)) + al(2 * rows)
           + 2 * (4 * al(4 * rows) + al(4 * tiles)))
    assert lbgmod.batch_workspace_bytes(Q, rows, arcs) == exp
    assert lbgmod.batch_workspace_bytes(0, rows, arcs) == 0
    assert lbgmod.batch_workspace_bytes(Q, 2**31, arcs) == 0
    assert lbgmod.batch_workspace_bytes(Q, rows, 2**32) == 0

    def solve(queries, n=100, m=50, rows=1000, arcs=100, ws_bytes=1 << 40):
        arr, _ = lbgmod.batch_queries(queries)
        return lib.lbg_batch_solve(FAKE, FAKE, FAKE, n, m, arr, len(arr), FAKE, rows, arcs, WS,
                                   ws_bytes, None, None)

    ok = (5, 0, 10, 0, 0)
    assert solve([(11, 0, 10, 0, 0)]) == lbgmod.ERANGE       # src outside its instance
    assert solve([(5, 0, 101, 0, 0)]) == lbgmod.ERANGE       # instance beyond n
    assert solve([(5, 6, 6, 0, 0)]) == lbgmod.ERANGE         # empty instance
    assert solve([(5, 0, 10, 2, 0)]) == lbgmod.EINVAL        # unknown kind
    assert solve([ok, (5, 0, 10, 1, 995)]) == lbgmod.ERANGE  # row beyond total_rows
    assert solve([ok], ws_bytes=64) == lbgmod.ENOMEM
    assert solve([ok], n=0) == lbgmod.EINVAL
    assert lib.lbg_batch_solve(FAKE, FAKE, FAKE, 100, 50, None, 0, FAKE, 10, 10, WS, 1 << 40,
                               None, None) == lbgmod.EINVAL


def test_bins_validation_and_round_trip():
    saved = lbgmod.get_bins()
    for bad in ((10, 8, 16), (-1, 8, 16), (128, 64, 32), (128, -1, 16)):
        with pytest.raises(lbgmod.LbgError):
            lbgmod.set_bins(*bad)
    assert lbgmod.get_bins() == saved  # a rejected call changes nothing
    lbgmod.set_bins(0, 8, 8)
    assert lbgmod.get_bins() == {"mdt": 0, "t_wave": 8, "t_block": 8}
    lbgmod.set_bins(**saved)
    assert lbgmod.get_bins() == saved
    out = ctypes.c_int32(0)
    assert lib.lbg_degree_mdt(FAKE, 0, 5, WS, 1 << 20, ctypes.byref(out), None, None) == lbgmod.EINVAL
    assert lib.lbg_degree_mdt(FAKE, 5, 5, WS, 8, ctypes.byref(out), None, None) == lbgmod.ENOMEM


def test_slice_min_setting():
    saved = lbgmod.get_slice_min()
    with pytest.raises(lbgmod.LbgError):
        lbgmod.set_slice_min(-1)
    assert lbgmod.get_slice_min() == saved
    lbgmod.set_slice_min(0)
    assert lbgmod.get_slice_min() == 0
    lbgmod.set_slice_min(2**31 - 1)
    assert lbgmod.get_slice_min() == 2**31 - 1
    lbgmod.set_slice_min(saved)


def test_addressing_setting():
    assert lbgmod.get_addressing() == 0
    for bad in (-1, 2, 64):
        with pytest.raises(lbgmod.LbgError):
            lbgmod.set_addressing(bad)
        assert lbgmod.get_addressing() == 0
    lbgmod.set_addressing(1)
    assert lbgmod.get_addressing() == 1
    lbgmod.set_addressing(0)
    assert lbgmod.get_addressing() == 0


def test_slice_sizes():
    for n, S in ((1, 64), (8, 64), (512, 64), (513, 128), (4194304, 524288), (1000, 128)):
        assert lbgmod.slice_nodes(n) == S
        assert 8 * S >= n and S % 64 == 0
    assert lbgmod.slice_nodes(0) == 0


def test_sliced_argument_errors():
    def grp(n=10, m=20, offsets=FAKE, cols=FAKE, w=FAKE, so=FAKE, cout=FAKE, wout=FAKE):
        return lib.lbg_slice_graph(offsets, cols, w, n, m, so, cout, wout, None)

    assert grp(n=0) == lbgmod.EINVAL
    assert grp(m=-1) == lbgmod.ERANGE
    assert grp(m=2**31) == lbgmod.ERANGE
    assert grp(offsets=None) == lbgmod.EINVAL
    assert grp(so=None) == lbgmod.EINVAL
    assert grp(cout=None) == lbgmod.EINVAL
    assert grp(wout=None) == lbgmod.EINVAL   # weights without weights_out
    assert grp(w=None) == lbgmod.EINVAL      # weights_out without weights
    ws = 1 << 40
    assert lib.lbg_bfs_sliced(FAKE, FAKE, FAKE, 10, 20, 10, FAKE, WS, ws, None, None) == lbgmod.ERANGE
    assert lib.lbg_bfs_sliced(FAKE, FAKE, FAKE, 0, 20, 0, FAKE, WS, ws, None, None) == lbgmod.EINVAL
    assert lib.lbg_bfs_sliced(FAKE, FAKE, FAKE, 10, 20, 0, FAKE, WS, 64, None, None) == lbgmod.ENOMEM
    assert lib.lbg_bfs_sliced(FAKE, None, FAKE, 10, 20, 0, FAKE, WS, ws, None, None) == lbgmod.EINVAL
    assert lib.lbg_sssp_sliced(FAKE, FAKE, FAKE, None, 10, 20, 0, FAKE, WS, ws, None, None) == lbgmod.EINVAL
    assert lib.lbg_sssp_sliced(None, FAKE, FAKE, FAKE, 10, 20, 0, FAKE, WS, ws, None, None) == lbgmod.EINVAL


def test_packed_argument_errors():
    wb = ctypes.c_int32(0)
    pk = lambda n=10, m=20, cols=FAKE, w=FAKE, out=FAKE, wbo=ctypes.byref(wb), ws=WS, wsb=1 << 20: \
        lib.lbg_pack_arcs(cols, w, n, m, out, wbo, ws, wsb, None)
    assert pk(n=0) == lbgmod.EINVAL
    assert pk(m=-1) == lbgmod.ERANGE
    assert pk(cols=None) == lbgmod.EINVAL
    assert pk(w=None) == lbgmod.EINVAL
    assert pk(out=None) == lbgmod.EINVAL
    assert pk(wbo=None) == lbgmod.EINVAL
    assert pk(ws=ctypes.c_void_p(0x10010)) == lbgmod.EINVAL
    assert pk(wsb=64) == lbgmod.ENOMEM
    sp = lambda n=10, m=20, arcs=FAKE, wbits=4, src=0, wsb=1 << 40: \
        lib.lbg_sssp_packed(FAKE, arcs, wbits, n, m, src, FAKE, WS, wsb, None, None)
    assert sp(wbits=32) == lbgmod.ERANGE
    assert sp(wbits=-1) == lbgmod.ERANGE
    assert sp(n=1 << 29, wbits=4) == lbgmod.ERANGE   # 29 id bits + 4 weight bits
    assert sp(arcs=None) == lbgmod.EINVAL
    assert sp(src=10) == lbgmod.ERANGE
    assert sp(wsb=16) == lbgmod.ENOMEM


def test_split_scratch_and_argument_errors():
    al = lambda x: (x + 255) // 256 * 256
    for n in (1, 4096, 4097, 10**6, 2**31 - 1):
        assert lib.lbg_split_scratch_bytes(n) == al(12 * ((n + 4095) // 4096 + 1))
    assert lib.lbg_split_scratch_bytes(0) == 0
    c = ctypes.c_int64(-1)
    cnt = lambda n=10, m=20, mdt=4, offsets=FAKE, co=ctypes.byref(c), sc=WS, scb=64: \
        lib.lbg_split_count(offsets, n, m, mdt, co, sc, scb, None)
    assert cnt(n=0) == lbgmod.EINVAL
    assert cnt(m=-1) == lbgmod.ERANGE
    assert cnt(m=2**31) == lbgmod.ERANGE
    assert cnt(mdt=-1) == lbgmod.EINVAL
    assert cnt(offsets=None) == lbgmod.EINVAL
    assert cnt(co=None) == lbgmod.EINVAL
    assert cnt(sc=None) == lbgmod.EINVAL
    assert cnt(sc=ctypes.c_void_p(0x10010)) == lbgmod.EINVAL
    assert cnt(scb=16) == lbgmod.ENOMEM        # 12 bytes per 4096 nodes + the totals
    assert c.value == -1                       # untouched on error

    def grp(n=10, m=20, offsets=FAKE, cols=FAKE, w=FAKE, so=FAKE, cb=FAKE, cout=FAKE, wout=FAKE, scb=16):
        return lib.lbg_split_graph(offsets, cols, w, n, m, 4, 3, so, cb, cout, wout, WS, scb, None)

    assert grp(so=None) == lbgmod.EINVAL
    assert grp(cb=None) == lbgmod.EINVAL
    assert grp(cols=None) == lbgmod.EINVAL
    assert grp(cout=None) == lbgmod.EINVAL
    assert grp(wout=None) == lbgmod.EINVAL     # weights without weights_out
    assert grp(w=None) == lbgmod.EINVAL        # weights_out without weights
    assert grp(n=0) == lbgmod.EINVAL
    assert grp(scb=16) == lbgmod.ENOMEM

    ws = 1 << 40
    bs = lambda n=10, children=3, m=20, src=0, cb=FAKE, wsb=ws: \
        lib.lbg_bfs_split(FAKE, cb, FAKE, n, children, m, src, FAKE, WS, wsb, None, None)
    assert bs(cb=None) == lbgmod.EINVAL
    assert bs(children=21) == lbgmod.ERANGE    # more children than arcs
    assert bs(children=-1) == lbgmod.ERANGE
    assert bs(src=10) == lbgmod.ERANGE
    assert bs(n=0) == lbgmod.EINVAL
    assert bs(wsb=64) == lbgmod.ENOMEM
    assert "children" in (bs(children=21), lib.lbg_last_error().decode())[1]
    ss = lambda w=FAKE, cb=FAKE, wsb=ws: \
        lib.lbg_sssp_split(FAKE, cb, FAKE, w, 10, 3, 20, 0, FAKE, WS, wsb, None, None)
    assert ss(w=None) == lbgmod.EINVAL
    assert ss(cb=None) == lbgmod.EINVAL
    assert ss(wsb=64) == lbgmod.ENOMEM


def test_order_scratch_and_argument_errors():
    al = lambda x: (x + 255) // 256 * 256
    for n in (1, 4096, 4097, 10**6):
        nb = (n + 4095) // 4096
        assert lib.lbg_order_scratch_bytes(n) == al(4 * (32 * nb + 1)) + al(4 * (nb + 1)) + al(4 * n)
    assert lib.lbg_order_scratch_bytes(0) == 0

    def og(n=10, m=20, offsets=FAKE, cols=FAKE, w=FAKE, oo=FAKE, oc=FAKE, ow=FAKE, nid=FAKE, sc=WS, scb=16):
        return lib.lbg_order_graph(offsets, cols, w, n, m, oo, oc, ow, nid, sc, scb, None)

    assert og(n=0) == lbgmod.EINVAL
    assert og(m=-1) == lbgmod.ERANGE
    assert og(m=2**31) == lbgmod.ERANGE
    assert og(offsets=None) == lbgmod.EINVAL
    assert og(oo=None) == lbgmod.EINVAL
    assert og(nid=None) == lbgmod.EINVAL
    assert og(cols=None) == lbgmod.EINVAL
    assert og(oc=None) == lbgmod.EINVAL
    assert og(ow=None) == lbgmod.EINVAL     # weights without order_weights
    assert og(w=None) == lbgmod.EINVAL      # order_weights without weights
    assert og(sc=None) == lbgmod.EINVAL
    assert og(sc=ctypes.c_void_p(0x10010)) == lbgmod.EINVAL
    assert og(scb=16) == lbgmod.ENOMEM      # every other argument is valid: fails on the size

    so = lambda n=10, m=20, src=0, nid=FAKE, w=FAKE, wsb=1 << 40: \
        lib.lbg_sssp_ordered(FAKE, FAKE, w, nid, n, m, src, FAKE, WS, wsb, None, None)
    assert so(nid=None) == lbgmod.EINVAL
    assert so(w=None) == lbgmod.EINVAL
    assert so(src=10) == lbgmod.ERANGE
    assert so(n=0) == lbgmod.EINVAL
    assert so(wsb=64) == lbgmod.ENOMEM


def test_header_is_plain_c(tmp_path):
    """include/lbg.h is a C header: it compiles as strict C99 with no
    warnings (no C++ or torch types in the boundary)."""
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    src = tmp_path / "h.c"
    src.write_text('#include "lbg.h"\nint main(void) { return (int)sizeof(lbg_stats) == 48 ? 0 : 1; }\n')
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-I", os.path.join(ROOT, "include"), "-o", str(tmp_path / "h"), str(src)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert subprocess.run([str(tmp_path / "h")], timeout=60).returncode == 0
