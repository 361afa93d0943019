"""GPU parity: BFS levels and SSSP distances from the HIP library (called
through the C ABI binding) against the CPU oracle, bit for bit, for every
work-assignment strategy, on edge cases, on inputs spanning many tiles with a
ragged tail, and at the full sizes of the workloads the benchmark times."""
import numpy as np
import pytest

import graphgen
import oracle
import pins

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
from paper_1711_00231_amd import lbg  # noqa: E402  (fails loudly if liblbg.so is missing)

STRATS = ["node", "edge", "balanced", "binned", "hier", "edge_nochunk", "sliced", "split"]
FULL_STRATS = ["node", "edge", "balanced", "binned", "hier", "sliced", "split"]  # the ablation is too slow at full size
O = oracle.get()


def _dev(g):
    return lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights)


def _gpu_bfs(dg, s, strat, **kw):
    out = lbg.bfs(dg, int(s), strategy=strat, **kw)
    if isinstance(out, tuple):
        return out[0].cpu().numpy(), out[1]
    return out.cpu().numpy()


def _gpu_sssp(dg, s, strat, **kw):
    out = lbg.sssp(dg, int(s), strategy=strat, **kw)
    if isinstance(out, tuple):
        return out[0].cpu().numpy().view(np.uint32), out[1]
    return out.cpu().numpy().view(np.uint32)


def _check(g, dg, srcs, strat):
    for s in srcs:
        exp_l = O.bfs(g.offsets, g.cols, s)
        got_l = _gpu_bfs(dg, s, strat)
        assert np.array_equal(got_l, exp_l), f"{g.name} bfs src={s} strat={strat}: " \
            f"{np.count_nonzero(got_l != exp_l)} mismatches"
        exp_d = O.dijkstra(g.offsets, g.cols, g.weights, s)
        got_d = _gpu_sssp(dg, s, strat)
        assert np.array_equal(got_d, exp_d), f"{g.name} sssp src={s} strat={strat}: " \
            f"{np.count_nonzero(got_d != exp_d)} mismatches"


# ------------------------------------------------------------- edge cases --
@pytest.mark.parametrize("strat", STRATS)
def test_tiny_random_graphs(strat):
    for g, s in pins.tiny_graphs(count=40, seed=21):
        _check(g, _dev(g), [s], strat)


@pytest.mark.parametrize("strat", STRATS)
def test_degenerate_graphs(strat):
    cases = [
        graphgen.from_edges(1, [], [], [], "single-node"),
        graphgen.from_edges(5, [1, 2], [2, 3], [4, 5], "isolated-source"),  # src 0 has no arcs
        graphgen.from_edges(3, [0, 0, 0, 1], [0, 1, 1, 1], [3, 7, 2, 0], "loops-and-dups"),
        graphgen.from_edges(4, [0, 1, 2], [1, 2, 3], [0, 0, 0], "zero-weights"),
        pins.path_graph(3000, np.full(2999, 7)),  # long chain: 3000 levels, many level batches
    ]
    for g in cases:
        _check(g, _dev(g), [0], strat)


@pytest.mark.parametrize("strat", STRATS)
def test_hub_spanning_many_tiles(strat):
    # one node with far more arcs than a tile, a second medium hub, a tail
    T = lbg.tile_edges()
    rng = np.random.default_rng(5)
    n = 20000
    hub = rng.integers(1, n, 7 * T + 13)
    med = rng.integers(1, n, T + 1)
    tail_src = rng.integers(1, n, 30000)
    tail_dst = rng.integers(0, n, 30000)
    src = np.concatenate([np.zeros(hub.size), np.full(med.size, 1), tail_src])
    dst = np.concatenate([hub, med, tail_dst])
    w = rng.integers(1, 50, src.size)
    g = graphgen.from_edges(n, src, dst, w, "hub")
    _check(g, _dev(g), [0, 1, 17], strat)


# ------------------------------------------------- several tiles, ragged --
@pytest.mark.parametrize("strat", STRATS)
def test_uniform_config(strat):
    """n = 2^14, 8 out-arcs per node, weights U[1,100], source 0."""
    g = graphgen.uniform(14)
    _check(g, _dev(g), [0, 1234], strat)


@pytest.mark.parametrize("strat", STRATS)
def test_rmat_small(strat):
    g = graphgen.rmat(15)
    srcs = graphgen.sources(g, 3, graphgen.FAMILY_RMAT)
    _check(g, _dev(g), srcs, strat)


@pytest.mark.parametrize("strat", STRATS)
def test_grid_small(strat):
    g = graphgen.grid(96)
    h = graphgen.grid(64, shortcut_frac=0)
    _check(g, _dev(g), [0, 4000], strat)
    _check(h, _dev(h), [0], strat)


def _barbell(path_len, n_mid, k_mid, salt):
    """A path, a dense uniform block, another path (all arcs both ways): the
    frontier is tiny for path_len levels, explodes inside the block, then is
    tiny again, so a solve switches between the small-frontier kernel and
    one-level launches and back."""
    blk = graphgen.uniform(n=n_mid, k=k_mid, wlo=1, whi=9, salt=salt)
    P = path_len
    n = 2 * P + n_mid
    src = [np.arange(P - 1), P + np.repeat(np.arange(n_mid), blk.degrees), P + n_mid + np.arange(P - 1),
           np.array([P - 1, P + n_mid - 1])]
    dst = [np.arange(1, P), P + blk.cols.astype(np.int64), P + n_mid + np.arange(1, P),
           np.array([P, P + n_mid])]
    w = [np.full(P - 1, 3), blk.weights.astype(np.int64), np.full(P - 1, 5), np.array([2, 4])]
    s_all, d_all, w_all = np.concatenate(src), np.concatenate(dst), np.concatenate(w)
    return graphgen.from_edges(n, np.concatenate([s_all, d_all]), np.concatenate([d_all, s_all]),
                               np.concatenate([w_all, w_all]), "barbell")


def test_small_frontier_switching():
    """Balanced solves run small levels in the single-workgroup kernel and
    large ones as one-level launches; results and work counters must not
    depend on where the switches fall."""
    g = _barbell(400, 20000, 48, salt=5)
    dg = _dev(g)
    exp_l = O.bfs(g.offsets, g.cols, 0)
    exp_d = O.dijkstra(g.offsets, g.cols, g.weights, 0)
    reached = exp_l != pins.BFS_INF
    lbg.profile_enable(True, reset=True)
    lv, st = _gpu_bfs(dg, 0, "balanced", stats=True)
    d, st_d = _gpu_sssp(dg, 0, "balanced", stats=True)
    lbg.profile_enable(False, reset=False)
    assert np.array_equal(lv, exp_l)
    assert np.array_equal(d, exp_d)
    one, small = lbg.profile_read("bfs"), lbg.profile_read("bfs_small")
    assert st["levels"] == int(exp_l[reached].max()) + 1
    assert one["frontier_entries"] + small["frontier_entries"] == st["frontier_entries"]
    assert one["edges_scanned"] + small["edges_scanned"] == st["edges_scanned"] == g.reached_arcs(reached)
    assert one["updates"] + small["updates"] == st["updates"] == int(reached.sum()) - 1
    # path, block, path: small -> one-level -> small at least
    assert small["launches"] >= 2 and one["launches"] >= 1
    assert lbg.profile_read("sssp_small")["launches"] >= 2
    # a chain long enough that almost every level runs on the device
    h = pins.path_graph(5000, np.arange(1, 5000) % 7)
    _check(h, _dev(h), [0, 2500], "balanced")


def _chain_of_blocks(path_len, n_mid, k_mid, blocks, salt):
    """path, block, path, block, ..., path (all arcs both ways): big levels
    inside each block, tiny ones along each path."""
    P = path_len
    parts_s, parts_d, parts_w = [], [], []
    base = 0
    for b in range(blocks + 1):
        # path of P nodes starting at base, joined to the previous block's last node
        parts_s.append(base + np.arange(P - 1)); parts_d.append(base + np.arange(1, P))
        parts_w.append(np.full(P - 1, 3 + b))
        if b:
            parts_s.append(np.array([base - 1])); parts_d.append(np.array([base])); parts_w.append(np.array([2]))
        base += P
        if b == blocks:
            break
        blk = graphgen.uniform(n=n_mid, k=k_mid, wlo=1, whi=9, salt=salt + b)
        parts_s.append(np.array([base - 1])); parts_d.append(np.array([base])); parts_w.append(np.array([2]))
        parts_s.append(base + np.repeat(np.arange(n_mid), blk.degrees))
        parts_d.append(base + blk.cols.astype(np.int64)); parts_w.append(blk.weights.astype(np.int64))
        base += n_mid
    s_all, d_all, w_all = (np.concatenate(x) for x in (parts_s, parts_d, parts_w))
    return graphgen.from_edges(base, np.concatenate([s_all, d_all]), np.concatenate([d_all, s_all]),
                               np.concatenate([w_all, w_all]), "blocks")


def test_tile_counters_across_small_frontier_phases():
    """Levels big enough for the dynamic part of the tile deal (more tiles
    than wavefronts) inside the second of two blocks, reached after a
    small-frontier phase that itself followed big levels: the per-XCD tile
    counters those levels use must have been cleared by the small-frontier
    kernel.  BFS (with scan levels) and SSSP equal the oracle."""
    g = _chain_of_blocks(300, 200_000, 16, 2, salt=41)
    dg = _dev(g)
    exp_l = O.bfs(g.offsets, g.cols, 0)
    exp_d = O.dijkstra(g.offsets, g.cols, g.weights, 0)
    # the big levels of the second block deal tiles dynamically
    deg = g.degrees
    second = np.arange(g.n) >= 300 + 200_000 + 300
    lv2 = exp_l[second & (exp_l != pins.BFS_INF)]
    arcs = np.bincount(lv2, weights=deg[second & (exp_l != pins.BFS_INF)])
    waves = lbg.grid_blocks() * 4
    assert arcs.max() > waves * 1024  # the BFS tile: 64 lanes x 16 arcs
    lbg.profile_enable(True, reset=True)
    lv = _gpu_bfs(dg, 0, "balanced")
    d = _gpu_sssp(dg, 0, "balanced")
    lbg.profile_enable(False, reset=False)
    assert np.array_equal(lv, exp_l)
    assert np.array_equal(d, exp_d)
    assert lbg.profile_read("bfs_small")["launches"] >= 2 and lbg.profile_read("sssp_small")["launches"] >= 2


def test_degree_mdt_matches_oracle():
    """The device MDT (Section III-B histogram rule) equals the oracle's on
    skewed, uniform and grid graphs (an integer: compared exactly)."""
    for g in (graphgen.rmat(16, salt=3), graphgen.uniform(12, k=5, salt=4), graphgen.grid(70),
              pins.path_graph(100, np.ones(99)), graphgen.from_edges(4, [], [], [], "no-arcs")):
        mdt, mx = lbg.degree_mdt(_dev(g))
        assert mx == int(g.degrees.max())
        assert mdt == O.mdt(g.offsets)[0], g.name


@pytest.mark.parametrize("bins", [(64, 0, 64), (64, 63, 64), (0, 8, 32), (16384, 64, 4096)])
def test_binned_bin_parameters(bins):
    """Results do not depend on the split size or the bin thresholds: heavy
    splitting (every node above 64 arcs cut into pieces), all-wavefront,
    no splitting, and coarse bins."""
    saved = lbg.get_bins()
    try:
        lbg.set_bins(*bins)
        g = graphgen.rmat(15)
        _check(g, _dev(g), graphgen.sources(g, 2, graphgen.FAMILY_RMAT), "binned")
        h = graphgen.uniform(13, k=9, salt=8)
        _check(h, _dev(h), [0], "binned")
    finally:
        lbg.set_bins(**saved)


def test_autotune_bins_keeps_results():
    saved = lbg.get_bins()
    try:
        g = graphgen.rmat(14)
        dg = _dev(g)
        srcs = graphgen.sources(g, 2, graphgen.FAMILY_RMAT)
        best = lbg.autotune_bins(dg, srcs)
        assert best == lbg.get_bins()
        assert best["mdt"] == 0 or best["mdt"] >= 64
        assert 0 <= best["t_wave"] <= best["t_block"]
        _check(g, dg, srcs, "binned")
    finally:
        lbg.set_bins(**saved)


def test_tuned_bins_cache_round_trip(tmp_path):
    """A cache miss tunes on the device and stores the result; a later hit
    sets the same parameters without tuning; results stay the oracle's."""
    from paper_1711_00231_amd import tuning

    saved = lbg.get_bins()
    try:
        g = graphgen.rmat(13)
        dg = _dev(g)
        srcs = graphgen.sources(g, 2, graphgen.FAMILY_RMAT)
        cache = tuning.BinsCache(str(tmp_path / "bins.json"))
        best, hit = tuning.tuned_bins(dg, srcs, "rmat", cache)
        assert not hit and lbg.get_bins() == best
        assert cache.get(tuning.cache_key("rmat", g.n, g.m, tuning.device_arch(dg.offsets.device))) == best
        lbg.set_bins(0, 0, 0)
        again, hit = tuning.tuned_bins(dg, srcs, "rmat", cache,
                                       tune=lambda *a: pytest.fail("tuned on a cache hit"))
        assert hit and again == best and lbg.get_bins() == best
        _check(g, dg, srcs, "binned")
    finally:
        lbg.set_bins(**saved)


@pytest.mark.parametrize("smin", [0, 1, 7, 2**31 - 1])
def test_sliced_thresholds(smin):
    """Every node split by slice (0, 1), small nodes mixed (7), no node split
    (INT32_MAX): the same results."""
    saved = lbg.get_slice_min()
    try:
        lbg.set_slice_min(smin)
        g = graphgen.rmat(14)
        _check(g, _dev(g), graphgen.sources(g, 2, graphgen.FAMILY_RMAT), "sliced")
        for gg, s in pins.tiny_graphs(count=10, seed=5):
            _check(gg, _dev(gg), [s], "sliced")
        h = graphgen.grid(48)
        _check(h, _dev(h), [0], "sliced")
    finally:
        lbg.set_slice_min(saved)


def _packed_cases():
    rng = np.random.default_rng(11)
    n = 20000
    hub_src = np.concatenate([np.zeros(7 * 512 + 13, np.int64), rng.integers(1, n, 30000)])
    hub = graphgen.from_edges(n, hub_src, rng.integers(0, n, hub_src.size), rng.integers(1, 50, hub_src.size), "hub")
    return [
        (graphgen.from_edges(1, [], [], [], "single-node"), [0]),
        (graphgen.from_edges(5, [1, 2], [2, 3], [4, 5], "isolated-source"), [0, 1]),
        (graphgen.from_edges(3, [0, 0, 0, 1], [0, 1, 1, 1], [3, 7, 2, 0], "loops-and-dups"), [0]),
        (graphgen.from_edges(4, [0, 1, 2], [1, 2, 3], [0, 0, 0], "zero-weights"), [0]),  # wbits = 0
        (pins.path_graph(3000, np.full(2999, 7)), [0]),
        (hub, [0, 1, 17]),
        (graphgen.uniform(14), [0, 1234]),
        (graphgen.rmat(15), list(graphgen.sources(graphgen.rmat(15), 2, graphgen.FAMILY_RMAT))),
        (graphgen.grid(96), [0, 4000]),            # weights up to 1000: 10 bits
        (_barbell(3000, 20000, 12, 5), [0]),       # small-frontier kernel in and out
    ]


def test_packed_sssp_matches_oracle():
    """SSSP on packed arcs (one 32-bit word per arc) gives the oracle's
    distances, bit for bit, on edge cases, tiles with ragged tails, the
    small-frontier kernel and several weight widths."""
    for g, srcs in _packed_cases():
        dg = _dev(g)
        arcs, wb = dg.ensure_packed()
        assert wb == int(g.weights.max()).bit_length() if g.m else wb == 0
        if g.m:
            exp = (g.cols.astype(np.uint64) << wb) | g.weights.astype(np.uint64)
            assert np.array_equal(arcs.cpu().numpy().view(np.uint32)[: g.m], exp.astype(np.uint32)), g.name
        for s in srcs:
            got = lbg.sssp(dg, int(s), packed=True).cpu().numpy().view(np.uint32)
            assert np.array_equal(got, O.dijkstra(g.offsets, g.cols, g.weights, int(s))), (g.name, s)
    for gg, s in pins.tiny_graphs(count=20, seed=9):
        got = lbg.sssp(_dev(gg), int(s), packed=True).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, O.dijkstra(gg.offsets, gg.cols, gg.weights, int(s)))


def test_packed_range_errors():
    # 2^23 node ids leave 9 bits: a weight of 1024 needs 11
    n = 1 << 23
    g = graphgen.from_edges(n, [0, 5], [n - 1, 3], [1024, 7], "wide")
    dg = _dev(g)
    with pytest.raises(lbg.LbgError, match="do not fit"):
        dg.ensure_packed()
    arcs = torch.zeros(2, dtype=torch.int32, device="cuda")
    ws = lbg.Workspace("cuda")
    buf = ws.get(lbg.workspace_bytes(n, 2, "balanced", True))
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    for wb in (32, -1, 10):
        rc = lbg.lib.lbg_sssp_packed(lbg._ptr(dg.offsets), lbg._ptr(arcs), wb, n, 2, 0, lbg._ptr(out),
                                     lbg._ptr(buf), buf.numel(), None, None)
        assert rc == lbg.ERANGE, wb


def _expected_slicing(g):
    S = lbg.slice_nodes(g.n)
    row = np.repeat(np.arange(g.n), g.degrees)
    sl = np.minimum(g.cols.astype(np.int64) // S, 7)
    order = np.lexsort((sl, row))  # by node, then slice; stable within a slice
    cnt = np.zeros((g.n, 8), np.int64)
    np.add.at(cnt, (row, sl), 1)
    first = g.offsets[:-1, None].astype(np.int64) + np.cumsum(cnt, axis=1) - cnt
    return order, np.concatenate([first.ravel(), [g.m]])


@pytest.mark.parametrize("which", ["uniform", "rmat", "hub", "tiny"])
def test_slice_graph_groups_adjacency(which):
    """lbg_slice_graph regroups every adjacency list by destination slice,
    keeping the input order within a slice (compared with a stable sort),
    and its slice offsets are the per-node slice prefix sums."""
    rng = np.random.default_rng(3)
    if which == "uniform":
        g = graphgen.uniform(13)          # unsorted adjacency lists
    elif which == "rmat":
        g = graphgen.rmat(14)
    elif which == "hub":
        n = 5000
        src = np.concatenate([np.zeros(4000, np.int64), rng.integers(0, n, 9000)])
        dst = rng.integers(0, n, src.size)
        g = graphgen.from_edges(n, src, dst, rng.integers(1, 9, src.size), "hub")
    else:
        g = graphgen.from_edges(3, [0, 0, 2], [2, 1, 0], [5, 6, 7], "tiny")
    dg = _dev(g)
    sg = lbg.slice_graph(dg)
    order, exp_so = _expected_slicing(g)
    assert np.array_equal(sg.slice_offsets.cpu().numpy().astype(np.int64), exp_so)
    assert np.array_equal(sg.cols.cpu().numpy()[: g.m], g.cols[order])
    assert np.array_equal(sg.weights.cpu().numpy().view(np.uint32)[: g.m], g.weights[order])
    # BFS-only graphs: no weights in, none out
    bg = lbg.DeviceGraph(dg.offsets, dg.cols, None)
    sb = lbg.slice_graph(bg)
    assert sb.weights is None and np.array_equal(sb.cols.cpu().numpy()[: g.m], g.cols[order])


def _expected_split(g, mdt):
    """The split graph written out from the node-splitting piece sizes of the
    oracle: parents' own pieces first (node order), then every child piece
    (parent order, piece order); mdt 0 leaves every node whole."""
    deg = g.degrees.astype(np.int64)
    pieces = [O.ns_pieces(int(d), mdt) if mdt > 0 else np.array([d], np.int64) for d in deg]
    own = np.array([p[0] for p in pieces], np.int64)
    kids = [p[1:] for p in pieces]
    nkids = np.array([k.size for k in kids], np.int64)
    child_base = np.concatenate([[0], np.cumsum(nkids)])
    P = int(own.sum())
    kid_sizes = np.concatenate(kids + [np.zeros(0, np.int64)])
    so = np.concatenate([np.concatenate([[0], np.cumsum(own)])[:-1], P + np.concatenate([[0], np.cumsum(kid_sizes)])])
    off = g.offsets.astype(np.int64)
    idx = np.arange(g.m, dtype=np.int64)
    node = np.repeat(np.arange(g.n), deg)
    first = idx < off[node] + own[node]
    order = np.concatenate([idx[first], idx[~first]])  # stable: node order, then arc order
    return so, child_base, order


@pytest.mark.parametrize("mdt", [0, 1, 2, 7, 64])
@pytest.mark.parametrize("which", ["uniform", "rmat", "hub", "tiny"])
def test_split_graph_layout(which, mdt):
    """lbg_split_graph against the split graph built from the oracle's piece
    sizes: offsets, child table and arc order, exactly."""
    rng = np.random.default_rng(4)
    if which == "uniform":
        g = graphgen.uniform(12)
    elif which == "rmat":
        g = graphgen.rmat(13)
    elif which == "hub":
        n = 5000
        src = np.concatenate([np.zeros(9000, np.int64), np.full(130, 7), rng.integers(0, n, 9000)])
        dst = rng.integers(0, n, src.size)
        g = graphgen.from_edges(n, src, dst, rng.integers(1, 9, src.size), "hub")
    else:
        g = graphgen.from_edges(3, [0, 0, 2], [2, 1, 0], [5, 6, 7], "tiny")
    dg = _dev(g)
    so, cb, order = _expected_split(g, mdt)
    assert lbg.split_count(dg, mdt) == cb[-1]
    sp = lbg.split_graph(dg, mdt)
    assert sp.children == cb[-1] and sp.split_offsets.numel() == g.n + sp.children + 1
    assert np.array_equal(sp.split_offsets.cpu().numpy().astype(np.int64), so)
    assert np.array_equal(sp.child_base.cpu().numpy().astype(np.int64), cb)
    assert np.array_equal(sp.cols.cpu().numpy()[: g.m], g.cols[order])
    assert np.array_equal(sp.weights.cpu().numpy().view(np.uint32)[: g.m], g.weights[order])
    bg = lbg.DeviceGraph(dg.offsets, dg.cols, None)  # BFS-only: no weights in, none out
    sb = lbg.split_graph(bg, mdt)
    assert sb.weights is None and np.array_equal(sb.cols.cpu().numpy()[: g.m], g.cols[order])


def test_split_graph_rejects_wrong_child_count():
    """lbg_split_graph recounts the children on the device and refuses a
    caller's count that differs (the output arrays would be mis-sized)."""
    import ctypes

    g = graphgen.rmat(11)
    dg = _dev(g)
    c = lbg.split_count(dg, 8)
    assert c > 0
    so = torch.empty(g.n + c + 1, dtype=torch.int32, device="cuda")
    cb = torch.empty(g.n + 1, dtype=torch.int32, device="cuda")
    cols = torch.empty(g.m, dtype=torch.int32, device="cuda")
    scratch = torch.empty(max(int(lbg.lib.lbg_split_scratch_bytes(g.n)), 256), dtype=torch.uint8, device="cuda")
    for wrong in (c - 1, c + 1):
        rc = lbg.lib.lbg_split_graph(lbg._ptr(dg.offsets), lbg._ptr(dg.cols), None, g.n, g.m, 8, wrong,
                                     lbg._ptr(so), lbg._ptr(cb), lbg._ptr(cols), None, lbg._ptr(scratch),
                                     scratch.numel(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == lbg.EINVAL and "child" in lbg.lib.lbg_last_error().decode()


@pytest.mark.parametrize("mdt", [1, 2, 7, 64, 5000])
def test_split_sizes(mdt):
    """Node splitting at split sizes from every arc its own child (1) to no
    split at all (5000): the same results as the oracle, and BFS frontier
    entries = the pieces of every reached node with arcs."""
    rng = np.random.default_rng(8)
    n = 4000
    src = np.concatenate([np.zeros(3000, np.int64), np.full(700, 3), rng.integers(0, n, 12000)])
    dst = rng.integers(0, n, src.size)
    hub = graphgen.from_edges(n, src, dst, rng.integers(0, 30, src.size), "hub")
    cases = [(hub, [0, 3, 11]), (graphgen.rmat(13), None), (graphgen.grid(40), [0])]
    cases += [(gg, [s]) for gg, s in pins.tiny_graphs(count=8, seed=9)]
    for g, srcs in cases:
        if srcs is None:
            srcs = graphgen.sources(g, 2, graphgen.FAMILY_RMAT)
        dg = _dev(g)
        for s in srcs:
            exp_l = O.bfs(g.offsets, g.cols, int(s))
            lv, st = _gpu_bfs(dg, s, "split", mdt=mdt, stats=True)
            assert np.array_equal(lv, exp_l), (g.name, s, mdt)
            reached = exp_l != pins.BFS_INF
            deg = g.degrees.astype(np.int64)
            pcs = np.where(deg > mdt, (deg + mdt - 1) // mdt, 1)
            assert st["frontier_entries"] == int(pcs[reached & (deg > 0)].sum()), (g.name, s, mdt)
            assert st["edges_scanned"] == g.reached_arcs(reached)
            # levels counts frontiers with at least one out-arc
            assert st["levels"] == int(exp_l[reached & (deg > 0)].max(initial=-1)) + 1
            d = _gpu_sssp(dg, s, "split", mdt=mdt)
            assert np.array_equal(d, O.dijkstra(g.offsets, g.cols, g.weights, int(s))), (g.name, s, mdt)


def _expected_order(g):
    """The degree-class ordered copy written out with numpy: classes by bit
    length of the out-degree, largest first, original order within a class;
    each list stably partitioned by its destinations' classes."""
    deg = g.degrees.astype(np.int64)
    cls = np.array([int(d).bit_length() for d in deg], np.int64)
    order = np.argsort(-cls, kind="stable")
    new_id = np.empty(g.n, np.int64)
    new_id[order] = np.arange(g.n)
    noff = np.concatenate([[0], np.cumsum(deg[order])])
    off = g.offsets.astype(np.int64)
    cols, ws = [], []
    for v in order:
        c = g.cols[off[v]: off[v + 1]].astype(np.int64)
        p = np.argsort(-cls[c], kind="stable")
        cols.append(new_id[c[p]])
        ws.append(g.weights[off[v]: off[v + 1]][p])
    cat = lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt)
    return new_id, noff, cat(cols, np.int64), cat(ws, np.uint32)


@pytest.mark.parametrize("which", ["uniform", "rmat", "hub", "tiny", "single"])
def test_order_graph_layout(which):
    """lbg_order_graph against the ordered copy built with numpy: new ids,
    offsets, renamed and partitioned adjacency, weights, exactly."""
    rng = np.random.default_rng(6)
    if which == "uniform":
        g = graphgen.uniform(12)
    elif which == "rmat":
        g = graphgen.rmat(14)
    elif which == "hub":
        n = 9000                       # more than two workgroups' chunks of nodes
        src = np.concatenate([np.zeros(7000, np.int64), np.full(300, 4321), rng.integers(0, n, 20000)])
        dst = rng.integers(0, n, src.size)
        g = graphgen.from_edges(n, src, dst, rng.integers(1, 9, src.size), "hub")
    elif which == "tiny":
        g = graphgen.from_edges(4, [0, 0, 2, 3, 3, 3], [2, 1, 0, 0, 1, 2], [5, 6, 7, 8, 9, 10], "tiny")
    else:
        g = graphgen.from_edges(1, [], [], [], "single")
    dg = _dev(g)
    og = lbg.order_graph(dg)
    new_id, noff, cols, ws = _expected_order(g)
    assert np.array_equal(og.new_id.cpu().numpy().astype(np.int64), new_id)
    assert np.array_equal(og.offsets.cpu().numpy().astype(np.int64), noff)
    assert np.array_equal(og.cols.cpu().numpy()[: g.m].astype(np.int64), cols)
    assert np.array_equal(og.weights.cpu().numpy().view(np.uint32)[: g.m], ws)
    bg = lbg.DeviceGraph(dg.offsets, dg.cols, None)  # BFS-only graph: no weights in, none out
    ob = lbg.order_graph(bg)
    assert ob.weights is None and np.array_equal(ob.cols.cpu().numpy()[: g.m].astype(np.int64), cols)


def test_ordered_sssp_matches_oracle():
    """SSSP on the ordered copy, source and distances in original ids, equals
    the oracle on the original graph: tiny, degenerate, skewed, grid."""
    cases = [(gg, [s]) for gg, s in pins.tiny_graphs(count=20, seed=31)]
    cases += [(graphgen.from_edges(1, [], [], [], "single-node"), [0]),
              (graphgen.from_edges(5, [1, 2], [2, 3], [4, 5], "isolated-source"), [0, 1]),
              (graphgen.from_edges(3, [0, 0, 0, 1], [0, 1, 1, 1], [3, 7, 2, 0], "loops-and-dups"), [0]),
              (pins.path_graph(3000, np.full(2999, 7)), [0, 1500]),
              (graphgen.rmat(15), None), (graphgen.grid(64), [0, 100]), (graphgen.uniform(13), [0, 77])]
    for g, srcs in cases:
        if srcs is None:
            srcs = graphgen.sources(g, 3, graphgen.FAMILY_RMAT)
        dg = _dev(g)
        for s in srcs:
            got = _gpu_sssp(dg, s, "balanced", ordered=True)
            assert np.array_equal(got, O.dijkstra(g.offsets, g.cols, g.weights, int(s))), (g.name, s)


def test_repeat_runs_identical():
    """Relaxation order differs from run to run; results must not."""
    g = graphgen.rmat(14)
    dg = _dev(g)
    s = int(graphgen.sources(g, 1, graphgen.FAMILY_RMAT)[0])
    exp = O.dijkstra(g.offsets, g.cols, g.weights, s)
    for strat in STRATS:
        for _ in range(5):
            assert np.array_equal(_gpu_sssp(dg, s, strat), exp)
    for _ in range(5):
        assert np.array_equal(_gpu_sssp(dg, s, "balanced", ordered=True), exp)


def test_stats_and_validate():
    g = graphgen.rmat(13)
    dg = _dev(g)
    s = int(graphgen.sources(g, 1, graphgen.FAMILY_RMAT)[0])
    lv_exp = O.bfs(g.offsets, g.cols, s)
    reached = lv_exp != pins.BFS_INF
    for strat in ("node", "balanced"):
        lv, st = _gpu_bfs(dg, s, strat, stats=True)
        assert np.array_equal(lv, lv_exp)
        assert st["levels"] == int(lv_exp[reached & (g.degrees > 0)].max()) + 1
        assert st["edges_scanned"] == g.reached_arcs(reached)
        assert st["updates"] == int(reached.sum()) - 1
        assert st["frontier_entries"] == int((reached & (g.degrees > 0)).sum())
    # sliced: one entry per (node, destination slice it has arcs into) for
    # nodes of degree >= slice_min, one entry for the others
    S = lbg.slice_nodes(g.n)
    row = np.repeat(np.arange(g.n), g.degrees)
    pairs = np.unique(row.astype(np.int64) * 8 + np.minimum(g.cols // S, 7))
    per_node = np.bincount(pairs // 8, minlength=g.n)
    saved = lbg.get_slice_min()
    try:
        for smin in (0, 16, 2**31 - 1):
            lbg.set_slice_min(smin)
            lv, st = _gpu_bfs(dg, s, "sliced", stats=True)
            assert np.array_equal(lv, lv_exp)
            assert st["levels"] == int(lv_exp[reached & (g.degrees > 0)].max()) + 1
            assert st["edges_scanned"] == g.reached_arcs(reached)
            assert st["updates"] == int(reached.sum()) - 1
            split = g.degrees >= smin
            exp_entries = per_node[reached & split].sum() + (reached & ~split & (g.degrees > 0)).sum()
            assert st["frontier_entries"] == int(exp_entries), smin
    finally:
        lbg.set_slice_min(saved)
    d, st = _gpu_sssp(dg, s, "balanced", stats=True)
    assert st["edges_scanned"] >= g.reached_arcs(reached)
    lbg.validate_csr(dg)
    bad = graphgen.Graph("bad", g.offsets.copy(), g.cols.copy(), g.weights.copy())
    bad.cols[7] = g.n + 3
    with pytest.raises(lbg.LbgError, match="outside"):
        lbg.validate_csr(_dev(bad))
    bad2 = graphgen.Graph("bad2", g.offsets.copy(), g.cols.copy(), g.weights.copy())
    bad2.offsets[5] = bad2.offsets[6] + 1
    with pytest.raises(lbg.LbgError, match="decrease"):
        lbg.validate_csr(_dev(bad2))


def test_device_argument_errors_leave_output_untouched():
    g = graphgen.uniform(8)
    dg = _dev(g)
    out = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(lbg.LbgError):
        lbg.bfs(dg, g.n + 1, out=out)
    assert int((out == -7).sum()) == g.n


# -------------------------------------------------------------- full size --
@pytest.fixture(scope="module")
def rmat22():
    g = graphgen.rmat(22)
    return g, _dev(g), graphgen.sources(g, 64, graphgen.FAMILY_RMAT)


def test_rmat22_full_ordered(rmat22):
    """The degree-class ordered copy at the benchmark size: full distance
    vectors against the oracle for two sources."""
    g, dg, srcs = rmat22
    og = dg.ensure_ordered()
    nid = og.new_id.cpu().numpy()
    assert np.array_equal(np.sort(nid), np.arange(g.n))  # a permutation
    for s in srcs[:2]:
        got = lbg.sssp(dg, int(s), ordered=True).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, O.dijkstra(g.offsets, g.cols, g.weights, int(s)))


def test_rmat22_full_packed(rmat22):
    g, dg, srcs = rmat22
    arcs, wb = dg.ensure_packed()
    assert wb == 8
    for s in srcs[:2]:
        got = lbg.sssp(dg, int(s), packed=True).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, O.dijkstra(g.offsets, g.cols, g.weights, int(s)))


@pytest.mark.parametrize("strat", FULL_STRATS)
def test_rmat22_full(rmat22, strat):
    """RMAT scale 22, edge factor 16 (the benchmark workload): full vectors
    against the oracle for two of the 64 sources, certificate for a third."""
    g, dg, srcs = rmat22
    _check(g, dg, srcs[:2] if strat == "balanced" else srcs[:1], strat)
    if strat == "balanced":
        s = int(srcs[2])
        d = _gpu_sssp(dg, s, strat)
        assert O.certificate(g.offsets, g.cols, g.weights, s, d)[0] == 0
        lv = _gpu_bfs(dg, s, strat)
        assert O.certificate(g.offsets, g.cols, None, s, lv)[0] == 0


@pytest.fixture(scope="module")
def grid2048():
    g = graphgen.grid(2048)
    return g, _dev(g), graphgen.sources(g, 16, graphgen.FAMILY_GRID)


@pytest.mark.parametrize("strat", FULL_STRATS)
def test_grid2048_full(grid2048, strat):
    """2048x2048 road-like grid (10% of edges dropped, 1% shortcuts, the
    high-diameter configuration): full BFS and SSSP vectors against the
    oracle for every strategy, each from its own one of the 16 sources."""
    g, dg, srcs = grid2048
    _check(g, dg, [int(srcs[FULL_STRATS.index(strat)])], strat)


@pytest.mark.parametrize("strat", ["balanced", "binned"])
def test_grid2048_noshortcut_full(grid2048, strat):
    """The no-shortcut companion (about 4000 levels of small frontiers): BFS
    and SSSP against the oracle with the balanced strategy (which runs most
    levels in the small-frontier kernel) and the degree-binned one (one
    launch per level throughout)."""
    h = graphgen.grid(2048, shortcut_frac=0)
    s = int(grid2048[2][15 - ["balanced", "binned"].index(strat)])
    _check(h, _dev(h), [s], strat)


@pytest.mark.parametrize("chunk", range(4))
def test_rmat22_all_sources_certified(rmat22, chunk):
    """Every one of the 64 benchmark sources (16 per chunk): balanced BFS on
    the input CSR and balanced SSSP on the degree-class ordered copy (the two
    solves the benchmark times) and on the input CSR, each certified exact by
    the oracle's O(m) certificate (source at 0, no arc relaxable, tight arcs
    reach exactly the finite nodes)."""
    from concurrent.futures import ThreadPoolExecutor

    g, dg, srcs = rmat22
    dg.ensure_ordered()
    jobs = []
    for s in srcs[16 * chunk: 16 * (chunk + 1)]:
        s = int(s)
        jobs.append((s, None, _gpu_bfs(dg, s, "balanced")))
        jobs.append((s, g.weights, lbg.sssp(dg, s, ordered=True).cpu().numpy().view(np.uint32)))
        jobs.append((s, g.weights, _gpu_sssp(dg, s, "balanced")))

    def cert(job):
        s, w, d = job
        return s, w is None, O.certificate(g.offsets, g.cols, w, s, d)[0]

    with ThreadPoolExecutor(8) as ex:  # the oracle's C calls release the interpreter lock
        bad = [(s, bfs) for s, bfs, code in ex.map(cert, jobs) if code != 0]
    assert not bad, bad


@pytest.mark.parametrize("strat", STRATS)
def test_workspace_reuse_across_sources(strat):
    """Back-to-back solves from different sources share one workspace: no
    state of an earlier solve (visited snapshots, filters, stamps) may leak
    into a later one.  A directed graph where the sources reach nested sets
    makes any leaked 'already visited' bit change a level."""
    g = graphgen.uniform(12, k=3)
    dg = _dev(g)
    ws = lbg.Workspace("cuda")
    srcs = [0, 1, 2, 3, 0, 5, 0]
    for s in srcs:
        lv = lbg.bfs(dg, s, strategy=strat, workspace=ws).cpu().numpy()
        assert np.array_equal(lv, O.bfs(g.offsets, g.cols, s)), f"bfs src={s}"
        d = lbg.sssp(dg, s, strategy=strat, workspace=ws).cpu().numpy().view(np.uint32)
        assert np.array_equal(d, O.dijkstra(g.offsets, g.cols, g.weights, s)), f"sssp src={s}"
        if strat == "balanced":  # the ordered copy shares the balanced workspace
            d = lbg.sssp(dg, s, workspace=ws, ordered=True).cpu().numpy().view(np.uint32)
            assert np.array_equal(d, O.dijkstra(g.offsets, g.cols, g.weights, s)), f"ordered src={s}"


def test_concurrent_solves_on_two_streams():
    """The header's thread-safety contract: solves running at the same time
    from two host threads, each with its own stream, workspace and output,
    give the oracle's answers (the library keeps per-thread control blocks
    and events; the interpreter lock is released during the C calls)."""
    import threading

    g = graphgen.rmat(16)
    dg = _dev(g)
    srcs = [int(s) for s in graphgen.sources(g, 6, graphgen.FAMILY_RMAT)]
    exp = {s: (O.bfs(g.offsets, g.cols, s), O.dijkstra(g.offsets, g.cols, g.weights, s)) for s in srcs}
    errors = []

    def worker(my_srcs, strat):
        try:
            stream = torch.cuda.Stream()
            ws = lbg.Workspace("cuda")
            for _ in range(3):
                for s in my_srcs:
                    lv = lbg.bfs(dg, s, strategy=strat, workspace=ws, stream=stream)
                    d = lbg.sssp(dg, s, strategy=strat, workspace=ws, stream=stream)
                    stream.synchronize()
                    if not np.array_equal(lv.cpu().numpy(), exp[s][0]):
                        errors.append(("bfs", strat, s))
                    if not np.array_equal(d.cpu().numpy().view(np.uint32), exp[s][1]):
                        errors.append(("sssp", strat, s))
        except Exception as exc:  # surfaced below
            errors.append(repr(exc))

    ts = [threading.Thread(target=worker, args=(srcs[:3], "balanced")),
          threading.Thread(target=worker, args=(srcs[3:], "binned"))]
    for t in ts:
        t.start()
    for t in ts:
        t.join(120)
    assert not any(t.is_alive() for t in ts)
    assert not errors, errors
