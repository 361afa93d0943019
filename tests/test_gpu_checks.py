"""GPU checks of the library's bookkeeping against the oracle and plain
numpy: the hierarchical strategy's sub-iteration schedule (Section III-C)
against oracle_hp_schedule, the skipped-arc counter behind the SSSP roofline
figure, the COO source builder, and the device guards that turn a foreign
renaming or split table into an error instead of an out-of-range access."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
from paper_1711_00231_amd import lbg  # noqa: E402

O = oracle.get()
HANDOVER = 1024  # sublists below this size are expanded edge-balanced, all at once


def _dev(g):
    return lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights)


def _expected_schedule(g, src, mdt):
    """Per BFS level: the oracle's sublist sizes of that level's worklist (the
    nodes at hop distance L with out-arcs), cut after the first sublist that
    is handed over to workload decomposition."""
    lv = O.bfs(g.offsets, g.cols, src)
    deg = g.degrees
    rows = []
    for L in range(int(lv[lv != np.iinfo(np.int32).max].max()) + 1):
        d = deg[(lv == L) & (deg > 0)]
        if d.size == 0:
            break
        sizes = list(O.hp_schedule(d, mdt))
        k = next((i for i, x in enumerate(sizes) if x < HANDOVER), len(sizes) - 1)
        rows.append(sizes[: k + 1])
    return rows


def _device_schedule(dg, src, mdt):
    lbg.set_hier_mdt(mdt)
    try:
        lv = lbg.bfs(dg, src, strategy="hier").cpu().numpy()
        sched, used = lbg.hier_last_schedule()
    finally:
        lbg.set_hier_mdt(0)
    assert used == mdt
    return lv, [[int(x) for x in row[row > 0]] for row in sched]


def test_hier_schedule_window_boundaries():
    """A level of 3000 nodes whose degrees are 3, 8 = 2 MDT (an exact multiple)
    and 9 under MDT 4: sublists 3000, 2400, 1200.  A node with exactly 8 arcs
    leaves after its second window."""
    rng = np.random.default_rng(3)
    n1, n2 = 3000, 20000
    degs = np.array([8] * 1200 + [9] * 1200 + [3] * 600)
    rng.shuffle(degs)
    src = [np.zeros(n1, dtype=np.int64)]
    dst = [np.arange(1, n1 + 1)]
    for i, d in enumerate(degs):
        src.append(np.full(d, i + 1))
        dst.append(rng.integers(n1 + 1, n1 + 1 + n2, d))
    src, dst = np.concatenate(src), np.concatenate(dst)
    g = graphgen.from_edges(n1 + 1 + n2, src, dst, np.ones(src.size), "hp-boundaries")
    exp = _expected_schedule(g, 0, 4)
    assert exp[1] == [3000, 2400, 1200]  # the construction
    lv, got = _device_schedule(_dev(g), 0, 4)
    assert np.array_equal(lv, O.bfs(g.offsets, g.cols, 0))
    assert got == exp


@pytest.mark.parametrize("mdt", [8, 32])
def test_hier_schedule_rmat(mdt):
    """Skewed degrees over several levels: every level's recorded sublist
    sizes equal the oracle's schedule of that level's worklist."""
    g = graphgen.rmat(15)
    s = int(graphgen.sources(g, 1, graphgen.FAMILY_RMAT)[0])
    exp = _expected_schedule(g, s, mdt)
    assert any(len(r) > 2 for r in exp)  # several sub-iterations somewhere
    lv, got = _device_schedule(_dev(g), s, mdt)
    assert np.array_equal(lv, O.bfs(g.offsets, g.cols, s))
    assert got == exp


def test_skipped_arcs_accounting():
    """SSSP loads every arc leaving the reached set at least once; skipped
    arcs are a part of the queued ones; BFS skips nothing."""
    g = graphgen.rmat(16)
    dg = _dev(g)
    reached_arcs = 0
    for s in graphgen.sources(g, 3, graphgen.FAMILY_RMAT):
        d, st = lbg.sssp(dg, int(s), stats=True)
        lv, sb = lbg.bfs(dg, int(s), stats=True)
        fin = lv.cpu().numpy() != lbg.BFS_INF
        reached_arcs = int(g.degrees[fin].sum())
        assert 0 <= st["edges_skipped"] <= st["edges_scanned"]
        assert st["edges_scanned"] - st["edges_skipped"] >= reached_arcs
        assert sb["edges_skipped"] == 0 and sb["edges_scanned"] == reached_arcs
        assert np.array_equal(d.cpu().numpy().view(np.uint32), O.dijkstra(g.offsets, g.cols, g.weights, int(s)))
        # the hierarchical strategy skips within windows: counted once per
        # entry, however many workgroups stage it at the hand-over
        dh, sh = lbg.sssp(dg, int(s), strategy="hier", stats=True)
        assert 0 <= sh["edges_skipped"] <= sh["edges_scanned"]
        assert np.array_equal(dh.cpu().numpy().view(np.uint32), d.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("name", ["rmat14", "uniform12", "empty-tail"])
def test_coo_sources(name):
    if name == "rmat14":
        g = graphgen.rmat(14)
    elif name == "uniform12":
        g = graphgen.uniform(12)
    else:  # trailing nodes without arcs, a node with a hub's worth of arcs
        g = graphgen.from_edges(5000, np.r_[np.zeros(3000), np.arange(1, 100)],
                                np.r_[np.arange(1, 3001), np.arange(2, 101)], None, "empty-tail")
    dg = lbg.DeviceGraph.from_numpy(g.offsets, g.cols, None)
    got = dg.ensure_coo().cpu().numpy()[: g.m]
    assert np.array_equal(got, np.repeat(np.arange(g.n, dtype=np.int32), g.degrees))


def test_foreign_renaming_table_is_an_error():
    """lbg_sssp_ordered with a new-id table that does not belong to the graph
    (the source maps outside [0, n)): the device guard stops the solve before
    any access through that id and the call reports it."""
    g = graphgen.rmat(12)
    dg = _dev(g)
    og = dg.ensure_ordered()
    bad = og.new_id.clone()
    bad[5] = g.n + 17
    good = lbg.sssp(dg, 5, ordered=True).cpu().numpy().view(np.uint32)
    assert np.array_equal(good, O.dijkstra(g.offsets, g.cols, g.weights, 5))
    saved = og.new_id
    og.new_id = bad
    try:
        with pytest.raises(lbg.LbgError, match="source outside"):
            lbg.sssp(dg, 5, ordered=True)
    finally:
        og.new_id = saved
    # the workspace and the library stay usable
    again = lbg.sssp(dg, 5, ordered=True).cpu().numpy().view(np.uint32)
    assert np.array_equal(again, good)


def test_malformed_split_table_is_an_error():
    """A split graph whose child table names a child piece without arcs (not
    one lbg_split_graph writes): reported as an error, never a silent wrong
    answer."""
    g = graphgen.rmat(12)
    dg = _dev(g)
    sp = dg.ensure_split(mdt=64)
    assert sp.children > 0
    s = int(graphgen.sources(g, 1, graphgen.FAMILY_RMAT)[0])
    ok = lbg.bfs(dg, s, strategy="split", mdt=64).cpu().numpy()
    assert np.array_equal(ok, O.bfs(g.offsets, g.cols, s))
    so = sp.split_offsets.cpu().numpy()
    cb = sp.child_base.cpu().numpy()
    # the first parent with children: empty its first child's piece
    v = int(np.nonzero(np.diff(cb) > 0)[0][0])
    c = int(cb[v])
    bad = so.copy()
    bad[g.n + c + 1] = bad[g.n + c]
    saved = sp.split_offsets
    sp.split_offsets = torch.from_numpy(bad).to(saved.device)
    try:
        with pytest.raises(lbg.LbgError, match="malformed split table"):
            lbg.bfs(dg, v, strategy="split", mdt=64)  # v's pieces are queued at once
    finally:
        sp.split_offsets = saved
    again = lbg.bfs(dg, s, strategy="split", mdt=64).cpu().numpy()
    assert np.array_equal(again, ok)
