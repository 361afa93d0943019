"""GPU parity of the 64-bit addressing form of every kernel.  Graphs of
2^29 nodes or 2^30 arcs and more are solved with 64-bit element addresses;
lbg_set_addressing(1) selects that form for any graph, so each strategy,
BFS scan levels, packed and ordered SSSP, batched solves and the engine are
compared with the oracle, bit for bit, on small graphs in it."""
import numpy as np
import pytest

import graphgen
import oracle
import pins

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
from paper_1711_00231_amd import lbg, serve  # noqa: E402

O = oracle.get()
STRATS = ["node", "edge", "balanced", "binned", "hier", "sliced", "split"]


@pytest.fixture(autouse=True)
def _wide():
    lbg.set_addressing(1)
    yield
    lbg.set_addressing(0)
    lbg.set_bfs_scan_min(-1)


def _dev(g):
    return lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights)


def _cases():
    gs = [(graphgen.rmat(14), graphgen.FAMILY_RMAT), (graphgen.uniform(13), graphgen.FAMILY_UNIFORM),
          (graphgen.grid(64), graphgen.FAMILY_GRID)]
    out = [(g, [int(s) for s in graphgen.sources(g, 2, f)]) for g, f in gs]
    out += [(gg, [int(s)]) for gg, s in pins.tiny_graphs(count=8, seed=41)]
    out += [(graphgen.from_edges(1, [], [], [], "single-node"), [0]),
            (pins.path_graph(3000, np.full(2999, 7)), [0, 1500])]
    return out


@pytest.mark.parametrize("strat", STRATS)
def test_strategies_wide(strat):
    for g, srcs in _cases():
        dg = _dev(g)
        for s in srcs:
            got = lbg.bfs(dg, s, strategy=strat).cpu().numpy()
            assert np.array_equal(got, O.bfs(g.offsets, g.cols, s)), (g.name, s, strat)
            got = lbg.sssp(dg, s, strategy=strat).cpu().numpy().view(np.uint32)
            assert np.array_equal(got, O.dijkstra(g.offsets, g.cols, g.weights, s)), (g.name, s, strat)


@pytest.mark.parametrize("scan_min", [0, -1])
def test_bfs_scan_levels_wide(scan_min):
    lbg.set_bfs_scan_min(scan_min)
    for g, srcs in _cases() + [(graphgen.rmat(18), [0, 1, 5])]:
        dg = _dev(g)
        for s in srcs:
            got = lbg.bfs(dg, s).cpu().numpy()
            assert np.array_equal(got, O.bfs(g.offsets, g.cols, s)), (g.name, s, scan_min)


def test_packed_and_ordered_sssp_wide():
    for g, srcs in _cases():
        dg = _dev(g)
        for s in srcs:
            exp = O.dijkstra(g.offsets, g.cols, g.weights, s)
            assert np.array_equal(lbg.sssp(dg, s, packed=True).cpu().numpy().view(np.uint32), exp), (g.name, s)
            assert np.array_equal(lbg.sssp(dg, s, ordered=True).cpu().numpy().view(np.uint32), exp), (g.name, s)


def _expected(g, s, kind):
    if kind == lbg.KIND_BFS:
        return O.bfs(g.offsets, g.cols, s)
    return O.dijkstra(g.offsets, g.cols, g.weights, s).view(np.int32)


def _packed():
    gs = [graphgen.rmat(11, salt=51), graphgen.uniform(n=3001, k=8, wlo=1, whi=255, salt=52),
          graphgen.grid(40, salt=53)] + [g for g, _ in pins.tiny_graphs(count=4, seed=54)]
    u, nb, _ = graphgen.pack(gs)
    return gs, u, nb


def test_batch_wide():
    gs, u, nb = _packed()
    dg = _dev(u)
    rng = np.random.default_rng(55)
    queries, expect = [], []
    for i, g in enumerate(gs):
        for s in rng.integers(0, g.n, 3):
            for kind in (lbg.KIND_BFS, lbg.KIND_SSSP):
                queries.append((int(nb[i] + s), int(nb[i]), int(nb[i + 1]), kind))
                expect.append(_expected(g, int(s), kind))
    ws = lbg.Workspace("cuda")
    for graph in (False, True, True):  # eager, then a captured batch replayed
        out = lbg.batch_solve(dg, queries, workspace=ws, graph=graph).cpu().numpy()
        off = 0
        for q, e in zip(queries, expect):
            assert np.array_equal(out[off: off + q[2] - q[1]], e), (q, graph)
            off += q[2] - q[1]


def test_engine_wide():
    gs, u, nb = _packed()
    dg = _dev(u)
    eng = lbg.Engine(dg, max_queries=8, max_rows=4 * u.n, max_level_arcs=8 * u.m)
    rows = serve.RowAllocator(eng.max_rows)
    rng = np.random.default_rng(56)
    waiting = [(i, int(rng.integers(gs[i].n)), k) for i in range(len(gs)) for k in (0, 1)]
    live, done, step = {}, 0, 0
    total = len(waiting)
    while waiting or live:
        while waiting:
            i, s, kind = waiting[0]
            n_i = int(nb[i + 1] - nb[i])
            row = rows.alloc(n_i)
            slot = eng.submit(int(nb[i] + s), int(nb[i]), int(nb[i + 1]), kind, row) if row is not None else -1
            if slot < 0:
                if row is not None:
                    rows.release(row, n_i)
                break
            live[slot] = (i, s, kind, row, n_i)
            waiting.pop(0)
        for slot in eng.step(1):
            i, s, kind, row, n_i = live.pop(slot)
            assert np.array_equal(eng.rows[row: row + n_i].cpu().numpy(), _expected(gs[i], s, kind)), (i, s, kind)
            eng.release(slot)
            rows.release(row, n_i)
            done += 1
        step += 1
        assert step < 10000
    assert done == total


def test_noalloc_sssp_wide():
    for g, srcs in _cases()[:4]:
        dg = _dev(g)
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        for s in srcs:
            lbg.sssp_noalloc(dg, s, out=out)
            assert np.array_equal(out.cpu().numpy().view(np.uint32),
                                  O.dijkstra(g.offsets, g.cols, g.weights, s)), (g.name, s)


def test_forms_alternate_on_one_workspace():
    """Narrow and wide solves of one graph in turn, on one workspace (the
    per-graph record of scan levels is shared by both forms)."""
    g = graphgen.rmat(16)
    dg = _dev(g)
    ws = lbg.Workspace()
    srcs = [int(s) for s in graphgen.sources(g, 4, graphgen.FAMILY_RMAT)]
    for k, s in enumerate(srcs * 2):
        lbg.set_addressing(k % 2)
        assert np.array_equal(lbg.bfs(dg, s, workspace=ws).cpu().numpy(), O.bfs(g.offsets, g.cols, s)), (k, s)
        assert np.array_equal(lbg.sssp(dg, s, workspace=ws, ordered=True).cpu().numpy().view(np.uint32),
                              O.dijkstra(g.offsets, g.cols, g.weights, s)), (k, s)
