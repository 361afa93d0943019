"""Batched solves: every query's row, computed inside one shared
level-synchronous batch, is bit-identical to the CPU oracle on the query's
own instance and to the single-query path."""
import numpy as np
import pytest

import graphgen
import oracle
import pins

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
from paper_1711_00231_amd import lbg  # noqa: E402

O = oracle.get()


def _instances():
    gs = [graphgen.rmat(s, salt=100 + s) for s in (8, 10, 11)]
    gs += [graphgen.uniform(n=n, k=8, wlo=1, whi=255, salt=200 + n) for n in (700, 1500, 3001)]
    gs += [graphgen.grid(30, salt=7)]
    gs += [g for g, _ in pins.tiny_graphs(count=6, seed=99)]
    gs += [graphgen.from_edges(1, [], [], [], "single")]
    return gs


def _expected(g, s, kind):
    if kind == lbg.KIND_BFS:
        return O.bfs(g.offsets, g.cols, s)
    return O.dijkstra(g.offsets, g.cols, g.weights, s).view(np.int32)


def test_batch_matches_oracle_per_query():
    gs = _instances()
    u, nb, _ = graphgen.pack(gs)
    dg = lbg.DeviceGraph.from_numpy(u.offsets, u.cols, u.weights)
    rng = np.random.default_rng(3)
    queries, expect = [], []
    for i, g in enumerate(gs):
        for s in rng.integers(0, g.n, 3):
            for kind in (lbg.KIND_BFS, lbg.KIND_SSSP):
                queries.append((int(nb[i] + s), int(nb[i]), int(nb[i + 1]), kind))
                expect.append(_expected(g, int(s), kind))
    out, st = lbg.batch_solve(dg, queries, stats=True)
    out = out.cpu().numpy()
    off = 0
    for q, e in zip(queries, expect):
        row = out[off: off + q[2] - q[1]]
        assert np.array_equal(row, e), f"query {q}"
        off += q[2] - q[1]
    assert st["levels"] >= 1 and st["edges_scanned"] > 0


def test_batch_equals_single_and_repeats():
    gs = [graphgen.rmat(12, salt=5), graphgen.uniform(n=5000, k=8, wlo=1, whi=255, salt=9)]
    u, nb, _ = graphgen.pack(gs)
    dg = lbg.DeviceGraph.from_numpy(u.offsets, u.cols, u.weights)
    singles = [lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights) for g in gs]
    queries, ref = [], []
    for i, g in enumerate(gs):
        for s in graphgen.sources(g, 4, graphgen.FAMILY_BATCH, salt=i):
            queries.append((int(nb[i] + s), int(nb[i]), int(nb[i + 1]), lbg.KIND_BFS))
            ref.append(lbg.bfs(singles[i], int(s)).cpu().numpy())
            queries.append((int(nb[i] + s), int(nb[i]), int(nb[i + 1]), lbg.KIND_SSSP))
            ref.append(lbg.sssp(singles[i], int(s)).cpu().numpy())
    ws = lbg.Workspace("cuda")
    for _ in range(3):  # reused workspace, different relaxation orders
        out = lbg.batch_solve(dg, queries, workspace=ws).cpu().numpy()
        off = 0
        for q, r in zip(queries, ref):
            assert np.array_equal(out[off: off + q[2] - q[1]], r), f"query {q}"
            off += q[2] - q[1]


def test_batch_explicit_rows_and_gaps():
    g = graphgen.uniform(n=300, k=4, wlo=1, whi=9, salt=1)
    dg = lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights)
    out = torch.full((1000,), -5, dtype=torch.int32, device="cuda")
    lbg.batch_solve(dg, [(7, 0, 300, lbg.KIND_SSSP, 650), (3, 0, 300, lbg.KIND_BFS, 10)], out=out)
    o = out.cpu().numpy()
    assert np.array_equal(o[650:950], _expected(g, 7, lbg.KIND_SSSP))
    assert np.array_equal(o[10:310], _expected(g, 3, lbg.KIND_BFS))
    assert np.all(o[:10] == -5) and np.all(o[310:650] == -5) and np.all(o[950:] == -5)


def test_batch_rejects_arc_leaving_instance():
    # two "instances" declared, but an arc crosses from the first into the second
    g = graphgen.from_edges(6, [0, 1, 2, 3], [1, 2, 4, 5], [1, 1, 1, 1], "crossing")
    dg = lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights)
    with pytest.raises(lbg.LbgError) as ei:
        lbg.batch_solve(dg, [(0, 0, 3, lbg.KIND_BFS), (3, 3, 6, lbg.KIND_BFS)])
    assert ei.value.code == lbg.EOVERFLOW


def test_graph_launched_batch_replays():
    """The graph-launched batch (a cached HIP graph of 64 levels, replayed
    until the batch is done) gives the oracle's rows on every call: reused
    with eager work and synchronisations in between, rebuilt for other
    buffers, and agreeing with the eager batch, including batches longer
    than one replay (a 300-node path needs 300 levels)."""
    gs = _instances() + [pins.path_graph(300, np.arange(1, 300) % 5 + 1)]
    u, nb, _ = graphgen.pack(gs)
    dg = lbg.DeviceGraph.from_numpy(u.offsets, u.cols, u.weights)
    rng = np.random.default_rng(17)
    queries, expect = [], []
    for i, g in enumerate(gs):
        for s in rng.integers(0, g.n, 2):
            for kind in (lbg.KIND_BFS, lbg.KIND_SSSP):
                queries.append((int(nb[i] + s), int(nb[i]), int(nb[i + 1]), kind))
                expect.append(_expected(g, int(s), kind))
    ws = lbg.Workspace("cuda")
    rows = sum(q[2] - q[1] for q in queries)
    out = torch.empty(rows, dtype=torch.int32, device="cuda")
    eager = lbg.batch_solve(dg, queries, workspace=ws).cpu().numpy()
    for rep in range(4):
        out.fill_(-9)
        lbg.batch_solve(dg, queries, out=out, workspace=ws, graph=True)
        got = out.cpu().numpy()
        assert np.array_equal(got, eager), rep
        off = 0
        for q, e in zip(queries, expect):
            assert np.array_equal(got[off: off + q[2] - q[1]], e), (rep, q)
            off += q[2] - q[1]
        lbg.bfs(dg, int(queries[0][0]), workspace=lbg.Workspace("cuda"))  # eager work in between
        torch.cuda.synchronize()
    # other buffers: the cached graph must not be reused
    out2 = torch.empty(rows, dtype=torch.int32, device="cuda")
    got2 = lbg.batch_solve(dg, queries[::-1], out=out2, workspace=lbg.Workspace("cuda"), graph=True)
    got2 = got2.cpu().numpy()
    off = 0
    for q, e in zip(queries[::-1], expect[::-1]):
        assert np.array_equal(got2[off: off + q[2] - q[1]], e), q
        off += q[2] - q[1]


def test_full_size_batch_sampled_against_oracle():
    """The batched benchmark configuration at full size (256 instances, 4
    sources each, BFS and SSSP: 2,048 queries in one lbg_batch_solve call):
    16 queries spread over the instances, the largest included, are checked
    against the oracle on their own instance, bit for bit."""
    gs = graphgen.batch_instances(256, hi_exp=18)
    u, nb, eb = graphgen.pack(gs)
    dg = lbg.DeviceGraph.from_numpy(u.offsets, u.cols, u.weights)
    queries, owner = [], []
    for i, g in enumerate(gs):
        for s in graphgen.sources(g, 4, graphgen.FAMILY_BATCH, salt=i):
            for kind in (lbg.KIND_BFS, lbg.KIND_SSSP):
                queries.append((int(nb[i] + s), int(nb[i]), int(nb[i + 1]), kind))
                owner.append((i, int(s), kind))
    assert len(queries) == 2048
    out = lbg.batch_solve(dg, queries)
    starts = np.concatenate([[0], np.cumsum([q[2] - q[1] for q in queries])])
    biggest = max(range(len(gs)), key=lambda i: gs[i].m)
    pick = sorted(set(list(range(0, 2048, 137)) + [8 * biggest, 8 * biggest + 1]))
    for k in pick:
        i, s, kind = owner[k]
        row = out[int(starts[k]): int(starts[k + 1])].cpu().numpy()
        assert np.array_equal(row, _expected(gs[i], s, kind)), f"query {k} (instance {i}, src {s}, kind {kind})"
