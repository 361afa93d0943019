"""GPU parity of balanced BFS with scan levels: a level of at least
lbg_set_bfs_scan_min() frontier arcs is expanded with plain level stores
(no claim atomics, no pushes) and the next worklist is built by a scan of
the levels array.  Every result is compared with the oracle's FIFO BFS at
every threshold (each level, the default n / 4, n / 8, never), over many
solves of one graph (the per-graph record of scan levels, including its
periodic re-check) and with graphs alternating on one thread (the record
is kept per graph)."""
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
NEVER = 1 << 40


@pytest.fixture(autouse=True)
def _default_threshold():
    yield
    lbg.set_bfs_scan_min(-1)


def _dev(g):
    return lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights)


def _graphs():
    return [("uniform14", graphgen.uniform(14), graphgen.FAMILY_UNIFORM),
            ("rmat16", graphgen.rmat(16), graphgen.FAMILY_RMAT),
            ("grid96", graphgen.grid(96), graphgen.FAMILY_GRID),
            ("rmat20", graphgen.rmat(20), graphgen.FAMILY_RMAT)]


@pytest.mark.parametrize("rule", ["every", "default", "n/8", "never"])
def test_scan_thresholds(rule):
    ws = lbg.Workspace()
    for name, g, fam in _graphs():
        lbg.set_bfs_scan_min({"every": 0, "default": -1, "n/8": g.n // 8, "never": NEVER}[rule])
        dg = _dev(g)
        for s in graphgen.sources(g, 3, fam):
            s = int(s)
            got, st = lbg.bfs(dg, s, workspace=ws, stats=True)
            assert np.array_equal(got.cpu().numpy(), O.bfs(g.offsets, g.cols, s)), (name, rule, s)
            if rule == "every" and not name.startswith("grid"):
                # low diameter: every level runs as a one-level launch, and
                # scans (the grid's long tail goes to the small-frontier
                # kernel, which claims)
                assert st["atomics"] < st["updates"], (name, st)
            if rule == "never":
                assert st["atomics"] >= st["updates"], (name, st)


def test_scan_record_over_many_solves():
    """33 solves of R-MAT 18 from different sources with the default
    threshold: the first and every 16th may scan at any level, the others
    only near the levels that scanned since."""
    g = graphgen.rmat(18)
    dg = _dev(g)
    ws = lbg.Workspace()
    srcs = graphgen.sources(g, 33, graphgen.FAMILY_RMAT)
    scanned = 0
    for s in srcs:
        s = int(s)
        got, st = lbg.bfs(dg, s, workspace=ws, stats=True)
        assert np.array_equal(got.cpu().numpy(), O.bfs(g.offsets, g.cols, s)), s
        scanned += st["atomics"] < st["updates"]
    assert scanned >= 16  # the big levels keep scanning


def test_scan_record_per_graph():
    """Two graphs solved alternately on one thread, plus a third graph of a
    different size, each result exact."""
    gs = [graphgen.rmat(17), graphgen.uniform(16), graphgen.grid(128)]
    fams = [graphgen.FAMILY_RMAT, graphgen.FAMILY_UNIFORM, graphgen.FAMILY_GRID]
    dgs = [_dev(g) for g in gs]
    ws = lbg.Workspace()
    srcs = [graphgen.sources(g, 6, f) for g, f in zip(gs, fams)]
    for k in range(6):
        for g, dg, ss in zip(gs, dgs, srcs):
            s = int(ss[k])
            assert np.array_equal(lbg.bfs(dg, s, workspace=ws).cpu().numpy(), O.bfs(g.offsets, g.cols, s))


def test_scan_setting_roundtrip():
    lbg.set_bfs_scan_min(12345)
    assert lbg.get_bfs_scan_min() == 12345
    lbg.set_bfs_scan_min(-7)
    assert lbg.get_bfs_scan_min() == -1
