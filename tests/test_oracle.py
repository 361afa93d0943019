"""The CPU oracle against its pins (no GPU).  Each planted mutant of the
oracle must be caught by at least one pin, which shows the pins would notice
a dropped term, a wrong index or a wrong rounding in the oracle itself."""
import numpy as np
import pytest

import graphgen
import oracle
import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    fails = pin(orc)
    assert not fails, fails


# mutant number -> the pin family expected to catch it
MUTANTS = {
    1: "BFS level without +1",
    2: "Dijkstra skips a node's last arc",
    3: "Dijkstra uses the first arc's weight for every arc",
    4: "certificate skips the relaxation check",
    5: "certificate skips the tight-arc reachability check",
    6: "MDT with a 0-based bin index",
    7: "WD split with floor instead of ceil",
    8: "HP sublist keeps a node whose edges end on a window boundary",
}


@pytest.mark.parametrize("k", sorted(MUTANTS), ids=lambda k: MUTANTS[k])
def test_mutant_is_caught(k):
    fails = pins.run_all(oracle.mutant(k))
    assert fails, f"planted mistake {k} ({MUTANTS[k]}) passed every pin"


def test_invariants_rmat(orc):
    """Properties that hold at any size, on a skewed graph."""
    g = graphgen.rmat(14)
    s = int(graphgen.sources(g, 1, graphgen.FAMILY_RMAT)[0])
    lv = orc.bfs(g.offsets, g.cols, s)
    d = orc.dijkstra(g.offsets, g.cols, g.weights, s)
    src = g.coo_src()
    fin = lv[src] != pins.BFS_INF
    # symmetric graph: levels of arc endpoints differ by at most one
    assert np.all(np.abs(lv[src][fin].astype(np.int64) - lv[g.cols][fin]) <= 1)
    # SSSP reachability equals BFS reachability; hop count bounds distance
    assert np.array_equal(lv == pins.BFS_INF, d == pins.SSSP_INF)
    assert np.all(d[lv != pins.BFS_INF] >= lv[lv != pins.BFS_INF])
    assert np.all(d[lv != pins.BFS_INF] <= 255 * lv[lv != pins.BFS_INF].astype(np.int64))
    assert orc.certificate(g.offsets, g.cols, g.weights, s, d)[0] == 0
    assert orc.certificate(g.offsets, g.cols, None, s, lv)[0] == 0


def test_bad_input_rejected(orc):
    g = graphgen.uniform(6)
    with pytest.raises(ValueError):
        orc.bfs(g.offsets, g.cols, g.n)
    bad = g.cols.copy()
    bad[0] = g.n
    with pytest.raises(ValueError):
        orc.dijkstra(g.offsets, bad, g.weights, 0)


def test_overflow_detected(orc):
    # a path whose total weight does not fit below UINT32_MAX
    g = pins.path_graph(4, [2**31, 2**31, 5])
    with pytest.raises(ValueError):
        orc.dijkstra(g.offsets, g.cols, g.weights, 0)
