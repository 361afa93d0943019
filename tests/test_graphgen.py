"""Seeded input generators: determinism and the structural properties each
workload family promises (no GPU)."""
import numpy as np

import graphgen


def test_splitmix_reference_vector():
    # First outputs of SplitMix64 seeded with 1234567 (published test vector of
    # the reference implementation by Steele, Lea and Flood / Vigna).
    assert graphgen.splitmix_at(1234567, 0) == 6457827717110365317
    assert graphgen.splitmix_at(1234567, 1) == 3203168211198807973


def _csr_ok(g):
    off = g.offsets.astype(np.int64)
    assert off[0] == 0 and off[-1] == g.m and np.all(np.diff(off) >= 0)
    assert g.cols.min(initial=0) >= 0 and g.cols.max(initial=0) < g.n


def _symmetric_simple(g):
    src = g.coo_src().astype(np.int64)
    dst = g.cols.astype(np.int64)
    assert not np.any(src == dst), "self-loop"
    key = src * g.n + dst
    assert np.all(np.diff(key) > 0), "rows not sorted / duplicate arc"
    rkey = np.sort(dst * g.n + src)
    assert np.array_equal(key, rkey), "not symmetric"
    # one weight per undirected edge: arc (u,v) and arc (v,u) carry the same
    pos = np.searchsorted(key, dst * g.n + src)
    w_rev = g.weights[pos]
    assert np.array_equal(g.weights, w_rev), "asymmetric weights"


def test_uniform_config():
    g = graphgen.uniform(14)
    _csr_ok(g)
    assert g.n == 16384 and g.m <= 8 * g.n and g.m > 8 * g.n - 40
    src = g.coo_src()
    assert not np.any(src == g.cols), "self-loop kept"
    assert g.weights.min() >= 1 and g.weights.max() <= 100
    g2 = graphgen.uniform(14)
    assert np.array_equal(g.cols, g2.cols) and np.array_equal(g.weights, g2.weights)


def test_rmat_small_properties():
    g = graphgen.rmat(14)
    _csr_ok(g)
    _symmetric_simple(g)
    deg = g.degrees
    assert deg.max() > 20 * deg.mean(), "RMAT should be skewed"
    assert g.weights.min() >= 1 and g.weights.max() <= 255
    graphgen.set_threads(1)
    try:
        g1 = graphgen.rmat(14)
    finally:
        graphgen.set_threads(0)
    assert np.array_equal(g.offsets, g1.offsets) and np.array_equal(g.cols, g1.cols)
    assert np.array_equal(g.weights, g1.weights), "thread count changed the graph"


def test_grid_properties():
    g = graphgen.grid(64)
    _csr_ok(g)
    _symmetric_simple(g)
    assert g.degrees.max() <= 8
    h = graphgen.grid(64, shortcut_frac=0)
    _symmetric_simple(h)
    # without shortcuts every arc joins lattice neighbours
    src = h.coo_src()
    diff = np.abs(src.astype(np.int64) - h.cols)
    assert np.all((diff == 1) | (diff == 64))
    assert h.degrees.max() <= 4
    kept = h.m // 2
    assert abs(kept - 0.9 * (2 * 63 * 64)) < 0.05 * 2 * 63 * 64
    assert g.weights.max() <= 1000


def test_sources_nonisolated_distinct():
    g = graphgen.rmat(12)
    s = graphgen.sources(g, 64, graphgen.FAMILY_RMAT)
    assert s.size == 64 and np.unique(s).size == 64
    assert np.all(g.degrees[s] > 0)
