"""Pins for the CPU oracle: checks against facts fixed independently of the
oracle's own code (brute force, closed forms, another library, the paper's
worked examples, an exactness certificate).  Each ``pin_*`` function takes an
``oracle.Oracle`` and returns a list of failure strings (empty = pass), so the
same pins run against the real oracle and against planted mutants."""
from __future__ import annotations

import os

import numpy as np

import graphgen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BFS_INF = 2**31 - 1
SSSP_INF = 2**32 - 1


# ----------------------------------------------------------------- inputs --
def tiny_graphs(count=60, seed=7):
    """Random tiny directed graphs with duplicates, self-loops, zero weights,
    isolated and unreachable parts."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(1, 40))
        m = int(rng.integers(0, 4 * n + 1))
        src = rng.integers(0, n, m)
        dst = rng.integers(0, n, m)
        if i % 5 == 0 and m:  # plant parallel arcs
            src = np.concatenate([src, src[: m // 3]])
            dst = np.concatenate([dst, dst[: m // 3]])
        w = rng.integers(0 if i % 4 == 0 else 1, 20, src.size)
        g = graphgen.from_edges(n, src, dst, w, name=f"tiny{i}")
        out.append((g, int(rng.integers(0, n))))
    return out


def path_graph(n, w):
    return graphgen.from_edges(n, np.arange(n - 1), np.arange(1, n), w, "path")


def clean_grid(k):
    """k x k 4-neighbour lattice, both directions, unit weights."""
    src, dst = [], []
    for r in range(k):
        for c in range(k):
            u = r * k + c
            if c + 1 < k:
                src += [u, u + 1]
                dst += [u + 1, u]
            if r + 1 < k:
                src += [u, u + k]
                dst += [u + k, u]
    return graphgen.from_edges(k * k, src, dst, None, "grid")


# ------------------------------------------------------------------- pins --
def pin_bruteforce(O):
    """Dijkstra and BFS agree with Bellman-Ford and Floyd-Warshall."""
    fails = []
    for g, s in tiny_graphs():
        d = O.dijkstra(g.offsets, g.cols, g.weights, s)
        bf = O.bellman_ford(g.offsets, g.cols, g.weights, s)
        fw = O.floyd_warshall(g.offsets, g.cols, g.weights)[s]
        if not (np.array_equal(d, bf) and np.array_equal(d, fw)):
            fails.append(f"{g.name}: dijkstra != brute force")
        unit = np.ones(g.m, dtype=np.uint32)
        lv = O.bfs(g.offsets, g.cols, s)
        bfu = O.bellman_ford(g.offsets, g.cols, unit, s)
        lv_as_u = np.where(lv == BFS_INF, SSSP_INF, lv).astype(np.uint32)
        if not np.array_equal(lv_as_u, bfu):
            fails.append(f"{g.name}: bfs != unit-weight Bellman-Ford")
    return fails


def pin_closed_forms(O):
    fails = []
    rng = np.random.default_rng(3)
    # path: d[i] = sum of the first i weights; levels = i
    n = 50
    w = rng.integers(1, 1000, n - 1)
    g = path_graph(n, w)
    exp = np.concatenate([[0], np.cumsum(w)]).astype(np.uint32)
    if not np.array_equal(O.dijkstra(g.offsets, g.cols, g.weights, 0), exp):
        fails.append("path: sssp")
    if not np.array_equal(O.bfs(g.offsets, g.cols, 0), np.arange(n, dtype=np.int32)):
        fails.append("path: bfs")
    # reversed source on a directed path: only the last node reachable
    lv = O.bfs(g.offsets, g.cols, n - 1)
    if not (lv[n - 1] == 0 and np.all(lv[:-1] == BFS_INF)):
        fails.append("path: unreachable")
    # star: centre 0 -> leaves; leaves at level 1, distance = own arc weight
    k = 30
    ws = rng.integers(1, 50, k)
    g = graphgen.from_edges(k + 1, np.zeros(k), np.arange(1, k + 1), ws, "star")
    if not np.array_equal(O.bfs(g.offsets, g.cols, 0), np.r_[0, np.ones(k)].astype(np.int32)):
        fails.append("star: bfs")
    if not np.array_equal(O.dijkstra(g.offsets, g.cols, g.weights, 0), np.r_[0, ws].astype(np.uint32)):
        fails.append("star: sssp")
    # clean grid, unit weights: Manhattan distance from the corner
    kk = 12
    g = clean_grid(kk)
    r, c = np.divmod(np.arange(kk * kk), kk)
    man = (r + c).astype(np.int32)
    if not np.array_equal(O.bfs(g.offsets, g.cols, 0), man):
        fails.append("grid: bfs")
    if not np.array_equal(O.dijkstra(g.offsets, g.cols, g.weights, 0), man.astype(np.uint32)):
        fails.append("grid: sssp")
    # complete digraph: everything at level 1; distance = direct arc when
    # weights make the direct arc shortest (w in [10, 19] < 2 * 10)
    n = 20
    s, t = np.nonzero(~np.eye(n, dtype=bool))
    wc = rng.integers(10, 20, s.size)
    g = graphgen.from_edges(n, s, t, wc, "complete")
    lv = O.bfs(g.offsets, g.cols, 5)
    if not (lv[5] == 0 and np.all(np.delete(lv, 5) == 1)):
        fails.append("complete: bfs")
    d = O.dijkstra(g.offsets, g.cols, g.weights, 5)
    direct = np.zeros(n, dtype=np.uint32)
    direct[t[s == 5]] = wc[s == 5]
    if not np.array_equal(d, direct):
        fails.append("complete: sssp")
    # binary out-tree: level of node i is floor(log2(i+1))
    n = 127
    ch = np.arange(1, n)
    g = graphgen.from_edges(n, (ch - 1) // 2, ch, None, "tree")
    exp = np.floor(np.log2(np.arange(n) + 1)).astype(np.int32)
    if not np.array_equal(O.bfs(g.offsets, g.cols, 0), exp):
        fails.append("tree: bfs")
    return fails


def _scipy_min_csr(g, unit=False):
    import scipy.sparse as sp

    src = g.coo_src()
    w = np.ones(g.m) if unit else g.weights.astype(np.float64)
    # parallel arcs: keep the minimum (csr_matrix would add them)
    key = src.astype(np.int64) * g.n + g.cols
    order = np.lexsort((w, key))
    key, w = key[order], w[order]
    first = np.r_[True, key[1:] != key[:-1]] if key.size else np.zeros(0, bool)
    key, w = key[first], w[first]
    return sp.csr_matrix((w, (key // g.n, key % g.n)), shape=(g.n, g.n))


def pin_scipy(O):
    """Cross-check against scipy.sparse.csgraph (float64 is exact here)."""
    from scipy.sparse.csgraph import dijkstra as sdij

    fails = []
    for g, srcs in ((graphgen.uniform(12), [0, 17, 999]),
                    (graphgen.rmat(12, edge_factor=8), None),
                    (graphgen.grid(40), [0, 801])):
        if srcs is None:
            srcs = list(graphgen.sources(g, 3, graphgen.FAMILY_RMAT))
        A = _scipy_min_csr(g)
        Au = _scipy_min_csr(g, unit=True)
        for s in srcs:
            ref = sdij(A, directed=True, indices=int(s))
            exp = np.where(np.isinf(ref), SSSP_INF, ref).astype(np.uint32)
            if not np.array_equal(O.dijkstra(g.offsets, g.cols, g.weights, s), exp):
                fails.append(f"{g.name} src {s}: sssp vs scipy")
            refu = sdij(Au, directed=True, indices=int(s))
            expu = np.where(np.isinf(refu), BFS_INF, refu).astype(np.int32)
            if not np.array_equal(O.bfs(g.offsets, g.cols, s), expu):
                fails.append(f"{g.name} src {s}: bfs vs scipy")
    return fails


def pin_certificate(O):
    """The certificate accepts exact distances and rejects every kind of
    perturbation (too small, too large, wrong reachability, wrong source)."""
    fails = []
    g = graphgen.uniform(10)
    s = 3
    d = O.dijkstra(g.offsets, g.cols, g.weights, s)
    lv = O.bfs(g.offsets, g.cols, s)
    if O.certificate(g.offsets, g.cols, g.weights, s, d)[0] != 0:
        fails.append("exact sssp rejected")
    if O.certificate(g.offsets, g.cols, None, s, lv)[0] != 0:
        fails.append("exact bfs rejected")
    reach = np.nonzero((d != SSSP_INF) & (np.arange(g.n) != s))[0]
    unreach = np.nonzero(d == SSSP_INF)[0]
    v = int(reach[len(reach) // 2])
    for label, mod in (("+1", lambda x: x.__setitem__(v, x[v] + 1)),
                       ("-1", lambda x: x.__setitem__(v, x[v] - 1)),
                       ("inf-on-reachable", lambda x: x.__setitem__(v, SSSP_INF)),
                       ("src-nonzero", lambda x: x.__setitem__(s, 1))):
        dd = d.copy()
        mod(dd)
        if O.certificate(g.offsets, g.cols, g.weights, s, dd)[0] == 0:
            fails.append(f"sssp perturbation {label} accepted")
    if unreach.size:
        dd = d.copy()
        dd[unreach[0]] = 5
        if O.certificate(g.offsets, g.cols, g.weights, s, dd)[0] == 0:
            fails.append("finite unreachable accepted")
    for delta in (1, -1):
        ll = lv.copy()
        ll[v] = ll[v] + delta
        if O.certificate(g.offsets, g.cols, None, s, ll)[0] == 0:
            fails.append(f"bfs perturbation {delta} accepted")
    # a tight-but-disconnected "island": two unreachable nodes that point at
    # each other with consistent finite labels must be rejected by (iii)
    h = graphgen.from_edges(4, [0, 2, 3], [1, 3, 2], [1, 1, 1], "island")
    dd = np.array([0, 1, 7, 8], dtype=np.uint32)
    if O.certificate(h.offsets, h.cols, h.weights, 0, dd)[0] == 0:
        fails.append("island accepted")
    # a too-large label on a node reachable through it: rejected by (ii)
    dd = np.array([0, 2, SSSP_INF, SSSP_INF], dtype=np.uint32)
    if O.certificate(h.offsets, h.cols, h.weights, 0, dd)[0] == 0:
        fails.append("relaxable arc accepted")
    return fails


def _read_kv(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


def pin_paper_examples(O):
    """Worked examples printed in the paper (tests/golden/*.txt)."""
    fails = []
    rows = _read_kv("wd_example.txt")
    i = rows.index(["nodes"])
    deg = [int(r[2]) for r in rows[i + 1: i + 3]]
    threads = int(dict((r[0], r[1]) for r in rows if len(r) == 2)["threads"])
    ept_exp = int(dict((r[0], r[1]) for r in rows if len(r) == 2)["edges_per_thread"])
    j = rows.index(["split"])
    split = np.array([[int(x) for x in r] for r in rows[j + 1: j + 1 + threads]])
    ept, node, edge = O.wd_offsets(deg, threads)
    if ept != ept_exp or not np.array_equal(node, split[:, 1]) or not np.array_equal(edge, split[:, 2]):
        fails.append(f"WD split: got ept={ept} node={node} edge={edge}")
    kv = {r[0]: r[1:] for r in _read_kv("hp_example.txt")}
    sizes = O.hp_schedule([int(x) for x in kv["degrees"]], int(kv["mdt"][0]))
    if list(sizes) != [int(x) for x in kv["sublist_sizes"]]:
        fails.append(f"HP schedule: got {list(sizes)}")
    one = O.hp_schedule([int(kv["single_degree"][0])], int(kv["single_mdt"][0]))
    if list(one) != [1] * int(kv["single_subiterations"][0]):
        fails.append(f"HP schedule of one node with {kv['single_degree'][0]} edges: got {list(one)}")
    kv = {r[0]: r[1:] for r in _read_kv("ns_example.txt")}
    pieces = O.ns_pieces(int(kv["degree"][0]), int(kv["mdt"][0]))
    if list(pieces) != [int(x) for x in kv["pieces"]]:
        fails.append(f"NS pieces: got {list(pieces)}")
    for name, maxdeg, tallest, mdt in _read_kv("mdt_example.txt"):
        maxdeg, tallest, mdt = int(maxdeg), int(tallest), int(mdt)
        # a degree population whose tallest 10-bin histogram bar is `tallest`
        width = maxdeg / 10.0
        lo = int(np.floor((tallest - 1) * width)) + 1
        hi = int(np.floor(tallest * width))
        degs = [maxdeg] + [lo] * 1000 + list(range(0, maxdeg + 1))
        degs += [min(max(lo, (lo + hi) // 2), hi)] * 50
        off = np.concatenate([[0], np.cumsum(degs)])
        got, hist = O.mdt(off, 10)
        if got != mdt or int(np.argmax(hist)) + 1 != tallest:
            fails.append(f"MDT {name}: got {got} (hist {hist.tolist()})")
    return fails


def pin_wd_split(O):
    """The block distribution of Section III-A hands every worklist edge to
    exactly one thread: the chunks [t*ept, (t+1)*ept) cover all E edges, and
    each thread's (node, edge offset) start names global edge t*ept."""
    fails = []
    rng = np.random.default_rng(11)
    for trial in range(200):
        cnt = int(rng.integers(0, 30))
        deg = rng.integers(0, 12, cnt)
        if trial % 7 == 0 and cnt:
            deg[0] = 200  # one hub
        T = int(rng.integers(1, 40))
        E = int(deg.sum())
        ept, node, edge = O.wd_offsets(deg, T)
        if T * ept < E:
            fails.append(f"trial {trial}: {T} threads x {ept} edges miss some of {E}")
            continue
        prefix = np.concatenate([[0], np.cumsum(deg)])
        for t in range(T):
            g = t * ept
            if g >= E:
                if node[t] != cnt:
                    fails.append(f"trial {trial}: idle thread {t} not past the end")
                continue
            k = int(node[t])
            if not (0 <= k < cnt and 0 <= edge[t] < deg[k] and prefix[k] + edge[t] == g):
                fails.append(f"trial {trial}: thread {t} start ({k},{edge[t]}) is not edge {g}")
        if len(fails) > 5:
            break
    return fails


ALL_PINS = [pin_bruteforce, pin_closed_forms, pin_scipy, pin_certificate, pin_paper_examples,
            pin_wd_split]


def run_all(O):
    fails = []
    for p in ALL_PINS:
        try:
            fails += [f"{p.__name__}: {f}" for f in p(O)]
        except Exception as e:  # a mutant may also crash a pin
            fails.append(f"{p.__name__}: raised {e!r}")
    return fails
