"""Serving scheduler on the CPU: admission by slots / rows / upload regions,
FCFS order, resource reuse, Poisson replay and result identity, with a fake
engine whose 'kernels' are the CPU oracle (no GPU)."""
import time

import numpy as np
import pytest

import graphgen
import oracle
from paper_1711_00231_amd import serve

torch = pytest.importorskip("torch")
O = oracle.get()


class _Rows:
    def __init__(self, n):
        self.a = np.full(n, -1, dtype=np.int32)

    def __getitem__(self, sl):
        return torch.from_numpy(self.a[sl])


class FakeEngine:
    """Engine stand-in: a query finishes `lag` steps after it was submitted
    (more for bigger instances); its row is then the oracle's answer on the
    packed graph restricted to its instance."""

    def __init__(self, packed, max_queries, max_rows, lag=2):
        self.g = packed
        self.max_queries, self.max_rows = max_queries, max_rows
        self.rows = _Rows(max_rows)
        self.slots = {}
        self.lag = lag
        self.tick = 0
        self.max_inflight = 0

    def submit(self, src, lo, hi, kind, out_off):
        if len(self.slots) >= self.max_queries:
            return -1
        for (s2, lo2, hi2, k2, o2, t2) in self.slots.values():  # rows never overlap
            assert out_off + hi - lo <= o2 or o2 + hi2 - lo2 <= out_off
        slot = min(set(range(self.max_queries)) - set(self.slots))
        self.slots[slot] = (src, lo, hi, kind, out_off, self.tick)
        self.max_inflight = max(self.max_inflight, len(self.slots))
        return slot

    def step(self, levels=1):
        self.tick += 1
        done = []
        for slot, (src, lo, hi, kind, off, t) in list(self.slots.items()):
            if self.tick - t >= self.lag + (hi - lo) // 2000:
                sub_off = self.g.offsets[lo: hi + 1].astype(np.int64)
                base = sub_off[0]
                cols = self.g.cols[base: sub_off[-1]] - lo
                w = self.g.weights[base: sub_off[-1]]
                sub = sub_off - base
                if kind == serve.KIND_BFS:
                    r = O.bfs(sub, cols, src - lo)
                else:
                    r = O.dijkstra(sub, cols, w, src - lo).view(np.int32)
                self.rows.a[off: off + hi - lo] = r
                done.append(slot)
                self.slots[slot] = self.slots[slot] + ("done",)
        return done

    def release(self, slot):
        assert len(self.slots[slot]) == 7, "released before finishing"
        del self.slots[slot]


def _setup():
    gs = [graphgen.uniform(n=3000, k=6, wlo=1, whi=50, salt=1), graphgen.rmat(11, salt=2),
          graphgen.grid(40, salt=3)]
    u, nb, eb = graphgen.pack(gs)
    inst = {f"g{i}": serve.Instance(int(nb[i]), int(nb[i + 1]), int(eb[i + 1] - eb[i]))
            for i in range(len(gs))}
    return gs, u, inst


def _check_results(report, gs):
    for r in report.completed:
        g = gs[int(r.instance[1:])]
        exp = O.bfs(g.offsets, g.cols, r.src) if r.kind == serve.KIND_BFS else \
            O.dijkstra(g.offsets, g.cols, g.weights, r.src).view(np.int32)
        assert np.array_equal(r.result, exp), r.rid


def test_row_allocator():
    a = serve.RowAllocator(100)
    x, y, z = a.alloc(30), a.alloc(30), a.alloc(30)
    assert (x, y, z) == (0, 30, 60) and a.alloc(20) is None
    a.release(30, 30)
    assert a.alloc(40) is None and a.alloc(25) == 30
    a.release(0, 30)
    a.release(30, 25)
    a.release(60, 30)
    assert a.free == [(0, 100)] and a.in_use == 0


def test_replay_all_complete_fcfs_and_identical():
    gs, u, inst = _setup()
    eng = FakeEngine(u, max_queries=4, max_rows=6000)
    reqs = serve.poisson_requests(1e4, 60, inst, seed=5)
    rep = serve.Server(eng, inst, keep_results=True).run(reqs, replay=True)
    assert len(rep.completed) == 60
    adm = [r.admitted for r in sorted(rep.completed, key=lambda r: r.rid)]
    assert adm == sorted(adm), "admission is first-come first-served"
    assert eng.max_inflight <= 4 and not eng.slots
    _check_results(rep, gs)
    s = rep.summary()
    assert s["requests"] == 60 and s["p99_ms"] >= s["p50_ms"] >= 0


def test_capacity_blocks_but_never_starves():
    gs, u, inst = _setup()
    # rows for only one big instance at a time
    eng = FakeEngine(u, max_queries=8, max_rows=3100)
    reqs = serve.poisson_requests(1e5, 25, inst, seed=9)
    rep = serve.Server(eng, inst, keep_results=True).run(reqs, replay=True)
    assert len(rep.completed) == 25
    _check_results(rep, gs)


def test_too_large_request_rejected_others_served():
    gs, u, inst = _setup()
    small = min(inst, key=lambda k: inst[k].hi - inst[k].lo)
    big = max(inst, key=lambda k: inst[k].hi - inst[k].lo)
    eng = FakeEngine(u, max_queries=2, max_rows=inst[small].hi - inst[small].lo)
    reqs = [serve.Request(0, 0.0, serve.KIND_BFS, big, 0),
            serve.Request(1, 0.0, serve.KIND_SSSP, small, 3)]
    rep = serve.Server(eng, inst, keep_results=True).run(reqs, replay=True)
    assert [r.rid for r in rep.dropped] == [0] and rep.dropped[0].status == "rejected"
    assert [r.rid for r in rep.completed] == [1] and rep.completed[0].status == "done"
    _check_results(rep, gs)
    assert rep.summary()["rejected"] == 1


def test_engine_without_slots_raises():
    gs, u, inst = _setup()
    eng = FakeEngine(u, max_queries=0, max_rows=10000)
    with pytest.raises(RuntimeError, match="never be admitted"):
        serve.Server(eng, inst).run([serve.Request(0, 0.0, serve.KIND_BFS, "g0", 0)], replay=True)


class _Clock:
    """Deterministic clock: advances by `dt` at every reading."""

    def __init__(self, dt):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        self.t += self.dt
        return self.t


def test_admission_timeout_drops_waiting_requests():
    gs, u, inst = _setup()
    # one slot; every query holds it for `lag` steps, so later requests wait
    eng = FakeEngine(u, max_queries=1, max_rows=10000, lag=5)
    reqs = [serve.Request(i, 0.0, serve.KIND_BFS, "g2", i) for i in range(6)]
    reqs[5].timeout = 1e9  # its own timeout overrides the server's
    srv = serve.Server(eng, inst, keep_results=True, timeout=0.05)
    rep = srv.run(reqs, replay=True, clock=_Clock(0.004))
    done = sorted(r.rid for r in rep.completed)
    late = sorted(r.rid for r in rep.dropped)
    assert 0 in done and 5 in done and late and set(done) | set(late) == set(range(6))
    for r in rep.dropped:
        assert r.status == "timeout" and r.done - r.arrival > 0.05 and r.admitted < 0
    for r in rep.completed:
        assert r.admitted - r.arrival <= 0.05 or r.rid == 5
    _check_results(rep, gs)
    assert not eng.slots and srv.rows.in_use == 0


def test_cancel_queued_and_running():
    gs, u, inst = _setup()

    class CancellingEngine(FakeEngine):
        def step(self, levels=1):
            if self.tick == 0:
                srv.cancel(0)   # running by now
                srv.cancel(3)   # still queued
                srv.cancel(99)  # unknown ids are ignored
            return super().step(levels)

    eng = CancellingEngine(u, max_queries=2, max_rows=10000, lag=3)
    reqs = [serve.Request(i, 0.0, serve.KIND_SSSP, "g1", i) for i in range(5)]
    srv = serve.Server(eng, inst, keep_results=True)
    rep = srv.run(reqs, replay=True)
    by = {r.rid: r for r in rep.completed + rep.dropped}
    assert by[0].status == "cancelled" and by[0].admitted >= 0 and by[0].result is None
    assert by[3].status == "cancelled" and by[3].admitted < 0
    assert sorted(r.rid for r in rep.completed) == [1, 2, 4]
    _check_results(rep, gs)
    assert not eng.slots and srv.rows.in_use == 0
    assert rep.summary()["cancelled"] == 2


def test_upload_larger_than_region_rejected():
    gs, u, inst = _setup()

    class Arena:
        node_cap, arc_cap = 100, 400

    g = graphgen.uniform(n=500, k=4, salt=7)
    eng = FakeEngine(u, max_queries=2, max_rows=10000)
    srv = serve.Server(eng, inst, upload=Arena())
    rep = srv.run([serve.Request(0, 0.0, serve.KIND_BFS, None, 0, graph=g)], replay=True)
    assert rep.dropped[0].status == "rejected" and not rep.completed


def test_wall_clock_arrivals():
    gs, u, inst = _setup()
    eng = FakeEngine(u, max_queries=4, max_rows=8000)
    reqs = serve.poisson_requests(400.0, 12, inst, seed=2)
    rep = serve.Server(eng, inst).run(reqs)
    assert len(rep.completed) == 12
    assert all(r.done >= r.arrival and r.admitted >= r.arrival - 1e-9 for r in rep.completed)


def test_upload_region_layout_matches_graph():
    """A graph loaded into an upload region of the packed CSR has exactly its
    own BFS/SSSP answers on [lo, lo + n') (CPU tensors stand in for HBM)."""
    from paper_1711_00231_amd.serve import UploadArena

    base = graphgen.rmat(9, salt=4)
    NC, MC, R = 600, 4000, 3
    off_e, cols_e, w_e = UploadArena.empty_arrays(R, NC, MC, base.n, base.m)
    p_off = np.concatenate([base.offsets[:-1].astype(np.int64), off_e, [base.m + R * MC]])
    p_cols = np.concatenate([base.cols, cols_e])
    p_w = np.concatenate([base.weights, w_e])

    class DG:  # minimal device-graph stand-in on the CPU
        offsets = torch.from_numpy(p_off.astype(np.int32))
        cols = torch.from_numpy(p_cols.astype(np.int32))
        weights = torch.from_numpy(p_w.view(np.int32))

    arena = UploadArena(DG, base.n, base.m, R, NC, MC)
    arena.warm()  # loads a tiny graph into a free region and frees it again
    assert arena.free == list(range(R))
    O.bfs(DG.offsets.numpy().astype(np.int64), DG.cols.numpy(), 0)  # packed CSR still valid
    for salt, region in ((1, arena.acquire()), (2, arena.acquire()), (3, 0)):
        g = graphgen.uniform(n=450 + 40 * salt, k=7, wlo=1, whi=30, salt=salt)
        lo, hi, arcs = arena.load(region, g)
        po = DG.offsets.numpy().astype(np.int64)
        assert np.all(np.diff(po) >= 0) and po[-1] == len(p_cols)
        sub = po[lo: hi + 1] - po[lo]
        sc = DG.cols.numpy()[po[lo]: po[hi]] - lo
        sw = DG.weights.numpy().view(np.uint32)[po[lo]: po[hi]]
        for s in (0, 17):
            assert np.array_equal(O.bfs(sub, sc, s), O.bfs(g.offsets, g.cols, s))
            assert np.array_equal(O.dijkstra(sub, sc, sw, s), O.dijkstra(g.offsets, g.cols, g.weights, s))
        # the whole packed graph stays valid (oracle rejects bad CSR)
        O.bfs(po, DG.cols.numpy(), 0)


def test_plain_lane_takes_large_instances():
    """Queries on instances at or above big_arcs go to the plain lane (a
    worker thread), the rest to the batched engine; all complete with the
    oracle's answers, whichever path served them."""
    gs, u, inst = _setup()
    big = max(inst, key=lambda k: inst[k].arcs)

    def solve(r, keep):
        g = gs[int(r.instance[1:])]
        if r.kind == serve.KIND_BFS:
            return O.bfs(g.offsets, g.cols, r.src)
        return O.dijkstra(g.offsets, g.cols, g.weights, r.src).view(np.int32)

    lane = serve.PlainLane(solve, big_arcs=inst[big].arcs)
    eng = FakeEngine(u, max_queries=3, max_rows=6000)
    reqs = serve.poisson_requests(1e4, 50, inst, seed=13)
    rep = serve.Server(eng, inst, keep_results=True, plain=lane).run(reqs, replay=True)
    assert len(rep.completed) == 50 and not eng.slots
    _check_results(rep, gs)
    via_lane = [r for r in rep.completed if r.slot < 0]
    assert via_lane and all(r.instance == big for r in via_lane)
    assert all(r.instance != big for r in rep.completed if r.slot >= 0)
    assert all(r.done >= r.admitted for r in rep.completed)  # replay admits ahead of arrival


def test_plain_lane_workers_overlap():
    """A lane with three workers runs queries at once (each worker its own
    solver), and every result is the oracle's."""
    import threading

    gs, u, inst = _setup()
    lock = threading.Lock()
    running, peak = [0], [0]

    def make(k):
        def solve(r, keep):
            with lock:
                running[0] += 1
                peak[0] = max(peak[0], running[0])
            time.sleep(0.01)
            g = gs[int(r.instance[1:])]
            res = (O.bfs(g.offsets, g.cols, r.src) if r.kind == serve.KIND_BFS
                   else O.dijkstra(g.offsets, g.cols, g.weights, r.src).view(np.int32))
            with lock:
                running[0] -= 1
            return res
        return solve

    lane = serve.PlainLane([make(k) for k in range(3)], big_arcs=0)
    assert lane.workers == 3
    eng = FakeEngine(u, max_queries=2, max_rows=6000)
    reqs = serve.poisson_requests(1e4, 24, inst, seed=17)
    rep = serve.Server(eng, inst, keep_results=True, plain=lane).run(reqs, replay=True)
    assert len(rep.completed) == 24 and all(r.slot < 0 for r in rep.completed)
    _check_results(rep, gs)
    assert peak[0] >= 2  # queries overlapped


def test_plain_lane_extra_workers_wait_for_a_backlog():
    """Spaced arrivals (each solve ends before the next request arrives)
    never build a queue, so the lane's extra workers never start one: the
    queries run one at a time, as in a plain FCFS queue."""
    import threading

    gs, u, inst = _setup()
    lock = threading.Lock()
    running, peak = [0], [0]

    def make(k):
        def solve(r, keep):
            with lock:
                running[0] += 1
                peak[0] = max(peak[0], running[0])
            time.sleep(0.005)
            with lock:
                running[0] -= 1
            return None
        return solve

    lane = serve.PlainLane([make(k) for k in range(3)], big_arcs=0)
    eng = FakeEngine(u, max_queries=2, max_rows=6000)
    reqs = serve.poisson_requests(1e4, 8, inst, seed=19)
    for i, r in enumerate(reqs):
        r.arrival = 0.05 * i
    rep = serve.Server(eng, inst, plain=lane).run(reqs)
    assert len(rep.completed) == 8 and peak[0] == 1


def test_engine_yields_to_a_busy_plain_lane():
    """engine_yield: while a (slow) plain solve runs, the engine takes no
    step until its query was admitted that long ago; without it the engine
    steps at once.  Results are exact either way."""
    import threading

    gs, u, inst = _setup()
    plain_running = threading.Event()

    def slow(r, keep):
        plain_running.set()
        time.sleep(0.06)
        plain_running.clear()
        return None

    def first_step_delay(yield_s):
        eng = FakeEngine(u, max_queries=4, max_rows=6000, lag=1)
        seen = {}
        step0 = eng.step

        def step(levels=1):
            if plain_running.is_set() and "t" not in seen:
                seen["t"] = time.perf_counter()
            return step0(levels)
        eng.step = step
        lane = serve.PlainLane(slow, big_arcs=inst["g1"].arcs)  # R-MAT 11, the largest: plain lane
        reqs = serve.poisson_requests(1e4, 2, inst, seed=5)
        reqs[0].instance, reqs[0].src, reqs[0].arrival = "g1", 0, 0.0
        reqs[1].instance, reqs[1].src, reqs[1].arrival = "g2", 0, 0.01  # the grid: engine
        t0 = time.perf_counter()
        rep = serve.Server(eng, inst, plain=lane, keep_results=True, engine_yield=yield_s).run(reqs)
        assert len(rep.completed) == 2
        _check_results(type(rep)(completed=[r for r in rep.completed if r.instance == "g2"]), gs)
        return seen.get("t", float("inf")) - t0

    assert first_step_delay(0.0) < 0.03        # steps beside the plain solve
    assert first_step_delay(0.03) >= 0.035     # waits until its query is 30 ms old


def test_plain_lane_warms_each_worker_before_the_clock():
    """A solver's warm hook runs once, on its own worker thread, before the
    server's clock starts and before the worker takes any query."""
    import threading

    gs, u, inst = _setup()
    log = []
    lock = threading.Lock()

    def make(k):
        def solve(r, keep):
            with lock:
                log.append(("solve", k, threading.get_ident(), time.perf_counter()))
            return None

        def warm():
            with lock:
                log.append(("warm", k, threading.get_ident(), time.perf_counter()))
            time.sleep(0.02)
        solve.warm = warm
        return solve

    lane = serve.PlainLane([make(k) for k in range(3)], big_arcs=0)
    eng = FakeEngine(u, max_queries=2, max_rows=6000)
    reqs = serve.poisson_requests(1e4, 12, inst, seed=23)
    t_before = time.perf_counter()
    serve.Server(eng, inst, plain=lane).run(reqs)
    warms = [e for e in log if e[0] == "warm"]
    solves = [e for e in log if e[0] == "solve"]
    assert sorted(e[1] for e in warms) == [0, 1, 2]
    assert len(solves) == 12
    assert min(e[3] for e in solves) > max(e[3] for e in warms) >= t_before
    thread_of = {e[1]: e[2] for e in warms}
    assert all(thread_of[e[1]] == e[2] for e in solves)  # same thread as its warm-up
    # a lane prepared and stopped without a run shuts down cleanly
    lane2 = serve.PlainLane([make(k) for k in range(2)], big_arcs=0)
    lane2.prepare()
    lane2.stop()


def test_plain_lane_error_surfaces():
    gs, u, inst = _setup()

    def solve(r, keep):
        raise ValueError("solver failed")

    lane = serve.PlainLane(solve, big_arcs=0)  # everything resident goes to the lane
    eng = FakeEngine(u, max_queries=2, max_rows=6000)
    reqs = serve.poisson_requests(1e4, 5, inst, seed=3)
    with pytest.raises(ValueError, match="solver failed"):
        serve.Server(eng, inst, plain=lane).run(reqs, replay=True)


def test_plain_lane_skips_cancelled_requests():
    """A request cancelled while it waits in the plain lane's queue is never
    solved; the lane's queue keeps its order for the rest."""
    import threading

    gs, u, inst = _setup()
    gate = threading.Event()
    solved = []

    def solve(r, keep):
        if r.rid == 0:
            gate.wait(10)  # hold the lane until the cancels are in
        solved.append(r.rid)
        g = gs[int(r.instance[1:])]
        return O.bfs(g.offsets, g.cols, r.src)

    lane = serve.PlainLane(solve, big_arcs=0)
    eng = FakeEngine(u, max_queries=2, max_rows=6000)
    reqs = [serve.Request(i, 0.0, serve.KIND_BFS, "g0", i) for i in range(4)]
    srv = serve.Server(eng, inst, keep_results=True, plain=lane)

    def cancel_then_release():
        srv.cancel(2)
        import time
        time.sleep(0.05)  # the loop applies the cancel on its next pass
        gate.set()

    threading.Thread(target=cancel_then_release).start()
    rep = srv.run(reqs, replay=True)
    assert solved == [0, 1, 3]
    assert sorted(r.rid for r in rep.completed) == [0, 1, 3]
    assert [(r.rid, r.status) for r in rep.dropped] == [(2, "cancelled")]
    _check_results(rep, gs)


def _oracle_solve(gs):
    def solve(r, keep):
        g = gs[int(r.instance[1:])]
        if r.kind == serve.KIND_BFS:
            return O.bfs(g.offsets, g.cols, r.src)
        return O.dijkstra(g.offsets, g.cols, g.weights, r.src).view(np.int32)
    return solve


@pytest.mark.parametrize("bypass", [False, True])
def test_idle_bypass_only_when_everything_is_idle(bypass):
    """With idle_bypass, the first of a burst (engine and lane idle) goes to
    the plain lane and most of the rest are batched; without it, small
    instances never leave the engine.  Results are the oracle's either way."""
    gs, u, inst = _setup()
    lane = serve.PlainLane(_oracle_solve(gs), big_arcs=1 << 40)  # nothing is big
    eng = FakeEngine(u, max_queries=4, max_rows=12000)
    reqs = serve.poisson_requests(1e4, 12, inst, seed=21)
    rep = serve.Server(eng, inst, keep_results=True, plain=lane, idle_bypass=bypass).run(reqs, replay=True)
    assert len(rep.completed) == 12 and not eng.slots
    _check_results(rep, gs)
    by = [r for r in rep.completed if r.bypass]
    assert [r.slot < 0 for r in rep.completed] == [r.bypass for r in rep.completed]
    if bypass:
        # the burst's first request finds everything idle; while the lane or
        # the engine is busy the others are batched (a later one may again
        # find both idle while it waits for engine capacity)
        assert by[0].rid == reqs[0].rid and len(by) < len(reqs) // 2
        assert rep.summary()["bypassed"] == len(by)
    else:
        assert not by and "bypassed" not in rep.summary()


def test_idle_bypass_on_spaced_arrivals_and_names():
    """Arrivals far apart find everything idle, so each one on an instance the
    lane holds is bypassed; instances the lane does not hold stay batched."""
    gs, u, inst = _setup()
    lane = serve.PlainLane(_oracle_solve(gs), big_arcs=1 << 40, names=["g0", "g2"])
    eng = FakeEngine(u, max_queries=4, max_rows=12000)
    reqs = [serve.Request(i, 0.1 * i, serve.KIND_BFS if i % 2 else serve.KIND_SSSP, f"g{i % 3}", 5 + i)
            for i in range(9)]
    rep = serve.Server(eng, inst, keep_results=True, plain=lane, idle_bypass=True).run(reqs)
    assert len(rep.completed) == 9
    _check_results(rep, gs)
    for r in rep.completed:
        assert r.bypass == (r.instance != "g1"), (r.rid, r.instance)


def test_bypass_modes():
    """'lane' bypasses whenever the lane is idle, even with queries in the
    engine; an unknown mode is refused."""
    gs, u, inst = _setup()
    lane = serve.PlainLane(_oracle_solve(gs), big_arcs=1 << 40)
    eng = FakeEngine(u, max_queries=4, max_rows=12000)
    srv = serve.Server(eng, inst, keep_results=True, plain=lane, idle_bypass="lane")
    srv.inflight[0] = object()  # pretend the engine is busy
    assert srv._bypass(serve.Request(0, 0.0, serve.KIND_BFS, "g0", 1))
    srv.idle_bypass = "idle"
    assert not srv._bypass(serve.Request(0, 0.0, serve.KIND_BFS, "g0", 1))
    with pytest.raises(ValueError, match="idle_bypass"):
        serve.Server(eng, inst, plain=lane, idle_bypass="always")
