#!/usr/bin/env python3
"""Benchmark: level-synchronous BFS and SSSP on one MI355X.

Default workload: R-MAT scale 22, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05),
relabelled, symmetrised, duplicates and self-loops removed (n = 4,194,304,
m = 128,307,136 arcs), uint32 weights U[1,255], 64 seeded non-isolated
sources.  One step = BFS then SSSP from each of `--sources-per-step` sources
(cycling through the 64) through the C ABI, graph resident in HBM.

value: GTEPS = arcs leaving reached nodes (the CSR arcs a traversal scans)
per second of wall time, summed over the step's BFS and SSSP solves; the
Graph500-style figure (half of that on a symmetrised graph) is printed beside.

roofline: the dominant frontier-expansion kernel's algorithmic bytes per
launch over its average launch duration, timed live with HIP events on the
stream it runs on, against 8 TB/s HBM.  Algorithmic bytes:
  BFS  8 B per arc scanned (column id + destination state) + 20 B per node
       discovered (two offsets, level write, worklist write and read);
  SSSP 12 B per arc loaded and relaxed (column id, weight, destination
       distance) + 4 B per successful update + 20 B per worklist entry; the
       arcs of entries skipped at staging (their node improved again in the
       same iteration, so they are relaxed in the next one) are never loaded
       and are not charged (the library counts them: edges_skipped).

cpu_baseline: the CPU oracle (queue BFS + binary-heap Dijkstra) on a bounded
sample of the same sources: all host cores at once (value, cores = threads
used) and a single-thread leg (per-source medians), with the host's core
count and CPU model.

extra objects on the same line (--no-extras skips them; --mode batch /
--mode serve run the full batched and serving sweeps alone):
  strategies: node- vs edge-based vs hierarchical vs balanced vs degree-
  binned vs destination-sliced vs split-graph solves on the same graph.
  grid: the 2048x2048 high-diameter grid (1 % shortcuts) and its
  no-shortcut companion, BFS and SSSP from 4 of the 16 seeded sources.
  batched: 256 instances of uneven size (n up to 2^18), 4 sources each,
  BFS + SSSP: the 2,048 solves as one lbg_batch_solve call vs one plain call
  per query.
  serving: resident R-MAT 20/22/24 plus per-request uploaded uniform graphs;
  a Poisson stream of BFS/SSSP requests (70/30) served with continuous
  batching (overlapping plain solves for the large instances, the engine
  for the rest) and, at 0.5x, with every resident instance in the engine;
  p50/p99 latency beside the same arrivals served FCFS by plain per-query
  launches, at fractions of the plain saturation rate.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "BFS/SSSP GTEPS on RMAT s22, % HBM roofline; batched vs plain; p99 ms"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    import graphgen

    if name == "rmat22":
        g = graphgen.rmat(22)
        srcs = graphgen.sources(g, 64, graphgen.FAMILY_RMAT)
        desc = ("R-MAT scale 22, edge factor 16, a=.57 b=.19 c=.19 d=.05, symmetrised, "
                "deduplicated, uint32 weights U[1,255], 64 seeded non-isolated sources")
        sym = True
    elif name == "uniform14":
        g = graphgen.uniform(14)
        srcs = np.array([0], dtype=np.int32)
        desc = "uniform random digraph n=2^14, 8 out-arcs per node, weights U[1,100], source 0"
        sym = False
    elif name == "grid2048":
        g = graphgen.grid(2048)
        srcs = graphgen.sources(g, 16, graphgen.FAMILY_GRID)
        desc = ("2048x2048 4-neighbour grid, 10% edges dropped, 1% random shortcuts, "
                "symmetrised, weights U[1,1000], 16 seeded sources")
        sym = True
    elif name == "grid2048-noshortcut":
        g = graphgen.grid(2048, shortcut_frac=0)
        srcs = graphgen.sources(g, 16, graphgen.FAMILY_GRID)
        desc = "2048x2048 4-neighbour grid, 10% edges dropped, no shortcuts, weights U[1,1000]"
        sym = True
    else:
        raise SystemExit(f"unknown workload {name}")
    return g, srcs, desc, sym


# Sources whose text decides the expansion kernels' memory traffic: the
# kernels, the host code that launches them and the ordered-copy builder
# (the SSSP layout the benchmark times).
TRAFFIC_SOURCES = ("paper_1711_00231_amd/csrc/lbg_kernels.hpp", "paper_1711_00231_amd/csrc/lbg_device.hpp",
                   "paper_1711_00231_amd/csrc/lbg_sliced.hpp", "paper_1711_00231_amd/csrc/lbg_order.hpp",
                   "paper_1711_00231_amd/csrc/lbg.hip")


def recorded_traffic():
    """HBM-side bytes per launch of the expansion kernels, from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary; empty when the kernel sources
    have changed since those counters were taken."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    out = {}
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_hbm_traffic.txt")):
        lines = open(path).read().splitlines()
        if f"kernel_sources_sha256: {h.hexdigest()}" not in lines:
            continue
        for ln in lines:
            if ln.startswith("traffic_per_launch "):
                name, val = ln[len("traffic_per_launch "):].rsplit(":", 1)
                out[name.strip()] = float(val)
    return out


def algorithmic_bytes(kind, prof):
    if kind == "bfs":
        return 8 * prof["edges_scanned"] + 20 * prof["updates"]
    loaded = prof["edges_scanned"] - prof.get("edges_skipped", 0)
    return 12 * loaded + 4 * prof["updates"] + 20 * prof["frontier_entries"]


def hmean_gteps(times_ms, arcs):
    """Harmonic mean over solves of arcs / time (the Graph500 convention for
    a set of sources), in GTEPS: len / sum(time_i / arcs_i)."""
    if not len(times_ms):
        return None
    return len(times_ms) / sum((t / 1e3) / max(int(a), 1) for t, a in zip(times_ms, arcs)) / 1e9


def host_info():
    """Cores this process may run on and the CPU model, read on the machine
    that runs the benchmark."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": cores, "cpu_os_count": os.cpu_count(), "cpu_model": model}


def cpu_baseline(g, srcs, budget_s):
    """The CPU oracle (FIFO BFS + binary-heap Dijkstra, C, -O2) on the same
    workload, as a baseline only: (1) single thread, source after source
    until half the budget is spent: per-source median ms and the harmonic
    mean of per-source GTEPS; (2) all host cores: one source per thread,
    as many sources as there are cores, run at once (the oracle's C calls
    release the interpreter lock): aggregate GTEPS.  `value` is (2)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    O = oracle.get()
    deg = g.degrees
    info = host_info()

    def one(s):
        t0 = time.perf_counter()
        lv = O.bfs(g.offsets, g.cols, int(s))
        t1 = time.perf_counter()
        O.dijkstra(g.offsets, g.cols, g.weights, int(s))
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, int(deg[lv != np.iinfo(np.int32).max].sum())

    bfs_t, sssp_t, rates = [], [], []
    spent = 0.0
    for s in srcs:
        tb, ts, arcs = one(s)
        bfs_t.append(tb)
        sssp_t.append(ts)
        rates += [arcs / tb / 1e9, arcs / ts / 1e9]
        spent += tb + ts
        if spent >= budget_s / 2:
            break
    used1 = len(bfs_t)
    threads = max(1, info["nproc"])
    batch = [srcs[(used1 + k) % len(srcs)] for k in range(threads)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, batch))
    wall = time.perf_counter() - t0
    arcs_all = 2 * sum(r[2] for r in res)
    return {"value": round(arcs_all / wall / 1e9, 5), "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "sample": f"{threads} sources of the same workload at once, one per thread, BFS + Dijkstra each "
                      f"({wall:.1f} s wall); single-thread leg: {used1} source(s) one after another "
                      f"({spent:.1f} s)",
            "single_thread": {"sources": used1,
                              "bfs_ms_p50": round(float(np.median(bfs_t)) * 1e3, 2),
                              "sssp_ms_p50": round(float(np.median(sssp_t)) * 1e3, 2),
                              "gteps_hmean": round(len(rates) / sum(1.0 / r for r in rates), 5)},
            "host": info}


# ---------------------------------------------------------------- plain --
def run_plain(args, lbg, torch, dev):
    t0 = time.perf_counter()
    g, srcs, desc, sym = make_workload(args.workload)
    log(f"workload {g.name}: n={g.n} m={g.m} built in {time.perf_counter() - t0:.1f}s")
    dg = lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights, device=dev,
                                    with_coo=(args.strategy in ("edge", "edge_nochunk")),
                                    with_slices=(args.strategy == "sliced"))
    ws = lbg.Workspace(dev)
    lv_out = torch.empty(g.n, dtype=torch.int32, device=dev)
    d_out = torch.empty(g.n, dtype=torch.int32, device=dev)
    deg = torch.from_numpy(g.degrees).to(dev)
    # SSSP on the degree-class ordered copy (balanced strategy): built once
    # per graph before timing, like the CSR itself
    ordered = args.sssp_layout == "ordered" and args.strategy in ("balanced", "auto")
    order_ms = None
    if ordered:
        torch.cuda.synchronize()
        t = time.perf_counter()
        dg.ensure_ordered()
        torch.cuda.synchronize()
        order_ms = (time.perf_counter() - t) * 1e3
        log(f"degree-class ordered copy built in {order_ms:.1f} ms")

    # arcs leaving the reached set, per source (a count, not an expected value)
    reach_arcs = {}
    for s in srcs:
        lbg.bfs(dg, int(s), strategy=args.strategy, out=lv_out, workspace=ws)
        reach_arcs[int(s)] = int(deg[lv_out != lbg.BFS_INF].sum().item())
    torch.cuda.synchronize()

    per = args.sources_per_step
    plan = [[int(srcs[(k * per + j) % len(srcs)]) for j in range(per)]
            for k in range(args.warmup + args.steps)]

    def step(sources, lat):
        arcs = 0
        for s in sources:
            t = time.perf_counter()
            lbg.bfs(dg, s, strategy=args.strategy, out=lv_out, workspace=ws)
            t1 = time.perf_counter()
            lbg.sssp(dg, s, strategy=args.strategy, out=d_out, workspace=ws, ordered=ordered)
            t2 = time.perf_counter()
            if lat is not None:
                lat["bfs"].append((t1 - t) * 1e3)
                lat["sssp"].append((t2 - t1) * 1e3)
                lat["arcs"].append(reach_arcs[s])
            arcs += 2 * reach_arcs[s]
        return arcs

    for k in range(args.warmup):
        step(plan[k], None)
    torch.cuda.synchronize()

    # Timed region.  With profiling on, the library brackets every expansion
    # launch with HIP events on the solve's stream (BFS and SSSP kernels are
    # accumulated separately).
    lat = {"bfs": [], "sssp": [], "arcs": []}
    if not args.no_profile:
        lbg.profile_enable(True, reset=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    arcs_total = 0
    for k in range(args.warmup, args.warmup + args.steps):
        arcs_total += step(plan[k], lat)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = {}
    if not args.no_profile:
        lbg.profile_enable(False, reset=False)
        prof = {"bfs": lbg.profile_read("bfs"), "sssp": lbg.profile_read("sssp"),
                "sssp_small": lbg.profile_read("sssp_small")}
    bfs_ms, sssp_ms = sum(lat["bfs"]), sum(lat["sssp"])
    n_solves = args.steps * per
    bfs_arcs = sum(reach_arcs[s] for k in range(args.warmup, args.warmup + args.steps)
                   for s in plan[k])

    out = {
        "metric": METRIC,
        "value": round(arcs_total / elapsed / 1e9, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": desc, "graph": g.name, "n": g.n, "m": g.m,
                   "sources_per_step": per, "strategy": args.strategy,
                   **({"slice_min": lbg.get_slice_min()} if args.strategy == "sliced" else {}),
                   "sssp_layout": "degree-class ordered copy" if ordered else "csr",
                   "solves_timed": 2 * n_solves},
        "bfs_gteps": round(bfs_arcs / (bfs_ms / 1e3) / 1e9, 4),
        "sssp_gteps": round(bfs_arcs / (sssp_ms / 1e3) / 1e9, 4),
        "graph500_gteps": round(arcs_total / elapsed / 1e9 / (2 if sym else 1), 4),
        "bfs_ms_p50": round(float(np.percentile(lat["bfs"], 50)), 4),
        "bfs_ms_p99": round(float(np.percentile(lat["bfs"], 99)), 4),
        "sssp_ms_p50": round(float(np.percentile(lat["sssp"], 50)), 4),
        "sssp_ms_p99": round(float(np.percentile(lat["sssp"], 99)), 4),
        # per-solve harmonic means over the timed sources (host clock around
        # each solve, which waits for its result)
        "bfs_gteps_hmean": round(hmean_gteps(lat["bfs"], lat["arcs"]), 4),
        "sssp_gteps_hmean": round(hmean_gteps(lat["sssp"], lat["arcs"]), 4),
    }
    if order_ms is not None:
        out["order_build_ms"] = round(order_ms, 3)
    if not args.no_profile:
        kern = {}
        for kind in ("bfs", "sssp"):
            p = prof[kind]
            nl = p["launches"] + p["empty_launches"]
            kname = "balanced" if args.strategy == "auto" else args.strategy
            label = f"k_expand_{kname}<{'true' if kind == 'sssp' else 'false'}>"
            if kind == "sssp" and ordered:
                label += " ordered"
            kern[kind] = {"kernel": label,
                          "launches": nl, "kernel_ms": p["kernel_ms"] + p["empty_ms"],
                          "bytes": algorithmic_bytes(kind, p),
                          "edges_scanned": p["edges_scanned"], "edges_skipped": p["edges_skipped"]}
        dom = max(kern, key=lambda k: kern[k]["kernel_ms"])
        traffic = recorded_traffic() if args.workload == "rmat22" else {}
        for kind, kd in kern.items():
            achieved = kd["bytes"] / (kd["kernel_ms"] / 1e3) / 1e9
            t = traffic.get(kd["kernel"])
            obj = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                   "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                   "traffic": round(t) if t is not None else None,
                   "kernel": kd["kernel"], "launches": kd["launches"],
                   "avg_launch_us": round(kd["kernel_ms"] * 1e3 / max(kd["launches"], 1), 3),
                   "bytes_per_launch": round(kd["bytes"] / max(kd["launches"], 1))}
            if kind == "sssp" and kd["edges_scanned"]:
                # arcs queued vs arcs actually loaded and relaxed by the
                # one-level launches, and all relaxations (small-frontier
                # levels included) per arc leaving the reached set: chaotic
                # Bellman-Ford relaxes some arcs more than once
                loaded = kd["edges_scanned"] - kd["edges_skipped"]
                obj["skipped_fraction"] = round(kd["edges_skipped"] / kd["edges_scanned"], 4)
                relaxed = loaded + prof["sssp_small"]["edges_scanned"]
                obj["relaxations_per_reached_arc"] = round(relaxed / max(bfs_arcs, 1), 4)
            out["roofline" if kind == dom else "roofline_" + kind] = obj
        out["kernel_share_of_wall"] = round(
            (kern["bfs"]["kernel_ms"] + kern["sssp"]["kernel_ms"]) / (elapsed * 1e3), 4)
    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        a_ = torch.empty(nb // 4, dtype=torch.int32, device=dev).fill_(1)
        b_ = torch.empty_like(a_)
        for _ in range(3):
            b_.copy_(a_)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nb
        del a_, b_
    return out, g, srcs


# ----------------------------------------------------------- strategies --
def run_strategies(lbg, torch, g, srcs, dev):
    """Node-based vs edge-based vs hierarchical vs balanced vs degree-binned
    vs destination-sliced vs node splitting with child nodes on the same
    graph: BFS and SSSP from two sources each (binned with bins autotuned on
    two other sources; the sliced graph, the split graph (split size by the
    histogram rule) and the COO array are built before timing)."""
    dg = lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights, device=dev, with_coo=True,
                                    with_slices=True)
    sp = dg.ensure_split()
    deg = g.degrees
    tuned = lbg.autotune_bins(dg, [int(x) for x in srcs[2:4]])
    ws = lbg.Workspace(dev)
    out = {"bins": tuned, "slice_min": lbg.get_slice_min(),
           "split_graph": {"mdt": sp.mdt, "children": sp.children}}
    for strat in ("node", "edge", "hier", "balanced", "binned", "sliced", "split"):
        res = {}
        for kind, f in (("bfs", lbg.bfs), ("sssp", lbg.sssp)):
            ts, arcs = [], 0
            for s in srcs[:2]:
                lv = lbg.bfs(dg, int(s), strategy="balanced", workspace=ws).cpu().numpy()
                arcs += int(deg[lv != lbg.BFS_INF].sum())
                f(dg, int(s), strategy=strat, workspace=ws)
                torch.cuda.synchronize()
                t = time.perf_counter()
                f(dg, int(s), strategy=strat, workspace=ws)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            res[f"{kind}_ms"] = [round(x * 1e3, 3) for x in ts]
            res[f"{kind}_gteps"] = round(arcs / sum(ts) / 1e9, 3)
        out[strat] = res
        log(f"strategy {strat}: {res}")

    def sssp_layout(name, **kw):
        ts, arcs = [], 0
        for s in srcs[:2]:
            lv = lbg.bfs(dg, int(s), strategy="balanced", workspace=ws).cpu().numpy()
            arcs += int(deg[lv != lbg.BFS_INF].sum())
            lbg.sssp(dg, int(s), workspace=ws, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            lbg.sssp(dg, int(s), workspace=ws, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        out[name] = {"sssp_ms": [round(x * 1e3, 3) for x in ts], "sssp_gteps": round(arcs / sum(ts) / 1e9, 3)}
        log(f"strategy {name}: {out[name]}")

    # hierarchical processing with a fixed window (MDT 256, the binned
    # strategy's tuned split size) beside the histogram rule's
    lbg.set_hier_mdt(256)
    try:
        res = {}
        for kind, f in (("bfs", lbg.bfs), ("sssp", lbg.sssp)):
            ts, arcs = [], 0
            for s in srcs[:2]:
                lv = lbg.bfs(dg, int(s), strategy="balanced", workspace=ws).cpu().numpy()
                arcs += int(deg[lv != lbg.BFS_INF].sum())
                f(dg, int(s), strategy="hier", workspace=ws)
                torch.cuda.synchronize()
                t = time.perf_counter()
                f(dg, int(s), strategy="hier", workspace=ws)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            res[f"{kind}_ms"] = [round(x * 1e3, 3) for x in ts]
            res[f"{kind}_gteps"] = round(arcs / sum(ts) / 1e9, 3)
        out["hier_mdt256"] = res
        log(f"strategy hier_mdt256: {res}")
    finally:
        lbg.set_hier_mdt(0)

    # balanced SSSP on packed 32-bit arcs (one load per arc), when ids and
    # weights fit in 32 bits, and on the degree-class ordered copy
    try:
        dg.ensure_packed()
        sssp_layout("balanced_packed", packed=True)
        out["balanced_packed"]["wbits"] = dg.packed[1]
    except lbg.LbgError:
        pass
    dg.ensure_ordered()
    sssp_layout("balanced_ordered", ordered=True)
    return out


# -------------------------------------------------------------- batched --
def run_batch(lbg, torch, dev, count, sources_per_instance, hi_exp, reps=3):
    """The same 2 x sources x count queries solved as one batch and as
    single-query calls; GTEPS over arcs leaving reached nodes."""
    import graphgen

    t0 = time.perf_counter()
    gs = graphgen.batch_instances(count, hi_exp=hi_exp)
    u, nb, eb = graphgen.pack(gs)
    log(f"batch: {count} instances, n={u.n} m={u.m} built in {time.perf_counter() - t0:.1f}s")
    dg = lbg.DeviceGraph.from_numpy(u.offsets, u.cols, u.weights, device=dev)
    singles = [lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights, device=dev) for g in gs]
    queries = []
    for i, g in enumerate(gs):
        for s in graphgen.sources(g, sources_per_instance, graphgen.FAMILY_BATCH, salt=i):
            for kind in (lbg.KIND_BFS, lbg.KIND_SSSP):
                queries.append((int(nb[i] + s), int(nb[i]), int(nb[i + 1]), kind))
    ws = lbg.Workspace(dev)
    ws1 = lbg.Workspace(dev)
    out, bst = lbg.batch_solve(dg, queries, workspace=ws, stats=True)  # warm-up + reached-arc count
    deg = torch.from_numpy(np.diff(u.offsets.astype(np.int64))).to(dev)
    reached = 0
    off = 0
    for q in queries:
        row = out[off: off + q[2] - q[1]]
        unreached = lbg.BFS_INF if q[3] == lbg.KIND_BFS else -1  # UINT32_MAX as int32
        reached += int(deg[q[1]: q[2]][row != unreached].sum().item())
        off += q[2] - q[1]
    torch.cuda.synchronize()
    tb, tg = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        lbg.batch_solve(dg, queries, out=out, workspace=ws)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t)
    lbg.batch_solve(dg, queries, out=out, workspace=ws, graph=True)  # builds the graph
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        lbg.batch_solve(dg, queries, out=out, workspace=ws, graph=True)
        torch.cuda.synchronize()
        tg.append(time.perf_counter() - t)
    # plain: one call per query on the query's own instance graph
    idx = np.searchsorted(nb, [q[0] for q in queries], side="right") - 1
    outs = [torch.empty(g.n, dtype=torch.int32, device=dev) for g in gs]
    for q, i in zip(queries[:64], idx[:64]):  # warm-up
        f = lbg.bfs if q[3] == lbg.KIND_BFS else lbg.sssp
        f(singles[i], q[0] - q[1], out=outs[i], workspace=ws1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    lat = []
    for q, i in zip(queries, idx):
        f = lbg.bfs if q[3] == lbg.KIND_BFS else lbg.sssp
        t1 = time.perf_counter()
        f(singles[i], q[0] - q[1], out=outs[i], workspace=ws1)
        lat.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t
    bt, gt = min(tb), min(tg)
    return {"queries": len(queries), "instances": count, "n": u.n, "m": u.m,
            "batched_s": round(bt, 5), "graph_batched_s": round(gt, 5), "plain_s": round(tp, 5),
            "batched_gteps": round(reached / bt / 1e9, 4),
            "graph_batched_gteps": round(reached / gt / 1e9, 4),
            "plain_gteps": round(reached / tp / 1e9, 4),
            "speedup": round(tp / bt, 3), "graph_speedup": round(tp / gt, 3),
            "levels": bst["levels"], "graph_launches_per_batch": -(-bst["levels"] // 64),
            "plain_query_ms_p50": round(float(np.percentile(lat, 50)) * 1e3, 4),
            "plain_query_ms_p99": round(float(np.percentile(lat, 99)) * 1e3, 4),
            "workload": f"{count} instances (half R-MAT scale U[10,{hi_exp}] ef 16 symmetrised, "
                        f"half uniform n=2^U(10,{hi_exp}) 8 out-arcs), weights U[1,255], "
                        f"{sources_per_instance} sources each, BFS + SSSP"}


# -------------------------------------------------------------- serving --
def run_serve(lbg, torch, dev, scales, fractions, requests_per_point, upload_count=8,
              big_arcs=1 << 23, workers=3, engine_only_fraction=None, engine_yield_ms=0.0):
    """Serving over resident R-MAT instances plus per-request uploads.
    Instances of at least big_arcs arcs are served by a plain lane of
    `workers` solves that run at once (queries overlap on the device), the
    rest, and every upload, are batched by the engine.  engine_only_fraction:
    also serve that load with every resident instance batched in the engine
    and no plain lane, for comparison."""
    import graphgen
    from paper_1711_00231_amd import serve

    t0 = time.perf_counter()
    resident = [graphgen.rmat(s, salt=50 + s) for s in scales]
    names = [f"rmat{s}" for s in scales]
    uploads = [graphgen.uniform(n=int(2 ** e), k=8, wlo=1, whi=255, salt=60 + i)
               for i, e in enumerate(np.linspace(12, 16, upload_count))]
    # every resident instance stays in HBM as its own CSR (plain solves);
    # the small ones are also packed, with the upload regions, for the engine
    singles = {nm: lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights, device=dev)
               for nm, g in zip(names, resident)}
    NC, MC, R = (1 << 16) + 1, (1 << 16) * 8, 8

    def engine_for(packed):
        """Engine over the packed instances (name, graph) plus the upload
        regions; returns (engine, packed device graph, pack, instance map)."""
        u, nb, eb = graphgen.pack([g for _, g in packed])
        off_e, cols_e, w_e = serve.UploadArena.empty_arrays(R, NC, MC, u.n, u.m)
        off = np.concatenate([u.offsets[:-1].astype(np.int64), off_e, [u.m + R * MC]])
        dg = lbg.DeviceGraph.from_numpy(off, np.concatenate([u.cols, cols_e]),
                                        np.concatenate([u.weights, w_e]), device=dev)
        del off, off_e, cols_e, w_e
        inst = {nm: serve.Instance(0, g.n, g.m) for nm, g in zip(names, resident)}
        for i, (nm, g) in enumerate(packed):
            inst[nm] = serve.Instance(int(nb[i]), int(nb[i + 1]), int(eb[i + 1] - eb[i]))
        max_rows = 6 * max([g.n for _, g in packed] + [1]) + 16 * NC
        eng = lbg.Engine(dg, max_queries=64, max_rows=max_rows,
                         max_level_arcs=min(2**32 - 1, 8 * (u.m + R * MC)))
        return eng, dg, u, inst

    small = [(nm, g) for nm, g in zip(names, resident) if g.m < big_arcs]
    eng, dg, u, inst = engine_for(small)
    log(f"serve: resident scales {scales} ({len(small)} batched), packed n={u.n} m={u.m} "
        f"built in {time.perf_counter() - t0:.1f}s")
    srcs = {nm: graphgen.sources(g, 64, graphgen.FAMILY_SERVE, salt=s)
            for nm, s, g in zip(names, scales, resident)}
    # saturation of plain per-query launches: mean service time of the mix
    up_dev = {id(g): lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights, device=dev)
              for g in uploads}
    ws1 = lbg.Workspace(dev)
    probe = serve.poisson_requests(1.0, 60, inst, upload_graphs=uploads, upload_share=0.25,
                                   seed=11, sources=srcs)
    def plain_call(r):
        """One plain solve of request r: resident instances run SSSP on their
        degree-class ordered copy, as the plain lane does; uploads use the CSR."""
        if r.kind == serve.KIND_BFS:
            lbg.bfs(singles[r.instance] if r.instance else up_dev[id(r.graph)], r.src, workspace=ws1)
        elif r.instance:
            lbg.sssp(singles[r.instance], r.src, workspace=ws1, ordered=True)
        else:
            lbg.sssp(up_dev[id(r.graph)], r.src, workspace=ws1)

    for gd in singles.values():
        gd.ensure_ordered()
    svc = []
    for r in probe:
        plain_call(r)
        torch.cuda.synchronize()
        t = time.perf_counter()
        plain_call(r)
        torch.cuda.synchronize()
        svc.append(time.perf_counter() - t)
    sat = 1.0 / float(np.mean(svc))
    # the plain lane holds every resident instance: large ones always go
    # there, small ones only when the engine and the lane are both idle
    # extra workers start a query only once a queue has built up and its
    # head has waited longer than the mean plain service time
    lane = serve.gpu_plain_lane(singles, big_arcs, ordered_sssp=True, workers=workers,
                                overlap_after=float(np.mean(svc)))

    def by_class(reqs, lat_ms):
        """p50 / p99 ms per target (resident instance name, or 'upload')."""
        out = {}
        for cls in sorted({r.instance or "upload" for r in reqs}):
            x = np.array([l for r, l in zip(reqs, lat_ms) if (r.instance or "upload") == cls])
            out[cls] = [round(float(np.percentile(x, 50)), 3), round(float(np.percentile(x, 99)), 3)]
        return out

    def plain_serve(reqs):
        """The same arrivals served FCFS by one plain call per request (upload
        graphs already resident: no copy is charged to the plain path)."""
        t0 = time.perf_counter()
        lat = []
        for r in reqs:
            while time.perf_counter() - t0 < r.arrival:
                pass
            plain_call(r)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0 - r.arrival)
        wall = time.perf_counter() - t0
        lat = np.array(lat) * 1e3
        return {"plain_p50_ms": round(float(np.percentile(lat, 50)), 4),
                "plain_p99_ms": round(float(np.percentile(lat, 99)), 4),
                "plain_qps": round(len(reqs) / wall, 2),
                "plain_by_target_p50_p99_ms": by_class(reqs, lat)}

    def requests_at(frac):
        return serve.poisson_requests(sat * frac, requests_per_point, inst, upload_graphs=uploads,
                                      upload_share=0.25, seed=int(frac * 1000), sources=srcs)

    points = []
    for frac in fractions:
        reqs = requests_at(frac)
        arena = serve.UploadArena(dg, u.n, u.m, R, NC, MC)
        rep = serve.Server(eng, inst, upload=arena, plain=lane, idle_bypass=True,
                           levels_per_step=2, engine_yield=engine_yield_ms * 1e-3).run(reqs)
        s = rep.summary()
        done = sorted(rep.completed, key=lambda r: r.rid)
        s["by_target_p50_p99_ms"] = by_class(done, [r.latency * 1e3 for r in done])
        s["offered_qps"] = round(sat * frac, 2)
        s["fraction_of_plain_saturation"] = frac
        s.update(plain_serve(reqs))
        points.append(s)
        log(f"serve {frac:.2f} x saturation: {s}")
    eng.close()
    out = {"plain_saturation_qps": round(sat, 2),
           "plain_service_ms_p50": round(float(np.percentile(svc, 50)) * 1e3, 4),
           "plain_service_ms_p99": round(float(np.percentile(svc, 99)) * 1e3, 4),
           "lane_workers": workers,
           "engine_yield_ms": engine_yield_ms,
           "points": points,
           "workload": f"resident R-MAT scales {list(scales)} (ef 16, symmetrised, weights "
                       f"U[1,255]) + per-request uploaded uniform graphs n in [2^12, 2^16]; "
                       f"Poisson arrivals, 70% BFS / 30% SSSP, 25% uploads; "
                       f"{requests_per_point} requests per point; gteps counts instance arcs; "
                       f"instances of >= {big_arcs} arcs are served by a plain lane of up to {workers} "
                       f"solves that run at once (each on its own stream and workspace: queries "
                       f"overlap on the device once a backlog has waited longer than the mean "
                       f"plain service time), the rest are batched by the engine unless the "
                       f"engine and the lane are both idle (then a resident query runs plain: "
                       f"'bypassed'); plain solves of resident instances run SSSP on their "
                       f"degree-class ordered copy; the engine advances 2 levels per step; "
                       f"plain_* = the same arrivals served FCFS by one plain call each"}
    if engine_only_fraction is not None:
        # every resident instance batched by the engine, no plain lane
        del eng, dg
        torch.cuda.empty_cache()
        eng2, dg2, u2, inst2 = engine_for(list(zip(names, resident)))
        reqs = serve.poisson_requests(sat * engine_only_fraction, requests_per_point, inst2,
                                      upload_graphs=uploads, upload_share=0.25,
                                      seed=int(engine_only_fraction * 1000), sources=srcs)
        arena = serve.UploadArena(dg2, u2.n, u2.m, R, NC, MC)
        rep = serve.Server(eng2, inst2, upload=arena, levels_per_step=2).run(reqs)
        s = rep.summary()
        s["offered_qps"] = round(sat * engine_only_fraction, 2)
        s["fraction_of_plain_saturation"] = engine_only_fraction
        s.update(plain_serve(reqs))
        eng2.close()
        out["engine_only"] = s
        log(f"serve, engine only, {engine_only_fraction:.2f} x saturation: {s}")
    return out


# ----------------------------------------------------------------- grid --
def run_grid(lbg, torch, dev, sources=4):
    """The high-diameter configuration: 2048x2048 grid with 1 % shortcuts
    and its no-shortcut companion, balanced BFS and SSSP from the first
    `sources` of the 16 seeded sources (one warm-up solve each)."""
    out = {}
    for name in ("grid2048", "grid2048-noshortcut"):
        g, srcs, desc, _ = make_workload(name)
        dg = lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights, device=dev)
        ws = lbg.Workspace(dev)
        deg = torch.from_numpy(g.degrees).to(dev)
        res = {"workload": desc, "n": g.n, "m": g.m}
        for kind, f in (("bfs", lbg.bfs), ("sssp", lbg.sssp)):
            ts, arcs, levels = [], 0, []
            for s in srcs[:sources]:
                s = int(s)
                lv = lbg.bfs(dg, s, workspace=ws)
                arcs += int(deg[lv != lbg.BFS_INF].sum().item())
                f(dg, s, workspace=ws)
                torch.cuda.synchronize()
                t = time.perf_counter()
                _, st = f(dg, s, workspace=ws, stats=True)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
                levels.append(st["levels"])
            res[f"{kind}_ms_p50"] = round(float(np.median(ts)) * 1e3, 3)
            res[f"{kind}_gteps"] = round(arcs / sum(ts) / 1e9, 4)
            res[f"{kind}_levels"] = levels
        out[name] = res
        log(f"grid {name}: {res}")
    return out


# ------------------------------------------------------------- capacity --
def run_capacity(lbg, torch, dev, scales=(24, 26), sources=2):
    """Largest R-MAT instances on one GPU (the space argument of the paper's
    Table I on 288 GB): per scale, the device bytes of the CSR, of the
    balanced and the edge-based workspaces (the latter with its COO array)
    as lbg_workspace_bytes gives them and as allocated, and balanced and
    edge-based BFS / SSSP from `sources` seeded sources, every result
    certified exact by the oracle's O(m) certificate.  Scale 26 is the
    largest whose arc count fits int32 CSR offsets."""
    import graphgen
    import oracle

    O = oracle.get()
    out = []
    for sc in scales:
        t0 = time.perf_counter()
        g = graphgen.rmat(sc)
        gen_s = time.perf_counter() - t0
        log(f"capacity: R-MAT scale {sc} n={g.n} m={g.m} generated in {gen_s:.1f}s")
        srcs = graphgen.sources(g, sources, graphgen.FAMILY_RMAT)
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        dg = lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights, device=dev)
        graph_bytes = torch.cuda.memory_allocated() - base
        rec = {"scale": sc, "n": g.n, "m": g.m, "generate_s": round(gen_s, 1), "graph_bytes": graph_bytes,
               "int32_offsets_headroom": round((2**31 - 1) / g.m, 3)}
        for strat in ("balanced", "edge"):
            wb = max(lbg.workspace_bytes(g.n, g.m, strat, False), lbg.workspace_bytes(g.n, g.m, strat, True))
            ws = lbg.Workspace(dev)
            before = torch.cuda.memory_allocated()
            ws.get(wb)
            if strat == "edge":
                dg.ensure_coo()
            rec[f"{strat}_workspace_bytes"] = wb
            rec[f"{strat}_allocated_bytes"] = torch.cuda.memory_allocated() - before
            for kind, f, w in (("bfs", lbg.bfs, None), ("sssp", lbg.sssp, g.weights)):
                ts, ok = [], True
                for s in srcs:
                    s = int(s)
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    res = f(dg, s, strategy=strat, workspace=ws)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t)
                    d = res.cpu().numpy()
                    if kind == "sssp":
                        d = d.view(np.uint32)
                    ok = ok and O.certificate(g.offsets, g.cols, w, s, d)[0] == 0
                rec[f"{strat}_{kind}_ms"] = [round(x * 1e3, 2) for x in ts]
                rec[f"{strat}_{kind}_certified"] = bool(ok)
                log(f"capacity scale {sc} {strat} {kind}: {rec[f'{strat}_{kind}_ms']} ms, certified {ok}")
            del ws
            torch.cuda.empty_cache()
        rec["peak_allocated_bytes"] = torch.cuda.max_memory_allocated() - base
        out.append(rec)
        log(f"capacity: {rec}")
        del dg, g
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="plain", choices=["plain", "batch", "serve", "capacity"])
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--strategy", default="balanced")
    ap.add_argument("--slice-min", type=int, default=None,
                    help="split degree of the sliced strategy (lbg_set_slice_min)")
    ap.add_argument("--sources-per-step", type=int, default=8)
    ap.add_argument("--sssp-layout", default="ordered", choices=["csr", "ordered"],
                    help="SSSP on the input CSR or on its degree-class ordered copy (balanced strategy)")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work for the cpu_baseline leg (0 = skip)")
    ap.add_argument("--no-profile", action="store_true",
                    help="do not bracket expansion launches with events (no roofline)")
    ap.add_argument("--no-extras", action="store_true",
                    help="plain mode: skip the compact batched and serving measurements")
    ap.add_argument("--engine-yield-ms", type=float, default=0.0,
                    help="serving: the engine waits while the plain lane has work, up to this "
                         "long after admitting a query (0: never waits)")
    ap.add_argument("--lane-workers", type=int, default=3,
                    help="serving: plain solves of large resident instances that may run at once")
    ap.add_argument("--switch-interval-us", type=float, default=0.0,
                    help="serving: the interpreter's thread switch interval (0 = leave Python's default)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed region, copy a buffer of this many MiB three times "
                         "(a plain copy kernel of known size, to scale rocprofv3 HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path (queries are "
              "independent, so several GPUs would each take a share of the sources).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1711_00231_amd import lbg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.slice_min is not None:
        lbg.set_slice_min(args.slice_min)
    if args.switch_interval_us > 0:
        sys.setswitchinterval(args.switch_interval_us * 1e-6)

    if args.mode == "batch":
        res = run_batch(lbg, torch, dev, count=256, sources_per_instance=4, hi_exp=18)
        print(json.dumps({"metric": "batched vs plain GTEPS", "value": res["batched_gteps"],
                          "unit": "GTEPS", "n_gpus": 1, "higher_is_better": True,
                          "dtype": "u32", "data": "synthetic", "vs_baseline": None,
                          "config": {"workload": res["workload"]}, "batched": res}), flush=True)
        return
    if args.mode == "capacity":
        res = run_capacity(lbg, torch, dev)
        print(json.dumps({"metric": "largest R-MAT instance solved and certified", "value": res[-1]["scale"],
                          "unit": "scale", "n_gpus": 1, "higher_is_better": True, "dtype": "u32",
                          "data": "synthetic", "vs_baseline": None,
                          "config": {"workload": "R-MAT scales 24 and 26, ef 16, symmetrised, "
                                                 "weights U[1,255], 2 sources, balanced and edge-based"},
                          "capacity": res}), flush=True)
        return
    if args.mode == "serve":
        res = run_serve(lbg, torch, dev, scales=(20, 22, 24),
                        fractions=(0.25, 0.5, 0.75, 1.0, 1.25), requests_per_point=2000,
                        workers=args.lane_workers, engine_yield_ms=args.engine_yield_ms)
        p99 = max(p["p99_ms"] for p in res["points"])
        print(json.dumps({"metric": "served p99 latency (ms) over a QPS sweep", "value": p99,
                          "unit": "ms", "n_gpus": 1, "higher_is_better": False, "dtype": "u32",
                          "data": "synthetic", "vs_baseline": None,
                          "config": {"workload": res["workload"]}, "serving": res}), flush=True)
        return

    out, g, srcs = run_plain(args, lbg, torch, dev)
    if not args.no_extras:
        log("strategy comparison")
        out["strategies"] = run_strategies(lbg, torch, g, srcs, dev)
        log("high-diameter grids")
        out["grid"] = run_grid(lbg, torch, dev)
        torch.cuda.empty_cache()
        log("batched comparison (256 instances, 2,048 solves)")
        out["batched"] = run_batch(lbg, torch, dev, count=256, sources_per_instance=4, hi_exp=18)
        torch.cuda.empty_cache()
        log("serving (resident R-MAT 20/22/24 + uploads)")
        out["serving"] = run_serve(lbg, torch, dev, scales=(20, 22, 24), fractions=(0.5, 1.0),
                                   requests_per_point=400, workers=args.lane_workers,
                                   engine_only_fraction=0.5)
        torch.cuda.empty_cache()
    if args.cpu_budget > 0:
        log("timing the CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(g, srcs, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
