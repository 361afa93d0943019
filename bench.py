#!/usr/bin/env python3
"""Benchmark: level-synchronous BFS and SSSP on one MI355X.

Workload (default): R-MAT scale 22, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05),
relabelled, symmetrised, duplicates and self-loops removed (n = 4,194,304,
m = 128,307,136 arcs), uint32 weights U[1,255], 64 seeded non-isolated
sources.  One step = BFS then SSSP from each of `--sources-per-step` sources
(cycling through the 64), through the C ABI, with the graph resident in HBM.

Throughput: GTEPS = arcs leaving reached nodes (the CSR arcs a traversal
scans) / wall time, summed over BFS and SSSP solves; the Graph500-style
figure (half of that on a symmetrised graph) is printed beside it.

Roofline: the dominant frontier-expansion kernel's algorithmic bytes per
launch / its average launch duration, timed live with HIP events on the
stream it runs on, against 8 TB/s HBM.  Algorithmic bytes per launch:
  BFS  8 B per arc scanned (column id + destination state) + 20 B per node
       discovered (two offsets, level write, worklist write and read);
  SSSP 12 B per relaxation (column id, weight, destination distance) + 4 B
       per successful update + 20 B per worklist entry.

cpu_baseline: the CPU oracle (queue BFS + binary-heap Dijkstra, one thread)
on a bounded sample of the same sources.
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


def algorithmic_bytes(kind, prof):
    if kind == "bfs":
        return 8 * prof["edges_scanned"] + 20 * prof["updates"]
    return 12 * prof["edges_scanned"] + 4 * prof["updates"] + 20 * prof["frontier_entries"]


def cpu_baseline(g, srcs, budget_s):
    """Oracle BFS + Dijkstra, single thread, on as many sources as fit the
    time budget (at least one)."""
    import oracle

    O = oracle.get()
    arcs = 0
    t_total = 0.0
    used = 0
    deg = g.degrees
    for s in srcs:
        t0 = time.perf_counter()
        lv = O.bfs(g.offsets, g.cols, int(s))
        O.dijkstra(g.offsets, g.cols, g.weights, int(s))
        t_total += time.perf_counter() - t0
        arcs += 2 * int(deg[lv != np.iinfo(np.int32).max].sum())
        used += 1
        if t_total >= budget_s:
            break
    return {"value": arcs / t_total / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{used} source(s) of the same workload, BFS + Dijkstra each, "
                      f"{t_total:.1f} s single-threaded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--strategy", default="balanced")
    ap.add_argument("--sources-per-step", type=int, default=8)
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work for the cpu_baseline leg (0 = skip)")
    ap.add_argument("--no-profile", action="store_true",
                    help="do not bracket expansion launches with events (no roofline)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed region, copy a buffer of this many MiB three times "
                         "(a plain copy kernel of known size, to scale rocprofv3 HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(queries are independent; see DESIGN.md for how it would shard).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1711_00231_amd import lbg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    t0 = time.perf_counter()
    g, srcs, desc, sym = make_workload(args.workload)
    log(f"workload {g.name}: n={g.n} m={g.m} built in {time.perf_counter() - t0:.1f}s")
    dg = lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights, device=dev,
                                    with_coo=(args.strategy == "edge"))
    ws = lbg.Workspace(dev)
    lv_out = torch.empty(g.n, dtype=torch.int32, device=dev)
    d_out = torch.empty(g.n, dtype=torch.int32, device=dev)
    deg = torch.from_numpy(g.degrees).to(dev)

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
            lbg.sssp(dg, s, strategy=args.strategy, out=d_out, workspace=ws)
            t2 = time.perf_counter()
            if lat is not None:
                lat["bfs"].append((t1 - t) * 1e3)
                lat["sssp"].append((t2 - t1) * 1e3)
            arcs += 2 * reach_arcs[s]
        return arcs

    for k in range(args.warmup):
        step(plan[k], None)
    torch.cuda.synchronize()

    # Timed region.  With profiling on, the library brackets every expansion
    # launch with HIP events on the solve's stream (BFS and SSSP kernels are
    # accumulated separately).
    lat = {"bfs": [], "sssp": []}
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
        prof = {"bfs": lbg.profile_read(False), "sssp": lbg.profile_read(True)}
    bfs_ms, sssp_ms = sum(lat["bfs"]), sum(lat["sssp"])
    solve_s = elapsed
    n_solves = args.steps * per
    bfs_arcs = sum(reach_arcs[s] for k in range(args.warmup, args.warmup + args.steps) for s in plan[k])

    out = {
        "metric": METRIC,
        "value": round(arcs_total / solve_s / 1e9, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(solve_s * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": desc, "graph": g.name, "n": g.n, "m": g.m,
                   "sources_per_step": per, "strategy": args.strategy,
                   "solves_timed": 2 * n_solves},
        "bfs_gteps": round(bfs_arcs / (bfs_ms / 1e3) / 1e9, 4),
        "sssp_gteps": round(bfs_arcs / (sssp_ms / 1e3) / 1e9, 4),
        "graph500_gteps": round(arcs_total / solve_s / 1e9 / (2 if sym else 1), 4),
        "bfs_ms_p50": round(float(np.percentile(lat["bfs"], 50)), 4),
        "bfs_ms_p99": round(float(np.percentile(lat["bfs"], 99)), 4),
        "sssp_ms_p50": round(float(np.percentile(lat["sssp"], 50)), 4),
        "sssp_ms_p99": round(float(np.percentile(lat["sssp"], 99)), 4),
        "wall_s_timed_region": round(elapsed, 4),
    }
    if not args.no_profile:
        kern = {}
        for kind in ("bfs", "sssp"):
            p = prof[kind]
            nl = p["launches"] + p["empty_launches"]
            byt = algorithmic_bytes(kind, p)
            kern[kind] = {
                "kernel": f"k_expand_{args.strategy}<{'true' if kind == 'sssp' else 'false'}>",
                "launches": nl, "kernel_ms": p["kernel_ms"] + p["empty_ms"],
                "bytes": byt, "edges_scanned": p["edges_scanned"],
                "avg_launch_us": (p["kernel_ms"] + p["empty_ms"]) * 1e3 / max(nl, 1),
            }
        dom = max(kern, key=lambda k: kern[k]["kernel_ms"])
        kd = kern[dom]
        achieved = kd["bytes"] / (kd["kernel_ms"] / 1e3) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                           "traffic": None, "kernel": kd["kernel"],
                           "avg_launch_us": round(kd["avg_launch_us"], 3),
                           "bytes_per_launch": round(kd["bytes"] / max(kd["launches"], 1))}
        other = "bfs" if dom == "sssp" else "sssp"
        ko = kern[other]
        out["roofline_other"] = {"kernel": ko["kernel"],
                                 "achieved": round(ko["bytes"] / (ko["kernel_ms"] / 1e3) / 1e9, 2),
                                 "avg_launch_us": round(ko["avg_launch_us"], 3),
                                 "bytes_per_launch": round(ko["bytes"] / max(ko["launches"], 1))}
        out["kernel_share_of_wall"] = round(
            (kern["bfs"]["kernel_ms"] + kern["sssp"]["kernel_ms"]) / (solve_s * 1e3), 4)
    if args.copy_probe_mib > 0:
        nb = args.copy_probe_mib << 20
        a_ = torch.empty(nb // 4, dtype=torch.int32, device=dev).fill_(1)
        b_ = torch.empty_like(a_)
        for _ in range(3):
            b_.copy_(a_)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nb
        del a_, b_
    if args.cpu_budget > 0:
        log("timing the CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(g, srcs, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
