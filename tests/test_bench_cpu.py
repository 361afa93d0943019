"""bench.py's host-side logic on the CPU: the one-GPU refusal, the
algorithmic-byte formulas, the recorded-traffic lookup and its source-hash
guard, the CPU-oracle baseline record and the workload table."""
import hashlib
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

SOURCES = bench.TRAFFIC_SOURCES


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_algorithmic_bytes():
    p = {"edges_scanned": 1000, "updates": 10, "frontier_entries": 7}
    assert bench.algorithmic_bytes("bfs", p) == 8 * 1000 + 20 * 10
    assert bench.algorithmic_bytes("sssp", p) == 12 * 1000 + 4 * 10 + 20 * 7
    # arcs of entries skipped at staging are never loaded: not charged
    p["edges_skipped"] = 300
    assert bench.algorithmic_bytes("sssp", p) == 12 * 700 + 4 * 10 + 20 * 7
    assert bench.algorithmic_bytes("bfs", p) == 8 * 1000 + 20 * 10


def _fake_root(tmp_path, digest_of=None):
    for f in SOURCES:
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, f), dst)
    h = hashlib.sha256()
    for f in SOURCES:
        h.update((tmp_path / f).read_bytes())
    (tmp_path / "profiles").mkdir()
    digest = digest_of or h.hexdigest()
    (tmp_path / "profiles" / "k_expand_balanced_x_hbm_traffic.txt").write_text(
        "header\n"
        f"kernel_sources_sha256: {digest}\n"
        "traffic_per_launch k_expand_balanced<true>: 123456\n"
        "traffic_per_launch k_expand_balanced<false>: 789\n")
    return tmp_path


def test_recorded_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(_fake_root(tmp_path)))
    got = bench.recorded_traffic()
    assert got == {"k_expand_balanced<true>": 123456.0, "k_expand_balanced<false>": 789.0}
    # any change to the sources makes the recorded figure stale
    with open(tmp_path / SOURCES[3], "a") as f:
        f.write("\n// changed\n")
    assert bench.recorded_traffic() == {}


def test_recorded_traffic_ignores_other_hashes(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(_fake_root(tmp_path, digest_of="0" * 64)))
    assert bench.recorded_traffic() == {}


def test_cpu_baseline_record():
    import graphgen

    g = graphgen.uniform(10)
    rec = bench.cpu_baseline(g, np.array([0, 1, 2], dtype=np.int32), budget_s=0.0)
    host = bench.host_info()
    assert rec["kind"] == "oracle" and rec["unit"] == "GTEPS"
    assert rec["cores"] == host["nproc"] >= 1 and rec["host"] == host
    assert rec["value"] > 0 and f"{host['nproc']} sources" in rec["sample"]
    st = rec["single_thread"]
    assert st["sources"] == 1 and st["bfs_ms_p50"] >= 0 and st["sssp_ms_p50"] >= 0 and st["gteps_hmean"] > 0


def test_workload_table():
    g, srcs, desc, sym = bench.make_workload("uniform14")
    assert g.n == 1 << 14 and len(srcs) == 1 and not sym and "uniform" in desc
    with pytest.raises(SystemExit):
        bench.make_workload("nope")


def test_harmonic_mean_gteps():
    # two solves of 1e9 arcs in 1 s and 2 s: 2 / (1 + 2) GTEPS
    assert abs(bench.hmean_gteps([1000.0, 2000.0], [10**9, 10**9]) - 2 / 3) < 1e-12
    # equal rates give that rate whatever the sizes
    assert abs(bench.hmean_gteps([1.0, 4.0], [10**6, 4 * 10**6]) - 1.0) < 1e-12
    assert bench.hmean_gteps([], []) is None
