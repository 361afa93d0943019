"""Persistent cache of tuned degree-bin parameters.

The binned strategy's split size (MDT, Section III-B) and its wavefront /
workgroup thresholds depend on the graph's degree distribution and on the
GPU.  lbg.autotune_bins finds good values by timing solves; this module keeps
the result in a JSON file keyed by (graph class, n, m, GPU architecture) so
that a later process serving the same kind of graph sets them without timing
anything.

File format: {"version": 1, "entries": {key: {"mdt": int, "t_wave": int,
"t_block": int}}}, key = "<class>|n=<n>|m=<m>|arch=<arch>".  Writes go to a
temporary file that then replaces the cache, so readers never see a partial
file; concurrent writers may lose each other's new entries (the cache is
advisory), never corrupt it.  Entries that fail validation are ignored and
overwritten.
"""
from __future__ import annotations

import json
import os
import tempfile
import warnings

VERSION = 1


def default_path() -> str:
    p = os.environ.get("LBG_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "lbg", "bins.json")


def cache_key(graph_class: str, n: int, m: int, arch: str) -> str:
    if not graph_class or "|" in graph_class:
        raise ValueError(f"graph class must be a non-empty name without '|': {graph_class!r}")
    return f"{graph_class}|n={int(n)}|m={int(m)}|arch={arch}"


def _valid(e) -> bool:
    """Same rules as lbg_set_bins: mdt 0 or >= 64, 0 <= t_wave <= t_block."""
    try:
        mdt, tw, tb = (int(e[k]) for k in ("mdt", "t_wave", "t_block"))
    except (KeyError, TypeError, ValueError):
        return False
    return (mdt == 0 or mdt >= 64) and 0 <= tw <= tb


class BinsCache:
    def __init__(self, path: str | None = None):
        self.path = path or default_path()

    def load(self) -> dict:
        try:
            with open(self.path) as f:
                data = json.load(f)
        except FileNotFoundError:
            return {}
        except (OSError, ValueError) as exc:
            warnings.warn(f"ignoring unreadable tuning cache {self.path}: {exc}")
            return {}
        if not isinstance(data, dict) or data.get("version") != VERSION:
            warnings.warn(f"ignoring tuning cache {self.path} of another format")
            return {}
        entries = data.get("entries", {})
        return {k: {f: int(v[f]) for f in ("mdt", "t_wave", "t_block")}
                for k, v in entries.items() if isinstance(v, dict) and _valid(v)}

    def get(self, key: str):
        return self.load().get(key)

    def put(self, key: str, bins: dict) -> None:
        if not _valid(bins):
            raise ValueError(f"invalid bin parameters {bins}")
        entries = self.load()
        entries[key] = {f: int(bins[f]) for f in ("mdt", "t_wave", "t_block")}
        d = os.path.dirname(os.path.abspath(self.path))
        os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d, prefix=".bins.", suffix=".tmp")
        try:
            with os.fdopen(fd, "w") as f:
                json.dump({"version": VERSION, "entries": entries}, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except BaseException:
            if os.path.exists(tmp):
                os.unlink(tmp)
            raise


def device_arch(device) -> str:
    import torch

    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def tuned_bins(g, sources, graph_class: str, cache: BinsCache | None = None, arch: str | None = None,
               tune=None, apply=None) -> tuple:
    """Bin parameters for graph `g` of class `graph_class`: the cached ones
    when present, else lbg.autotune_bins over `sources`, stored for next
    time.  The parameters are made current (lbg.set_bins) either way.
    Returns (bins dict, True if they came from the cache).  `tune` and
    `apply` default to lbg.autotune_bins and lbg.set_bins."""
    if tune is None or apply is None:
        from . import lbg

        tune = tune or lbg.autotune_bins
        apply = apply or lbg.set_bins
    cache = cache or BinsCache()
    key = cache_key(graph_class, g.n, g.m, arch or device_arch(g.offsets.device))
    hit = cache.get(key)
    if hit is not None:
        apply(**hit)
        return hit, True
    best = tune(g, sources)
    cache.put(key, best)
    apply(**best)
    return dict(best), False
