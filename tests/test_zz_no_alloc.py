"""lbg_sssp_noalloc (the SSSP entry point for callers that cannot allocate)
against lbg_sssp with a caller workspace and against the oracle: two calls
in a row on one GPU, the second on a smaller graph, so the second reads
scratch the first left behind."""
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


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("strategy", ["balanced", "node", "binned", "hier"])
def test_noalloc_matches_workspace_entry_point(strategy):
    big = graphgen.rmat(16)
    small = graphgen.uniform(12)
    srcs = [int(graphgen.sources(big, 1, graphgen.FAMILY_RMAT)[0]), 0]
    for g, s in zip((big, small), srcs):
        print(f"noalloc {strategy}: {g.name} n={g.n} m={g.m} src={s}", flush=True)
        dg = lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights)
        ref = _u32(lbg.sssp(dg, s, strategy=strategy))
        out = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
        got = st = None  # drop the previous graph's result first
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        got, st = lbg.sssp_noalloc(dg, s, strategy=strategy, out=out, stats=True)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before  # nothing taken from torch's allocator
        assert got.data_ptr() == out.data_ptr()
        assert np.array_equal(_u32(got), ref)
        assert np.array_equal(ref, O.dijkstra(g.offsets, g.cols, g.weights, s))
        assert st["levels"] > 0 and st["edges_scanned"] >= st["edges_skipped"] >= 0


def test_noalloc_rejects_oversize_and_stays_usable():
    g = graphgen.uniform(12)
    dg = lbg.DeviceGraph.from_numpy(g.offsets, g.cols, g.weights)
    out = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
    # a size the static scratch cannot hold is refused on the host, before
    # any launch (the pointers are never dereferenced)
    rc = lbg.lib.lbg_sssp_noalloc(lbg._ptr(dg.offsets), lbg._ptr(dg.cols), lbg._ptr(dg.weights), 1 << 22,
                                  128_307_136, 0, lbg._ptr(out), lbg.BALANCED, None, lbg._stream(None))
    assert rc == lbg.ENOMEM
    assert np.all(out.cpu().numpy() == -7)
    got = lbg.sssp_noalloc(dg, 5, out=out)
    assert np.array_equal(_u32(got), O.dijkstra(g.offsets, g.cols, g.weights, 5))
