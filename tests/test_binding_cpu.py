"""The binding checks the tensors whose pointers it hands to the library:
the library writes n 4-byte results through `out` and reads the graph
arrays as 1-D 32-bit integers, and cannot see a tensor's size, type or
layout itself.  CPU tensors stand in for device ones (no call reaches the
library)."""
import pytest

torch = pytest.importorskip("torch")
from paper_1711_00231_amd import lbg  # noqa: E402

CPU = torch.device("cpu")


def _graph():
    off = torch.tensor([0, 1, 2, 2], dtype=torch.int32)
    cols = torch.tensor([1, 0], dtype=torch.int32)
    return lbg.DeviceGraph(off, cols, torch.tensor([3, 4], dtype=torch.int32))


def test_out_tensor_checks():
    t = torch.empty(10, dtype=torch.int32)
    assert lbg._out(t, 10, CPU) is t
    assert lbg._out(torch.empty(12, dtype=torch.uint32), 10, CPU).numel() == 12
    assert lbg._out(None, 3, CPU).shape == (3,)
    bad = [torch.empty(9, dtype=torch.int32),                 # too short
           torch.empty(10, dtype=torch.int64),                # 8-byte words
           torch.empty(20, dtype=torch.int32)[::2],           # strided
           torch.empty(2, 5, dtype=torch.int32),              # not 1-D
           torch.empty(10, dtype=torch.float32)]
    for t in bad:
        with pytest.raises(ValueError):
            lbg._out(t, 10, CPU)


def test_solves_refuse_a_bad_out_before_any_call():
    g = _graph()
    with pytest.raises(ValueError):
        lbg.bfs(g, 0, out=torch.empty(2, dtype=torch.int32))
    with pytest.raises(ValueError):
        lbg.sssp(g, 0, out=torch.empty(3, dtype=torch.int64))
    with pytest.raises(ValueError):
        lbg.sssp_noalloc(g, 0, out=torch.empty(6, dtype=torch.int32)[::2])


def test_device_graph_checks():
    g = _graph()
    assert (g.n, g.m) == (3, 2)
    off, cols = g.offsets, g.cols
    for args in ((off.long(), cols, None),                          # 64-bit offsets
                 (off, cols.long(), None),                          # 64-bit cols
                 (off, cols, torch.tensor([1], dtype=torch.int32)),  # one weight for two arcs
                 (torch.empty(0, dtype=torch.int32), cols, None),   # no offsets at all
                 (off, cols, torch.tensor([1.0, 2.0])),             # float weights
                 (off.view(1, 4), cols, None)):                     # not 1-D
        with pytest.raises(ValueError):
            lbg.DeviceGraph(*args)
    assert lbg.DeviceGraph(off, cols, None).weights is None
