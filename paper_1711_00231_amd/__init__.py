"""lbg: level-synchronous BFS and SSSP with load-balanced frontier expansion
for AMD MI355X (gfx950).

The compute path is the HIP library ``liblbg.so`` behind the C ABI declared
in ``include/lbg.h``; ``paper_1711_00231_amd.lbg`` is its Python binding.
Importing the binding without a built library raises ImportError.
"""
import importlib

__all__ = ["lbg"]


def __getattr__(name):
    if name == "lbg":
        return importlib.import_module(__name__ + ".lbg")
    raise AttributeError(name)
