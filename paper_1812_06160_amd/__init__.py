"""MI355X (gfx950) incomplete-LU hot path after Booth & Bolet, "Javelin: A Scalable
Implementation for Sparse Incomplete LU Factorization" (arXiv:1812.06160).

The numerics live in libjavelin.so (C ABI: include/javelin.h, HIP kernels in
csrc/); this package only marshals arguments.  Build with
``python -m paper_1812_06160_amd.build``.
"""
from . import _lib
from ._lib import IluError, load

__all__ = ["load", "Ilu", "IluApply", "IluError", "build", "levels_device", "permute_device", "transpose_device"]


def __getattr__(name):
    # torch-dependent pieces load lazily so that `import paper_1812_06160_amd`
    # works for the symbol checks without a GPU
    if name == "Ilu":
        from .ilu import Ilu
        return Ilu
    if name == "levels_device":
        from .ilu import levels_device
        return levels_device
    if name == "permute_device":
        from .ilu import permute_device
        return permute_device
    if name == "transpose_device":
        from .ilu import transpose_device
        return transpose_device
    if name == "IluApply":
        from .autograd import IluApply
        return IluApply
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
