"""MI355X-native TV-regularised cone-beam CT reconstruction (forward-backward splitting).

The compute path is libcbct.so (HIP kernels for gfx950 behind the C ABI of
include/cbct.h); this package is its thin Python binding.  Importing it does not
touch the GPU; the library is loaded on first use and its absence is an error.
"""
from ._lib import CbctError, lib  # noqa: F401


def __getattr__(name):
    if name == "Plan":
        from .ops import Plan
        return Plan
    raise AttributeError(name)
