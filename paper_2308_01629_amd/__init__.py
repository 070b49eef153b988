"""MI355X-native HR upsampling step of arXiv 2308.01629 (Section 4).

The compute path lives in the HIP library ``libupsample.so`` (C ABI in
``include/upsample.h``); this package holds its build script and a thin
PyTorch-facing binding.  Importing the binding requires the built library.
"""
from ._lib import UpsampleError, lib  # noqa: F401

__all__ = ["UpsampleError", "lib", "Upsampler", "grid_info_for"]


def __getattr__(name):
    if name in ("Upsampler", "grid_info_for", "make_params"):
        from . import upsampler
        return getattr(upsampler, name)
    raise AttributeError(name)
