"""MI355X-native spectral Gaussian-random-field generator.

The arithmetic runs in hand-written HIP kernels for gfx950 behind a C-ABI
library (``libgrf.so``, declared in ``include/grf.h``).  This package is the thin
Python binding over that library; see ``paper_2212_10961_amd.grf``.
Submodules are imported lazily so that ``workloads`` can be used without the
binding.
"""
import importlib

__all__ = ["grf", "workloads"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
