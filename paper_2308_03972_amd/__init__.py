"""MI355X-native forecast-analysis cycle of LBM-LETKF.

The compute path is the C-ABI library ``liblbmletkf.so`` (hand-written HIP
kernels for gfx950, declared in ``include/lbmletkf.h``); ``binding`` is its
thin ctypes wrapper.  ``inputs`` holds the seeded synthetic input generators.
Submodules are imported on first use so that importing the package (for
example to reach ``inputs``) needs neither a GPU nor the built library.
"""
import importlib

__all__ = ["inputs", "binding", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
