"""MI355X-native forecast-analysis cycle of LBM-LETKF.

The compute path is the C-ABI library ``liblbmletkf.so`` (hand-written HIP
kernels for gfx950, declared in ``include/lbmletkf.h``); ``binding`` is its
thin ctypes wrapper.  ``inputs`` holds the seeded synthetic input generators.
The binding is imported lazily so that importing the package (for example to
reach ``inputs``) needs neither a GPU nor the built library.
"""
__all__ = ["inputs", "binding"]


def __getattr__(name):
    if name == "binding":
        from . import binding as _b
        return _b
    if name == "inputs":
        from . import inputs as _i
        return _i
    raise AttributeError(name)
