"""MI355X-native tile rasterizer for feature-distilled 4D Gaussian splatting.

The compute path is the HIP library ``libfe4dgs_rast.so`` (kernels for
gfx950 behind a C ABI, declared in ``include/fe4dgs_rast.h``); the Python
modules here only marshal arguments to it.  Import the binding lazily so
that the scene generator can be used without a GPU.
"""
__all__ = ["scenes", "rast"]


def __getattr__(name):
    if name == "rast":
        from . import rast
        return rast
    raise AttributeError(name)
