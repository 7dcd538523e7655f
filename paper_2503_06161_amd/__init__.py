"""MI355X-native tile rasterizer for feature-distilled 4D Gaussian splatting.

The compute path is the HIP library ``libfe4dgs_rast.so`` (kernels for
gfx950 behind a C ABI, declared in ``include/fe4dgs_rast.h``); the Python
modules only marshal arguments to it:

* ``rast``     ctypes binding, forward / backward, ``torch.autograd.Function``
* ``batch``    many frames replayed as one captured HIP graph
* ``autotune`` tile-shape selection by timing
* ``scenes``   seeded synthetic workloads (no rasterizer arithmetic)
* ``build``    compiles the library in-tree for gfx950

Submodules are imported explicitly so that the scene generator works
without the library or a GPU.
"""
