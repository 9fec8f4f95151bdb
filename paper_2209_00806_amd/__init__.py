"""MI355X-native TBPM (tight-binding propagation method) hot path.

The compute path is the C-ABI library ``libtbpm.so`` (hand-written HIP
kernels for gfx950); :mod:`paper_2209_00806_amd.tbpm` is its thin Python
binding and :mod:`paper_2209_00806_amd.inputs` generates seeded synthetic
lattices and random-phase states.  Importing the package does not load the
library; the binding loads it on first use and raises if it is missing.
"""

__all__ = ["inputs", "tbpm", "autograd"]


def __getattr__(name):
    if name in __all__:
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
