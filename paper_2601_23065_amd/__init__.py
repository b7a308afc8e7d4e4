"""MI355X (gfx950) ray and path tracing through 2D Gaussian surfels.

The computations run in libeag.so (hand-written HIP kernels behind the C ABI
of include/eag.h); this package only marshals arguments. Importing the
package does not load the library; the first call does, and raises if it has
not been built.
"""
from ._lib import (ADDITIVE_EMISSION, DETACH_BOUNCE, EDIT_SCALE_RADIANCE, EDIT_SET_ALBEDO,  # noqa: F401
                   EDIT_SET_EMISSIVE, EDIT_SET_RADIANCE, EDIT_TRANSFORM, JITTER, EagError, load)


def __getattr__(name):
    # the torch-facing API is imported lazily so that the package can be
    # imported (e.g. for build()) without touching the GPU
    import importlib
    if name in ("api", "build", "_lib"):
        return importlib.import_module(f"{__name__}.{name}")
    if name.startswith("__"):
        raise AttributeError(name)
    return getattr(importlib.import_module(f"{__name__}.api"), name)
