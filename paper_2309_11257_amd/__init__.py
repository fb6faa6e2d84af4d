"""MI355X (gfx950) ray-volume tracer for the MS-GWaM-3D gravity-wave
parameterization (Voelker et al., arXiv 2309.11257).

The compute path is the HIP library ``librt.so`` (C ABI in ``include/rt.h``);
``Tracer`` is its ctypes binding.  ``workloads`` builds seeded synthetic
inputs.  Importing the package is cheap: the library is loaded on first use
and its absence raises ImportError.
"""
from . import workloads  # noqa: F401

__all__ = ["Tracer", "workloads", "lib"]


def __getattr__(name):
    if name in ("Tracer", "lib", "RTError"):
        from . import _rt
        return getattr(_rt, name)
    raise AttributeError(name)
