"""TAPS slab-solve hot path for MI355X (gfx950): HIP kernels behind a C ABI.

The library (libtaps.so, built from csrc/ by build.py) holds every step of the
method; ``capi`` is its ctypes binding and ``problem`` builds device problems
for the synthetic workloads.
"""
from . import capi  # noqa: F401

__all__ = ["capi"]
