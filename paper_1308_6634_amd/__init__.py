"""MI355X-native priorconditioned LSQR with lagged diffusivity.

The compute path is the HIP library ``libplsqr.so`` (kernels for gfx950 behind the C ABI
of ``include/plsqr.h``); ``plsqr`` is its ctypes binding and ``engine`` a small
convenience layer over torch device memory. Nothing here computes the method in Python.
"""

__all__ = ["plsqr", "engine"]
