"""MI355X-native linearized Poisson-Boltzmann grid solver (HIP, gfx950).

The compute path lives in the C-ABI library ``libpb.so`` (``csrc/``); ``binding``
is the thin ctypes layer over it.  Importing this package loads nothing.
"""
__all__ = ["inputs", "binding"]
