"""MI355X-native (gfx950 HIP) dual-time EDAC SPH pseudo-time hot path.

The library ``libdtsph.so`` (C-ABI, declared in ``include/dtsph.h``) does every
step of the path in hand-written HIP kernels; :mod:`.dtsph` is its thin ctypes
binding and :mod:`.inputs` the seeded workload generators. Nothing is loaded at
import time; the binding loads the library on first use and raises if it is
missing.
"""
__all__ = ["dtsph", "inputs"]
