"""libibpoisson: MI355X-native staggered-grid pressure Poisson solver.

The solver runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/ibpoisson.h``; ``paper_2609_19130_amd.ibpoisson`` is a
thin ctypes binding (argument marshalling only).  ``synth`` holds the seeded
synthetic input generators.  Importing this package loads nothing native;
the binding loads the shared library on first use and raises if it is
missing.
"""

__all__ = ["ibpoisson", "synth"]
