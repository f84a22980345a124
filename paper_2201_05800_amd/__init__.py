"""Space-time DG-SEM slab solver for MI355X (gfx950).

The compute path is the C-ABI library ``libstdg.so`` built from ``csrc/``
(hand-written HIP kernels plus the host engine).  ``paper_2201_05800_amd.st``
is the thin ctypes binding with the same names as the C entry points; it
raises if the library is missing.  ``paper_2201_05800_amd.inputs`` holds the
seeded synthetic workload generators.
"""
__all__ = ["st", "inputs"]
