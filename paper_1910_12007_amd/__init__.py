"""MI355X-native batched forward model of an elastic filament swimmer in a
Brinkman fluid (regularized Brinkmanlet, forward Euler) with ABC and an MLP
surrogate around it.

The compute path lives in the HIP library ``libswim.so`` (C ABI declared in
``include/swim.h``); ``paper_1910_12007_amd.swim`` is the thin ctypes binding
with the same names.  ``paper_1910_12007_amd.inputs`` holds the seeded
synthetic-input generators (no physics).
"""
__all__ = ["inputs", "swim"]
