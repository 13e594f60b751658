"""AO-direct J/K build on AMD MI355X (gfx950).

The compute path is the HIP library ``libjk.so`` (C-ABI in include/jk.h)
behind the ctypes binding in ``jk``.  Importing the package loads nothing;
``synth`` (seeded synthetic workloads) has no dependency on the library.
"""
__all__ = ["jk", "synth"]
