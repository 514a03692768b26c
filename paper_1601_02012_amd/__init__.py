"""MI355X-native Method-B weak-lensing ray tracer (RAY-RAMSES, arXiv:1601.02012).

The compute path is the HIP library ``librayramses.so`` (C-ABI declared in
``include/rayramses.h``); this package is its thin Python binding plus the
seeded input generators in :mod:`.inputs`.  Importing the package does not
load the library; :mod:`.api` does, and fails loudly if it is missing.
"""
__all__ = ["api", "inputs"]
