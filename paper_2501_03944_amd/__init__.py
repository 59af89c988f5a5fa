"""MI355X-native hot path of the multi-guiding spark fireworks algorithm (MGFWA).

Submodules:
  inputs -- seeded synthetic workloads (data only)
  mgfwa  -- thin ctypes binding of the C-ABI library libmgfwa.so (HIP, gfx950)
The binding is imported lazily so that importing the package for its inputs does
not need the compiled library.
"""
__all__ = ["inputs", "mgfwa"]
