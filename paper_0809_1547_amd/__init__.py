"""MI355X (gfx950) Maxwell-Bloch FDTD stepper.

Submodules:
  mbf     -- ctypes binding of the C ABI (include/mbf.h); loads libmbf.so
  inputs  -- seeded synthetic inputs (sphere packings, material maps, probes)
"""
__all__ = ["mbf", "inputs"]
