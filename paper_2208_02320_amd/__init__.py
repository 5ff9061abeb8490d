"""MI355X (gfx950) implementation of hierarchical homogenization (arXiv 2208.02320).

Submodules:
  hh     -- ctypes binding of the C ABI in include/hh.h (libhh.so)
  synth  -- seeded synthetic label images (inputs only)
  build  -- compiles libhh.so with hipcc for gfx950
"""
__all__ = ["hh", "synth", "build"]
