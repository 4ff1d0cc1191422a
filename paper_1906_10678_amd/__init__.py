"""MI355X staged reach / path solver for the gap map-seeking arm method (arXiv 1906.10678).

Modules:
  msc    -- ctypes binding of the HIP library libmsc.so (include/msc.h)
  synth  -- seeded synthetic arms, scenes, start poses and targets
  build  -- hipcc build of libmsc.so for gfx950
"""
from . import synth  # noqa: F401

__all__ = ["synth", "msc", "build"]
