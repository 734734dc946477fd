"""MI355X-native batched Gaussian-splat renderer (RGB + expected depth).

The renderer lives in the HIP library libgsmi.so (C interface in
include/gs.h); this package is its thin Python binding.
"""
from .binding import (GS_MODE_BATCHED, GS_MODE_PLAIN, EXPORTS, GsError, Renderer,  # noqa: F401
                      load)

__all__ = ["Renderer", "GsError", "load", "EXPORTS", "GS_MODE_PLAIN", "GS_MODE_BATCHED"]
