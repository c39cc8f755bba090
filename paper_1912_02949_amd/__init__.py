"""SketchyCGAL for the MaxCut SDP on MI355X (gfx950).

The numerical work runs in the HIP library libsketchycgal.so behind the C ABI
of include/sketchycgal.h; this package only marshals arguments to it.
"""
from .api import BatchedSketchyCGAL, Params, SketchyCGAL  # noqa: F401

__all__ = ["BatchedSketchyCGAL", "Params", "SketchyCGAL"]
