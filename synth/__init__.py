"""Seeded synthetic fragment streams (shared by the tests, the oracle checks and the benchmark).

This package only draws inputs; it contains none of the method's arithmetic. Every stream is a structure of
arrays in the layout the library consumes:

* ``pixel`` uint32 [F]  -- y * width + x
* ``depth`` float32 [F] -- normalised depth
* ``alpha`` float32 [F] (one channel) or [F, 3] (per-channel transmittance)
* ``rgb``   float32 [F, 3] -- straight colour

The paper measures on rendered scenes (the Bistro bar, smoke and particle systems) that are not available
here; the workloads below are synthetic stand-ins with the shapes, counts and value ranges of those cases.
"""
from .frames import (Frame, REQUEST_RESOLUTIONS, frame_c1, frame_c2, frame_c3, frame_c4, frame_c5, frame_uniform,
                     make_frame, poisson_arrivals, scrambled_multiplier, scrambled_stream, smoke_density,
                     sparse_stream, target_image, torch_frame)

__all__ = ["Frame", "REQUEST_RESOLUTIONS", "frame_c1", "frame_c2", "frame_c3", "frame_c4", "frame_c5", "frame_uniform",
           "make_frame", "poisson_arrivals", "scrambled_multiplier", "scrambled_stream", "smoke_density",
           "sparse_stream", "target_image", "torch_frame"]
