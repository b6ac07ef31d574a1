"""CPU oracle for the differentiable RGB-D Gaussian rasterizer.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path. Shares no code with
the GPU implementation. See `oracle.cpp` for what is computed and which
readings of the paper it takes; `brute.py` is an independent numpy
re-derivation used to cross-check it on tiny scenes.
"""
from .oracle import (  # noqa: F401
    build, load, project, tile_lists, forward, backward, record, frozen_loss,
    pinned_log2, apply_twist,
)
