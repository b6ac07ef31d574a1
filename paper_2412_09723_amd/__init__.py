"""MI355X-native differentiable RGB-D Gaussian rasterizer (the hot path of
MAC-Ego3D's tracking and mapping, arXiv 2412.09723).

Submodules:
  scenes  - seeded synthetic inputs (no rasterizer arithmetic)
  _lib    - ctypes binding of libmacsplat.so (the C ABI in include/macsplat.h)
  raster  - torch-facing jobs and the autograd Function
  build   - compiles libmacsplat.so for gfx950

Importing the package loads nothing on the GPU.
"""
__all__ = ["scenes", "raster", "build"]
