"""MI355X-native differentiable tile rasterizer for Deformable Beta Splatting
(arXiv 2501.18630).

Submodules:
  scenes    seeded synthetic scenes and cameras (inputs only)
  _lib      ctypes binding of the C-ABI in include/dbs.h (libdbs.so)
  renderer  buffer management, per-view and batched rendering, autograd
  autotune  tile-shape / batch-depth autotuner

Importing the package loads nothing; the HIP library is loaded on first use
and its absence is an error (there is no CPU fallback).
"""
__all__ = ["scenes"]
