"""MI355X-native batched 3D Gaussian Splatting training step.

Hot path (HIP kernels behind the C ABI of include/gs.h, libgs.so):
transformation, Z-buffer binning + radix sort, render forward, L1 loss,
render + transformation backward, fused Adam with the paper's batch scaling
rules. Above it: an autograd Function, a batched graph-captured trainer
whose render passes take the tiles heaviest first by the previous step's
per-tile work (or another launch order where the autotuner measures it
faster), and a continuous-batching render server.
"""
from . import _lib  # noqa: F401

__all__ = ["raster", "autograd", "train", "serve", "autotune"]
