"""MI355X-native (gfx950, HIP) rasterizer for 3D skew Gaussians.

The compute path lives in the C-ABI library libsgs.so (include/sgs.h); this
package holds its build script and the Python binding.  Importing the package
does not load the library; the first call does, and fails loudly if it is
missing (no CPU fallback exists).
"""
from ._abi import SgsError, default_options, load
from .raster import (CameraBatch, Frame, GaussianSet, Renderer, SkewGaussianRasterizer, bin_sort, densify,
                     densify_stats, preprocess, rasterize, render, render_backward)

__all__ = ["SgsError", "default_options", "load", "CameraBatch", "Frame", "GaussianSet", "Renderer",
           "SkewGaussianRasterizer", "bin_sort", "densify", "densify_stats", "preprocess", "rasterize", "render",
           "render_backward"]
