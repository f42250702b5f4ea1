"""Sort-free Weighted Sum Rendering (arXiv 2410.18931) on AMD MI355X.

The rendering path runs in hand-written HIP kernels for gfx950 (libwsr.so,
C-ABI in include/wsr.h); this package is its thin Python binding.
"""
from .render import WSRContext, globals_tensor, render, scene_to_device  # noqa: F401
