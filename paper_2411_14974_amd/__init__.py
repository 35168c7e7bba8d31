"""MI355X-native differentiable rasterizer for smooth 3D convexes (3D Convex Splatting).

The compute path lives in ``libconvexsplat.so`` (hand-written HIP kernels for
gfx950 behind a C ABI, ``include/convexsplat.h``); this package only marshals
arguments to it.  Importing the package does not load the library; the
binding (``paper_2411_14974_amd.binding``) does, and fails loudly when it is
missing.
"""
__all__ = ["scenes"]
