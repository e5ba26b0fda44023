"""MI355X (gfx950) masked Gaussian rasterizer.

The compute path is ``libmaskgs.so`` (HIP kernels behind the C ABI in
``include/maskgs.h``); ``maskgs`` is its ctypes binding and ``raster`` the
rasterizer objects and the autograd Function.  Importing the package does not
load the library; importing ``maskgs`` or ``raster`` does, and fails loudly
if it has not been built.
"""
import os

PACKAGE_DIR = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(PACKAGE_DIR, "libmaskgs.so")

__all__ = ["PACKAGE_DIR", "LIBRARY"]
