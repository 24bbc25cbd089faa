"""Plane-wise multi-view Richardson-Lucy deconvolution on AMD MI355X (gfx950).

The computation runs in the HIP library ``libmvd.so`` (C ABI in
``include/mvd.h``); this package is its Python binding.  Importing it does not
load the library; the first call does, and fails loudly if it is not built.
"""
from .api import *  # noqa: F401,F403
from .api import Deconvolver, deconvolve  # noqa: F401
