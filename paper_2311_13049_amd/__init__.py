"""vofl: matrix-free variable-order fractional Laplacian and TSFP2 wave solver
(arXiv 2311.13049) on AMD Instinct MI355X.

The compute path is libvofl.so (hand-written HIP for gfx950, C ABI in
include/vofl.h); ``vofl`` is its ctypes binding. There is no CPU fallback:
calls raise if the library is missing or no GPU is present.
"""

from . import vofl  # noqa: F401
from .vofl import Plan, VoflError  # noqa: F401

__all__ = ["vofl", "Plan", "VoflError"]
