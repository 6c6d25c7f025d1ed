"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only draws and shapes input data (grids of sample points, quality
factor fields, initial wavefields, request streams). It holds none of the
method's arithmetic: no fractional symbols, no expansion, no propagators. Both
the CPU oracle and the HIP path receive the arrays it produces, so the generator
never influences a parity comparison.
"""

from .generators import *  # noqa: F401,F403
