"""CPU FP64 oracle for the variable-order fractional Laplacian and the TSFP2 solver.

TEST INFRASTRUCTURE ONLY. This package exists to check the HIP implementation
and is imported only by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``. The product package never imports, links
or executes anything from here, and this package imports nothing from it.

Parity status of each function is listed in ``vofl_oracle``'s module header.
"""

from .vofl_oracle import *  # noqa: F401,F403
