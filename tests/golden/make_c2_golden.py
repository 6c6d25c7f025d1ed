"""Writes tests/golden/c2_1000_steps_fp64.json: the FP64 oracle's TSFP2 solution
of the 2D workload (1024^2 on [-32,32)^2, Gaussian-random-field Q in [10,200],
M = 16, dt = 5e-4) after 1000 steps, for the GPU parity tests.

The oracle's step is TSFP2 for (1.1) under the splitting of Section 3.3
(eqs. (3.7)-(3.13)) with the apply (2.13). The full field is 16 MB per
component, so the file keeps what the tests compare element by element:

* the central 128 x 128 window (where the pulse has travelled) at every
  second point, for u and v;
* the full row and the full column through the centre, for u and v;
* projections of u and v onto 32 seeded standard-normal fields
  (workloads.probe_field): for an error field e, the root mean square of its
  projections estimates ||e||_2 over the whole grid;
* the L2 norm and the maximum modulus of u and v.

Run (about 20 minutes on 8 threads):
    python tests/golden/make_c2_golden.py [workers]
Calls only oracle/ (and the seeded input generator).
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from workloads import c2_inputs, probe_field  # noqa: E402

STEPS = 1000
NPROBE = 32
WIN = 128
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_1000_steps_fp64.json")


def summarize(f):
    n = f.shape[0]
    c, h = n // 2, WIN // 2
    def digits(a):  # 16 significant digits: far below the FP64 tolerance of the tests
        return [[float(f"{x:.15e}") for x in row] for row in a] if a.ndim == 2 else [float(f"{x:.15e}") for x in a]
    return {
        "window_stride2": digits(f[c - h:c + h:2, c - h:c + h:2]),
        "row_center": digits(f[c, :]),
        "col_center": digits(f[:, c]),
        "projections": [float(np.vdot(probe_field(f.shape, i), f)) for i in range(NPROBE)],
        "l2": float(np.linalg.norm(f)),
        "max_abs": float(np.max(np.abs(f))),
    }


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    c = c2_inputs()
    O.set_fft_workers(workers)
    t0 = time.time()
    u, v = O.tsfp2_seismic(c["u0"], c["v0"], O.gamma_from_Q(c["Q"]), c["c0"], c["omega0"],
                           c["lo"], c["hi"], c["M"], c["dt"], STEPS)
    secs = time.time() - t0
    n = c["shape"][0]
    doc = {
        "source": "FP64 oracle (tsfp2_seismic: TSFP2 of Section 3.3 applied to (1.1), apply (2.13)) "
                  "on the 2D workload: 1024^2 on [-32,32)^2, Q from the seeded Gaussian random field "
                  "(correlation length 4) mapped to [10,200], gamma = arctan(1/Q)/pi, c0 = omega0 = 1, "
                  "M = 16, u0 = exp(-|x|^2), v0 = 0, dt = 5e-4, 1000 steps",
        "script": "tests/golden/make_c2_golden.py",
        "steps": STEPS,
        "shape": [n, n],
        "window": {"size": WIN, "stride": 2, "start": [n // 2 - WIN // 2] * 2},
        "probes": {"count": NPROBE, "generator": "workloads.probe_field(shape, i), i = 0..count-1"},
        "oracle_seconds": round(secs, 1),
        "u": summarize(u),
        "v": summarize(v),
    }
    with open(OUT, "w") as fh:
        json.dump(doc, fh)
    print(f"wrote {OUT} ({secs:.0f} s)")


if __name__ == "__main__":
    main()
