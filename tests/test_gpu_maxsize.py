"""The 3D workload at 512^3: every pass addresses half spectra of about 1 GiB
(FP64), eight times the 256^3 workload, through the same 32-bit byte offsets
and padded rows. The operator (2.13) is checked against the FP64 oracle at
sampled points (each evaluated on its own from the full spectrum), and one
TSFP2 step (3.13) of the FP32 path against the FP64 path over the whole
field."""

import numpy as np
import pytest

import oracle as O
from gpu_helpers import dev, host, parity_err, require_gpu, say, tol
from workloads import c3_inputs

pytestmark = pytest.mark.gpu

N = 512
M = 4
POINTS = [(256, 256, 256), (0, 0, 0), (511, 3, 300), (100, 400, 17), (255, 256, 257)]


@pytest.fixture(scope="module")
def inputs():
    say(f"{N}^3 inputs and the oracle at {len(POINTS)} points")
    c = c3_inputs(n=N)
    gamma = O.gamma_from_Q(c["Q"])
    # FP32-representable input: both precisions see the same values
    x = c["u0"].astype(np.float32).astype(np.float64)
    O.set_fft_workers(16)
    try:
        ref = O.mterm_apply_at(x, 1.0 + gamma, c["lo"], c["hi"], M, POINTS)
    finally:
        O.set_fft_workers(0)
    return c, x, ref


def _plan(c, precision):
    require_gpu()
    from paper_2311_13049_amd import vofl as V
    return V.Plan(c["shape"], c["lo"], c["hi"], Q=c["Q"], M=M, dt=c["dt"], precision=precision,
                  c0=c["c0"], omega0=c["omega0"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_apply_512cube_at_sampled_points(inputs, precision):
    c, x, ref = inputs
    say(f"{N}^3 apply {precision}")
    p = _plan(c, precision)
    out = host(p.apply(1, dev(x, precision))).reshape(c["shape"])
    p.close()
    got = np.array([out[j] for j in POINTS])
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(out)))
    say(f"  max error over max output {err:.2e}")
    assert err <= tol(precision)


def test_step_512cube_fp32_against_fp64(inputs):
    import torch
    c, x, _ = inputs
    res = {}
    for precision in ("fp64", "fp32"):
        say(f"{N}^3 one step {precision}")
        p = _plan(c, precision)
        u, v = dev(x, precision), dev(np.zeros(c["shape"]), precision)
        p.step(u, v, 1)
        assert p.sync_status() == 0
        res[precision] = (host(u), host(v))
        p.close()
        del u, v
        torch.cuda.empty_cache()
    eu = parity_err(res["fp32"][0], res["fp64"][0])
    ev = parity_err(res["fp32"][1], res["fp64"][1])
    say(f"  FP32 vs FP64 path: u {eu:.2e}, v {ev:.2e}")
    assert eu <= tol("fp32") and ev <= tol("fp32")
