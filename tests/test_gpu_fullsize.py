"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (256^3, M=16, FP32 with FP64 coefficients; 1024^2 FP64):
full-field comparisons where the oracle finishes in seconds, sampled points
(each computed by the oracle on its own) where it does not, and the FP32
path against the FP64 path over long runs (the FP64 path being pinned to the
oracle at the same size)."""

import numpy as np
import pytest

import oracle as O
from gpu_helpers import as_seen, dev, host, rel_l2, require_gpu, say
from workloads import c2_inputs, c3_inputs, rng_for

pytestmark = pytest.mark.gpu


def _plan(c, precision, M=None, **kw):
    require_gpu()
    from paper_2311_13049_amd import vofl as V
    return V.Plan(c["shape"], c["lo"], c["hi"], Q=c["Q"], M=c["M"] if M is None else M,
                  dt=c["dt"], precision=precision, c0=c["c0"], omega0=c["omega0"], **kw)


@pytest.fixture(scope="module")
def c2():
    return c2_inputs()


@pytest.fixture(scope="module")
def c3():
    return c3_inputs()


def test_c2_apply_fp64_full_field(c2):
    say("C2 1024^2 apply fp64 vs oracle")
    p = _plan(c2, "fp64")
    g = O.gamma_from_Q(c2["Q"])
    u = dev(c2["u0"], "fp64")
    for op in (1, 2):
        out = host(p.apply(op, u))
        ref = O.mterm_apply(c2["u0"], O.seismic_op_order(g, op), c2["lo"], c2["hi"], c2["M"])
        assert rel_l2(out, ref) <= 1e-12, (op, rel_l2(out, ref))


def test_c2_three_steps_fp64_full_field(c2):
    say("C2 1024^2 3 steps fp64 vs oracle")
    p = _plan(c2, "fp64")
    u, v = dev(c2["u0"], "fp64"), dev(c2["v0"], "fp64")
    p.step(u, v, 3)
    assert p.sync_status() == 0
    ru, rv = O.tsfp2_seismic(c2["u0"], c2["v0"], O.gamma_from_Q(c2["Q"]), c2["c0"], c2["omega0"],
                             c2["lo"], c2["hi"], c2["M"], c2["dt"], 3)
    eu, ev = rel_l2(host(u), ru), rel_l2(host(v), rv)
    say(f"  rel L2 u {eu:.2e} v {ev:.2e}")
    assert eu <= 1e-12, eu
    assert ev <= 1e-12, ev


def test_c2_fp32_1000_steps_against_fp64(c2):
    """North-star FP32 claim: <= 1e-5 relative L2 after 1000 steps."""
    say("C2 1024^2 1000 steps fp32 vs fp64")
    out = {}
    for prec in ("fp64", "fp32"):
        p = _plan(c2, prec)
        u, v = dev(c2["u0"], prec), dev(c2["v0"], prec)
        p.step(u, v, 1000)
        assert p.sync_status() == 0
        out[prec] = host(u)
    assert rel_l2(out["fp32"], out["fp64"]) <= 1e-5, rel_l2(out["fp32"], out["fp64"])


def _sample_points(shape, count, seed):
    rng = rng_for(95, seed)
    pts = [tuple(int(n // 2) for n in shape)]
    for _ in range(count - 1):
        pts.append(tuple(int(rng.integers(n)) for n in shape))
    return pts


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_c3_apply_sampled_points(c3, precision):
    say(f"C3 256^3 apply {precision} sampled vs oracle")
    p = _plan(c3, precision, max_batch=2)
    g = O.gamma_from_Q(c3["Q"])
    x = as_seen(c3["u0"], precision)
    u = dev(c3["u0"], precision)
    pts = _sample_points(c3["shape"], 6, 0)
    tol = 1e-5 if precision == "fp32" else 1e-12
    for op in (1, 2):
        out = host(p.apply(op, u))
        scale = np.max(np.abs(out))
        ref = O.mterm_apply_at(x, O.seismic_op_order(g, op), c3["lo"], c3["hi"], c3["M"], pts)
        got = np.array([out[j] for j in pts])
        assert np.max(np.abs(got - ref)) <= tol * scale, (op, got, ref)


def test_c3_one_step_fp64_full_field(c3):
    say("C3 256^3 one step fp64 vs oracle (threaded library FFT)")
    p = _plan(c3, "fp64")
    u, v = dev(c3["u0"], "fp64"), dev(c3["v0"], "fp64")
    p.step(u, v, 1)
    assert p.sync_status() == 0
    O.set_fft_workers(16)
    try:
        ru, rv = O.tsfp2_seismic(c3["u0"], c3["v0"], O.gamma_from_Q(c3["Q"]), c3["c0"], c3["omega0"],
                                 c3["lo"], c3["hi"], c3["M"], c3["dt"], 1)
    finally:
        O.set_fft_workers(0)
    eu, ev = rel_l2(host(u), ru), rel_l2(host(v), rv)
    say(f"  rel L2 u {eu:.2e} v {ev:.2e}")
    assert eu <= 1e-12, eu
    assert ev <= 1e-12, ev


def test_c3_fp32_500_steps_against_fp64(c3):
    say("C3 256^3 500 steps fp32 vs fp64")
    out = {}
    for prec in ("fp64", "fp32"):
        p = _plan(c3, prec, max_batch=2)
        u, v = dev(c3["u0"], prec), dev(c3["v0"], prec)
        p.step(u, v, 500)
        assert p.sync_status() == 0
        out[prec] = host(u)
        p.close()
    assert rel_l2(out["fp32"], out["fp64"]) <= 1e-5, rel_l2(out["fp32"], out["fp64"])
