"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (256^3, M=16, FP32 with FP64 coefficients; 1024^2 FP64):
full-field comparisons where the oracle finishes in seconds (256^3 with the
threaded library FFT), the 2D workload's full 1000 steps against a stored
oracle solution (tests/golden/make_c2_golden.py), sampled points (each
computed by the oracle on its own), and the FP32 path against the FP64 path
over long runs."""

import json
import os

import numpy as np
import pytest

import oracle as O
from gpu_helpers import as_seen, dev, host, parity_err, require_gpu, say
from workloads import c2_inputs, c3_inputs, probe_field, rng_for

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

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
        assert parity_err(out, ref) <= 1e-12, (op, parity_err(out, ref))


def test_c2_three_steps_fp64_full_field(c2):
    say("C2 1024^2 3 steps fp64 vs oracle")
    p = _plan(c2, "fp64")
    u, v = dev(c2["u0"], "fp64"), dev(c2["v0"], "fp64")
    p.step(u, v, 3)
    assert p.sync_status() == 0
    ru, rv = O.tsfp2_seismic(c2["u0"], c2["v0"], O.gamma_from_Q(c2["Q"]), c2["c0"], c2["omega0"],
                             c2["lo"], c2["hi"], c2["M"], c2["dt"], 3)
    eu, ev = parity_err(host(u), ru), parity_err(host(v), rv)
    say(f"  parity err u {eu:.2e} v {ev:.2e}")
    assert eu <= 1e-12, eu
    assert ev <= 1e-12, ev


@pytest.fixture(scope="module")
def c2_golden():
    with open(os.path.join(GOLD, "c2_1000_steps_fp64.json")) as fh:
        return json.load(fh)


def _vs_golden(f, gold, tol, what):
    """Compare a full 1024^2 result with the stored oracle summary: element by
    element on the central window and on the centre row and column (bound
    tol * max|ref| over the whole field), and in relative L2 over the whole
    field through the stored random projections."""
    n = f.shape[0]
    c, h = n // 2, gold["window"]["size"] // 2
    scale = gold[what]["max_abs"]
    pieces = ((f[c - h:c + h:2, c - h:c + h:2], gold[what]["window_stride2"]),
              (f[c, :], gold[what]["row_center"]), (f[:, c], gold[what]["col_center"]))
    e_max = max(float(np.max(np.abs(a - np.asarray(b)))) for a, b in pieces) / scale
    proj = np.array([np.vdot(probe_field(f.shape, i), f) for i in range(gold["probes"]["count"])])
    e_l2 = float(np.sqrt(np.mean((proj - np.asarray(gold[what]["projections"])) ** 2))) / gold[what]["l2"]
    e_norm = abs(float(np.linalg.norm(f)) / gold[what]["l2"] - 1.0)
    say(f"  {what}: max err / max|ref| {e_max:.2e}, projected rel-L2 {e_l2:.2e}, norm {e_norm:.2e}")
    assert e_max <= tol and e_l2 <= tol and e_norm <= tol, (what, e_max, e_l2, e_norm)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c2_1000_steps_vs_oracle(c2, c2_golden, precision):
    """The 2D workload's full 1000 steps against the FP64 oracle's stored
    solution: the FP64 path within 1e-12, the FP32 path (FP64 coefficients
    and spectral state) within 1e-5 (same initial data, FP32-representable)."""
    say(f"C2 1024^2 1000 steps {precision} vs stored oracle solution")
    p = _plan(c2, precision)
    u, v = dev(c2["u0"], precision), dev(c2["v0"], precision)
    p.step(u, v, 1000)
    assert p.sync_status() == 0
    t = 1e-5 if precision == "fp32" else 1e-12
    _vs_golden(host(u), c2_golden, t, "u")
    _vs_golden(host(v), c2_golden, t, "v")


def test_c2_fp32_1000_steps_against_fp64(c2):
    """FP32 against the FP64 path over the same 1000 steps, whole field."""
    say("C2 1024^2 1000 steps fp32 vs fp64")
    out = {}
    for prec in ("fp64", "fp32"):
        p = _plan(c2, prec)
        u, v = dev(c2["u0"], prec), dev(c2["v0"], prec)
        p.step(u, v, 1000)
        assert p.sync_status() == 0
        out[prec] = host(u)
    assert parity_err(out["fp32"], out["fp64"]) <= 1e-5, parity_err(out["fp32"], out["fp64"])


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


@pytest.fixture(scope="module")
def c3_fp32_inputs(c3):
    """The 256^3 initial field rounded to FP32: both precisions receive
    exactly these values, so one oracle run serves both."""
    return as_seen(c3["u0"], "fp32"), as_seen(c3["v0"], "fp32")


@pytest.fixture(scope="module")
def c3_oracle_apply(c3, c3_fp32_inputs):
    g = O.gamma_from_Q(c3["Q"])
    O.set_fft_workers(16)
    try:
        return {op: O.mterm_apply(c3_fp32_inputs[0], O.seismic_op_order(g, op), c3["lo"], c3["hi"], c3["M"])
                for op in (1, 2)}
    finally:
        O.set_fft_workers(0)


@pytest.fixture(scope="module")
def c3_oracle_step(c3, c3_fp32_inputs):
    O.set_fft_workers(16)
    try:
        return O.tsfp2_seismic(c3_fp32_inputs[0], c3_fp32_inputs[1], O.gamma_from_Q(c3["Q"]), c3["c0"],
                               c3["omega0"], c3["lo"], c3["hi"], c3["M"], c3["dt"], 1)
    finally:
        O.set_fft_workers(0)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_c3_apply_full_field(c3, c3_fp32_inputs, c3_oracle_apply, precision):
    """(2.13) of L1 and L2 on the whole 256^3 field, in the benchmark's plan
    configuration, against the oracle (threaded library FFT), element-wise."""
    say(f"C3 256^3 apply {precision} full field vs oracle")
    p = _plan(c3, precision, max_batch=4)
    u = dev(c3_fp32_inputs[0], precision)
    t = 1e-5 if precision == "fp32" else 1e-12
    for op in (1, 2):
        out = host(p.apply(op, u))
        e = parity_err(out, c3_oracle_apply[op])
        say(f"  op {op}: parity err {e:.2e}")
        assert e <= t, (op, e)
    p.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_c3_one_step_full_field(c3, c3_fp32_inputs, c3_oracle_step, precision):
    """One TSFP2 step (3.13) of the 256^3 workload, whole field, both
    precisions, against the oracle; the FP32 plan runs the non-temporal
    kernel variants that switch on only above the last-level cache size."""
    say(f"C3 256^3 one step {precision} vs oracle (threaded library FFT)")
    p = _plan(c3, precision, max_batch=4)
    u, v = dev(c3_fp32_inputs[0], precision), dev(c3_fp32_inputs[1], precision)
    p.step(u, v, 1)
    assert p.sync_status() == 0
    ru, rv = c3_oracle_step
    eu, ev = parity_err(host(u), ru), parity_err(host(v), rv)
    say(f"  parity err u {eu:.2e} v {ev:.2e}")
    t = 1e-5 if precision == "fp32" else 1e-12
    assert eu <= t, eu
    assert ev <= t, ev
    p.close()


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
    assert parity_err(out["fp32"], out["fp64"]) <= 1e-5, parity_err(out["fp32"], out["fp64"])
