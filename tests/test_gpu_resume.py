"""Resumable TSFP2 runs (vofl_step_begin / vofl_step_advance / vofl_step_end):
the spectral state kept in the plan between calls gives vofl_step's result
bit for bit in 2D/3D, however the steps are split and whether or not the
chunks are graph replays, and matches the FP64 oracle."""

import numpy as np
import pytest

import oracle as O
from gpu_helpers import as_seen, dev, host, parity_err, require_gpu, say, tol
from workloads import gaussian_pulse, grf_Q, mesh, rng_for

pytestmark = pytest.mark.gpu


def _seismic(shape, precision, batch=1, M=6, dt=2e-3):
    require_gpu()
    from paper_2311_13049_amd import vofl as V
    lo = tuple(-0.25 * n for n in shape)
    hi = tuple(0.25 * n for n in shape)
    Q = grf_Q(shape, lo, hi, rng_for(93, len(shape)), corr_len=1.0, qmin=2.0, qmax=40.0)
    u0 = gaussian_pulse(shape, lo, hi, [0.1] * len(shape))
    v0 = 0.3 * gaussian_pulse(shape, lo, hi, [-0.2] * len(shape))
    if batch > 1:
        u0 = np.stack([u0, 0.5 * u0[::-1].copy()])
        v0 = np.stack([v0, -v0])
    p = V.Plan(shape, lo, hi, Q=Q, M=M, dt=dt, precision=precision, batch=batch)
    return p, lo, hi, Q, u0, v0


def _chunked(p, u0, v0, precision, chunks, graph=False):
    u, v = dev(u0, precision), dev(v0, precision)
    p.begin(u, v)
    for k in chunks:
        p.advance(k, graph=graph)
    ou, ov = dev(np.zeros_like(u0), precision), dev(np.zeros_like(v0), precision)
    p.end(ou, ov)
    return ou, ov


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(32, 16, 16), (48, 32)])
def test_chunks_equal_one_call_bitwise(shape, precision):
    import torch
    say(f"resume {shape} {precision}")
    p, lo, hi, Q, u0, v0 = _seismic(shape, precision)
    u, v = dev(u0, precision), dev(v0, precision)
    p.step(u, v, 7)
    for chunks, graph in (((3, 1, 3), False), ((1,) * 7, False), ((7,), True), ((2, 2, 3), True)):
        ou, ov = _chunked(p, u0, v0, precision, chunks, graph)
        assert torch.equal(ou, u) and torch.equal(ov, v), (chunks, graph)
    assert p.sync_status() == 0


def test_end_mid_run_and_continue_fp64():
    """end() leaves the run open: reading the fields after 4 steps and again
    after 7 gives vofl_step's 4- and 7-step results, and the oracle's."""
    import torch
    shape = (32, 16, 16)
    p, lo, hi, Q, u0, v0 = _seismic(shape, "fp64")
    u, v = dev(u0, "fp64"), dev(v0, "fp64")
    p.begin(u, v)
    p.advance(4)
    u4, v4 = dev(np.zeros(shape), "fp64"), dev(np.zeros(shape), "fp64")
    p.end(u4, v4)
    p.advance(3, graph=True)
    u7, v7 = dev(np.zeros(shape), "fp64"), dev(np.zeros(shape), "fp64")
    p.end(u7, v7)
    for n, (a, b) in ((4, (u4, v4)), (7, (u7, v7))):
        ru, rv = dev(u0, "fp64"), dev(v0, "fp64")
        p.step(ru, rv, n)
        assert torch.equal(a, ru) and torch.equal(b, rv), n
    ou, ov = O.tsfp2_seismic(u0, v0, O.gamma_from_Q(Q), 1.0, 1.0, lo, hi, 6, 2e-3, 7)
    assert parity_err(host(u7), ou) <= 1e-12
    assert parity_err(host(v7), ov) <= 1e-12


def test_end_right_after_begin_returns_the_input():
    shape = (16, 32)
    p, lo, hi, Q, u0, v0 = _seismic(shape, "fp64")
    ou, ov = _chunked(p, u0, v0, "fp64", ())
    assert parity_err(host(ou), u0) <= 1e-14 and parity_err(host(ov), v0) <= 1e-14


def test_batched_plan_chunks_bitwise():
    import torch
    shape = (32, 32)
    p, lo, hi, Q, u0, v0 = _seismic(shape, "fp32", batch=2)
    u, v = dev(u0, "fp32"), dev(v0, "fp32")
    p.step(u, v, 5)
    ou, ov = _chunked(p, u0, v0, "fp32", (2, 3), graph=True)
    assert torch.equal(ou, u) and torch.equal(ov, v)


def test_generic_fourth_order_chunks_bitwise():
    """The generic model with the fourth-order composition (three sub-steps
    per step): the pending half sub-step spans the step boundary."""
    import torch
    from paper_2311_13049_amd import vofl as V
    shape, lo, hi = (32, 32), (-8.0, -8.0), (8.0, 8.0)
    X = mesh(shape, lo, hi)
    s = 1.0 - 0.3 * np.cos(np.pi * X[0] / 4) * np.cos(np.pi * X[1] / 4)
    u0 = gaussian_pulse(shape, lo, hi, (0.0, 0.0))
    p = V.Plan(shape, lo, hi, precision="fp64", model="generic", s=s, kappa=0.7, lam=0.5, M=8, dt=2e-3,
               order=4)
    u, v = dev(u0, "fp64"), dev(np.zeros(shape), "fp64")
    p.step(u, v, 5)
    ou, ov = _chunked(p, u0, np.zeros(shape), "fp64", (1, 4))
    assert torch.equal(ou, u) and torch.equal(ov, v)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_1d_chunks_match_one_call(precision):
    from paper_2311_13049_amd import vofl as V
    require_gpu()
    J, lo, hi = 256, (-16.0,), (16.0,)
    x = lo[0] + (hi[0] - lo[0]) * np.arange(J) / J
    gamma = 0.1 + 0.05 * np.sin(np.pi * x / 16)
    u0 = np.exp(-x * x)
    p = V.Plan((J,), lo, hi, gamma=gamma, M=8, dt=1e-3, precision=precision)
    u, v = dev(u0, precision), dev(np.zeros(J), precision)
    p.step(u, v, 20)
    ou, ov = _chunked(p, u0, np.zeros(J), precision, (5, 15))
    assert parity_err(host(ou), host(u)) <= tol(precision)
    ref, _ = O.tsfp2_seismic(as_seen(u0, precision), np.zeros(J), gamma, 1.0, 1.0, lo, hi, 8, 1e-3, 20)
    assert parity_err(host(ou), ref) <= tol(precision)


def test_run_is_closed_by_other_calls():
    from paper_2311_13049_amd import vofl as V
    shape = (16, 32)
    p, lo, hi, Q, u0, v0 = _seismic(shape, "fp64")
    with pytest.raises(V.VoflError) as ei:
        p.advance(1)
    assert ei.value.code == V.VOFL_ERR_INVALID
    u, v = dev(u0, "fp64"), dev(v0, "fp64")
    p.begin(u, v)
    p.advance(1)
    p.apply(V.VOFL_OP_S1, u)           # reuses the run's buffers: the run ends
    with pytest.raises(V.VoflError) as ei:
        p.end(u, v)
    assert ei.value.code == V.VOFL_ERR_INVALID
