"""GPU parity of the leap-frog scheme for the viscoacoustic model (1.1)
(vofl_lffp_start / vofl_lffp_step on seismic plans) against the FP64 oracle
lffp_seismic, including per-point phase velocities (c0_field) and the
two-layer medium of Example 3 (Section 4).
"""

import math

import numpy as np
import pytest

import oracle as O
from gpu_helpers import as_seen, dev, host, parity_err, require_gpu, say, tol
from workloads import c1_inputs, ex3_inputs, gaussian_pulse, grf_Q, grid_1d, mesh, rng_for, ricker

pytestmark = pytest.mark.gpu


def _plan(shape, lo, hi, precision, **kw):
    require_gpu()
    from paper_2311_13049_amd import vofl as V
    return V.Plan(shape, lo, hi, precision=precision, model="seismic", **kw)


def _run_gpu(p, phi, psi, precision, nsteps):
    up, u = p.lffp_start(dev(phi, precision), dev(psi, precision))
    if nsteps > 1:
        p.lffp_step(up, u, nsteps - 1)
    assert p.sync_status() == 0
    return host(up), host(u)


def _layers(shape, lo, hi):
    """Ex. 3 structure on a small box: gamma = a1 + a2 tanh(100(y-1)) and c0 = 11/18 above y = 1."""
    _, Y = mesh(shape, lo, hi)
    return 0.02 + 0.01 * np.tanh(100.0 * (Y - 1.0)), np.where(Y > 1.0, 11.0 / 18.0, 1.0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_1d_c1_vs_oracle(precision):
    """1D n = 256, gamma given, M = 8, 100 steps (one kernel for the whole run)."""
    c = c1_inputs()
    say(f"lffp seismic 1D n=256 {precision}")
    p = _plan((256,), c["lo"], c["hi"], precision, gamma=c["gamma"], c0=1.3, omega0=0.7,
              M=c["M"], dt=c["dt"])
    x = grid_1d(256, c["lo"][0], c["hi"][0])
    psi = 0.2 * np.exp(-(x - 2.0) ** 2)
    up, u = _run_gpu(p, c["u0"], psi, precision, 100)
    rp, ru = O.lffp_seismic(as_seen(c["u0"], precision), as_seen(psi, precision), c["gamma"], 1.3, 0.7,
                            c["lo"], c["hi"], c["M"], c["dt"], 100)
    eu, ep = parity_err(u, ru), parity_err(up, rp)
    say(f"  parity err u {eu:.2e} u_prev {ep:.2e}")
    assert eu <= tol(precision) and ep <= tol(precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(64, 96), (48, 128)])
def test_2d_layered_medium_vs_oracle(precision, shape):
    """Two-layer gamma and phase velocity (Ex. 3 structure) on [0,2)^2, a
    Ricker pulse resolved on the grid (nu0 = 4), 60 steps, M = 6."""
    lo, hi = (0.0, 0.0), (2.0, 2.0)
    gamma, c0 = _layers(shape, lo, hi)
    phi = ricker(shape, lo, hi, (1.0, 0.85), 4.0)
    psi = 0.1 * phi
    dt, M, steps = 2e-3, 6, 60
    say(f"lffp seismic 2D {shape} {precision}")
    p = _plan(shape, lo, hi, precision, gamma=gamma, c0_field=c0, omega0=1.0, M=M, dt=dt)
    up, u = _run_gpu(p, phi, psi, precision, steps)
    rp, ru = O.lffp_seismic(as_seen(phi, precision), as_seen(psi, precision), gamma, c0, 1.0, lo, hi, M, dt,
                            steps)
    eu, ep = parity_err(u, ru), parity_err(up, rp)
    say(f"  parity err u {eu:.2e} u_prev {ep:.2e}")
    assert eu <= tol(precision) and ep <= tol(precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_3d_batch_own_coefficients_vs_oracle(precision):
    """3D 16 x 48 x 32, two solves with their own Q and c0 fields (coef_per_solve), 30 steps."""
    shape, lo, hi = (16, 48, 32), (-4.0, -6.0, -8.0), (4.0, 6.0, 8.0)
    rng = rng_for(91)
    Qs = [grf_Q(shape, lo, hi, rng, corr_len=2.0, qmin=2.0, qmax=40.0) for _ in range(2)]
    X = mesh(shape, lo, hi)
    c0s = [1.0 + 0.2 * np.tanh(X[2]), 0.8 + 0.1 * np.cos(np.pi * X[0] / 4.0)]
    u0s = [gaussian_pulse(shape, lo, hi, (0.5, -1.0, 1.0)), gaussian_pulse(shape, lo, hi, (-1.0, 2.0, 0.0))]
    dt, M, steps = 5e-3, 8, 30
    say(f"lffp seismic 3D {shape} x 2 {precision}")
    p = _plan(shape, lo, hi, precision, Q=np.stack(Qs), c0_field=np.stack(c0s), omega0=1.5, M=M, dt=dt,
              batch=2, coef_per_solve=True)
    up, u = _run_gpu(p, np.stack(u0s), np.zeros((2,) + shape), precision, steps)
    u = u.reshape((2,) + shape)
    up = up.reshape((2,) + shape)
    for b in range(2):
        rp, ru = O.lffp_seismic(as_seen(u0s[b], precision), np.zeros(shape), O.gamma_from_Q(Qs[b]), c0s[b], 1.5,
                                lo, hi, M, dt, steps)
        eu, ep = parity_err(u[b], ru), parity_err(up[b], rp)
        say(f"  solve {b}: parity err u {eu:.2e} u_prev {ep:.2e}")
        assert eu <= tol(precision) and ep <= tol(precision)


def test_gamma_zero_single_mode_is_the_classical_leapfrog():
    """Q = inf: the GPU path follows u^n = cos(n theta) u^0, cos(theta) =
    1 - dt^2 c0^2 |mu|^2 / 2, for one mode in 2D (FP64)."""
    shape, lo, hi = (32, 48), (0.0, 0.0), (2.0, 3.0)
    X, Y = mesh(shape, lo, hi)
    mx, my = 2 * np.pi * 3 / 2.0, 2 * np.pi * 2 / 3.0
    u0 = np.cos(mx * X + my * Y)
    c0, dt, steps = 1.2, 1e-3, 150
    p = _plan(shape, lo, hi, "fp64", Q=np.full(shape, np.inf), c0=c0, omega0=1.0, M=4, dt=dt)
    up, u = _run_gpu(p, u0, np.zeros(shape), "fp64", steps)
    theta = math.acos(1 - 0.5 * dt * dt * c0 * c0 * (mx * mx + my * my))
    say(f"gamma = 0 mode: max err {np.abs(u - math.cos(steps * theta) * u0).max():.2e}")
    np.testing.assert_allclose(u, math.cos(steps * theta) * u0, atol=1e-12)
    np.testing.assert_allclose(up, math.cos((steps - 1) * theta) * u0, atol=1e-12)


def test_restart_equals_one_call():
    """k steps then m steps equal k + m steps in one call (the first call's
    later steps and the restart use the same difference quotient)."""
    import torch
    shape, lo, hi = (32, 32), (0.0, 0.0), (2.0, 2.0)
    gamma, c0 = _layers(shape, lo, hi)
    phi = ricker(shape, lo, hi, (1.0, 0.85), 3.0)
    p = _plan(shape, lo, hi, "fp64", gamma=gamma, c0_field=c0, M=5, dt=2e-3)
    a_prev, a = p.lffp_start(dev(phi, "fp64"), dev(np.zeros(shape), "fp64"))
    b_prev, b = a_prev.clone(), a.clone()
    p.lffp_step(a_prev, a, 20)
    p.lffp_step(b_prev, b, 7)
    p.lffp_step(b_prev, b, 13)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a_prev, b_prev)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_example3_full_grid_vs_oracle(precision):
    """Example 3 at the paper's mesh h = 0.002 (1000 x 1000 on [0,2)^2),
    case a1 = 0.02, a2 = 0.01, M = 8, dt = 1e-4, 10 steps, against the oracle
    (the only configuration of the paper that uses a per-point c0)."""
    ex = ex3_inputs(1000, case=1)
    from paper_2311_13049_amd import vofl as V
    require_gpu()
    try:
        p = _plan(ex["shape"], ex["lo"], ex["hi"], precision, gamma=ex["gamma"], c0_field=ex["c0"],
                  omega0=ex["omega0"], M=ex["M"], dt=ex["dt"])
    except V.VoflError as e:
        if e.code == V.VOFL_ERR_UNSUPPORTED:
            pytest.skip("no compiled transform of length 1000")
        raise
    steps = 10
    say(f"example 3 1000^2 {precision}, {steps} steps")
    up, u = _run_gpu(p, ex["phi"], ex["psi"], precision, steps)
    O.set_fft_workers(8)
    try:
        rp, ru = O.lffp_seismic(as_seen(ex["phi"], precision), ex["psi"], ex["gamma"], ex["c0"], ex["omega0"],
                                ex["lo"], ex["hi"], ex["M"], ex["dt"], steps)
    finally:
        O.set_fft_workers(0)
    eu = parity_err(u.reshape(ex["shape"]), ru)
    say(f"  parity err u {eu:.2e}")
    assert eu <= tol(precision)


def test_unstable_step_sets_flag():
    """dt far above the leap-frog limit (dt c0 |mu|_max^{1+gamma} >> 2): the
    state overflows and the device flag reports VOFL_ERR_UNSTABLE."""
    from paper_2311_13049_amd import vofl as V
    shape, lo, hi = (32, 32), (0.0, 0.0), (2.0, 2.0)
    gamma, c0 = _layers(shape, lo, hi)
    phi = ricker(shape, lo, hi, (1.0, 0.85), 3.0)
    p = _plan(shape, lo, hi, "fp64", gamma=gamma, c0_field=c0, M=4, dt=0.5)
    up, u = p.lffp_start(dev(phi, "fp64"), dev(np.zeros(shape), "fp64"))
    p.lffp_step(up, u, 2000)
    assert p.sync_status() == V.VOFL_ERR_UNSTABLE


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_1d_batch_own_gamma_and_c0_vs_oracle(precision):
    """1D, three solves with their own gamma and c0 fields in one kernel launch."""
    n, lo, hi = 256, (-16.0,), (16.0,)
    x = grid_1d(n, lo[0], hi[0])
    gammas = [0.05 + 0.03 * np.sin(np.pi * x / 8.0 + k) for k in range(3)]
    c0s = [1.0 + 0.2 * np.tanh(x - k) for k in range(3)]
    phis = [np.exp(-(x - k) ** 2) for k in range(3)]
    dt, M, steps = 1e-3, 8, 80
    say(f"lffp seismic 1D batch 3 {precision}")
    p = _plan((n,), lo, hi, precision, gamma=np.stack(gammas), c0_field=np.stack(c0s), omega0=1.2, M=M, dt=dt,
              batch=3, coef_per_solve=True)
    up, u = _run_gpu(p, np.stack(phis), np.zeros((3, n)), precision, steps)
    u = u.reshape(3, n)
    for b in range(3):
        _, ru = O.lffp_seismic(as_seen(phis[b], precision), np.zeros(n), gammas[b], c0s[b], 1.2, lo, hi, M, dt,
                               steps)
        e = parity_err(u[b], ru)
        say(f"  solve {b}: parity err u {e:.2e}")
        assert e <= tol(precision)


def test_2d_radix3_grid_vs_oracle():
    """768 x 96 (radix-3 lengths on both axes), layered medium, FP64."""
    shape, lo, hi = (768, 96), (0.0, 0.0), (12.0, 1.5)
    gamma, c0 = _layers(shape, lo, hi)
    phi = ricker(shape, lo, hi, (6.0, 0.7), 2.0)
    dt, M, steps = 2e-3, 6, 25
    say("lffp seismic 2D 768 x 96 fp64")
    p = _plan(shape, lo, hi, "fp64", gamma=gamma, c0_field=c0, M=M, dt=dt)
    up, u = _run_gpu(p, phi, np.zeros(shape), "fp64", steps)
    _, ru = O.lffp_seismic(phi, np.zeros(shape), gamma, c0, 1.0, lo, hi, M, dt, steps)
    e = parity_err(u.reshape(shape), ru)
    say(f"  parity err u {e:.2e}")
    assert e <= tol("fp64")
