"""GPU parity of the Crank-Nicolson scheme CNFP (3.2) for the generic model
(1.5) against the FP64 oracle, and Table 2 (largest steps) on the GPU."""

import json
import os

import numpy as np
import pytest

import oracle as O
from gpu_helpers import as_seen, dev, host, parity_err, require_gpu, say, tol
from workloads import gaussian_pulse, grid_1d, mesh, paper_s1

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _plan(shape, lo, hi, precision, **kw):
    require_gpu()
    from paper_2311_13049_amd import vofl as V
    return V.Plan(shape, lo, hi, precision=precision, model="generic", **kw)


def _run(p, phi, psi, precision, steps, solver_tol):
    up, u = p.lffp_start(dev(phi, precision), dev(psi, precision))
    its = p.cnfp_step(up, u, steps - 1, tol=solver_tol, max_iter=300)
    return up, u, its


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_1d_example_41_vs_oracle(precision):
    J, lo, hi = 512, (-32.0,), (32.0,)
    x = grid_1d(J, lo[0], hi[0])
    s = paper_s1(x)
    phi, psi = np.exp(-x * x), np.zeros(J)
    dt, M, steps = 2.0 ** -8, 15, 20
    say(f"cnfp 1D J=512 {precision}")
    p = _plan((J,), lo, hi, precision, s=s, kappa=1.0, lam=1.0, M=M, dt=dt)
    up, u, its = _run(p, phi, psi, precision, steps, 1e-14 if precision == "fp64" else 1e-6)
    rp, ru = O.cnfp_generic(as_seen(phi, precision), psi, s, 1.0, lo, hi, M, dt, steps, f=lambda w: w ** 3)
    eu, ep = parity_err(host(u), ru), parity_err(host(up), rp)
    say(f"  BiCGSTAB iterations {its}; parity err u {eu:.2e} u_prev {ep:.2e}")
    assert eu <= tol(precision) and ep <= tol(precision)


def test_1d_table2_largest_steps_on_gpu():
    """Table 2, s = 1 column at tau = 2^-7 and 2^-8, against a GPU CNFP
    reference with tau = 1e-4 (see the oracle test for the choice of rows)."""
    tab = json.load(open(os.path.join(GOLD, "table2_cnfp_temporal.json")))
    col = tab["columns"].index("s=1")
    J, lo, hi = 4096, (-32.0,), (32.0,)
    x = grid_1d(J, lo[0], hi[0])
    phi = np.exp(-x * x)

    def run(dt, steps):
        p = _plan((J,), lo, hi, "fp64", s=np.ones(J), kappa=1.0, lam=1.0, M=15, dt=dt)
        _, u, _ = _run(p, phi, np.zeros(J), "fp64", steps, 1e-13)
        return host(u)
    say("table 2 reference: 10000 CNFP steps")
    ref = run(1e-4, 10000)
    for key in ("7", "8"):
        k = int(key)
        err = O.weighted_l2(run(2.0 ** -k, 2 ** k) - ref, 1.0 / 64)
        printed = float(tab["rows"][key][col])
        say(f"  tau 2^-{k}: {err:.4e} (printed {printed:.4e})")
        assert abs(err - printed) <= 5e-3 * printed


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(32, 64), (16, 16, 32)])
def test_nd_vs_oracle(shape, precision):
    lo = (-8.0,) * len(shape)
    hi = (8.0,) * len(shape)
    X = mesh(shape, lo, hi)
    s = 1.0 - 0.4 * np.cos(np.pi * X[0] / 4) * np.cos(np.pi * X[1] / 4)
    phi = gaussian_pulse(shape, lo, hi, [0.0] * len(shape))
    psi = 0.3 * gaussian_pulse(shape, lo, hi, [0.5] * len(shape))
    say(f"cnfp {shape} {precision}")
    p = _plan(shape, lo, hi, precision, s=s, kappa=0.7, lam=0.5, M=8, dt=5e-3)
    up, u, its = _run(p, phi, psi, precision, 8, 1e-13 if precision == "fp64" else 1e-6)
    rp, ru = O.cnfp_generic(as_seen(phi, precision), as_seen(psi, precision), s, 0.7, lo, hi, 8, 5e-3, 8,
                            f=lambda w: 0.5 * w ** 3)
    eu, ep = parity_err(host(u), ru), parity_err(host(up), rp)
    say(f"  BiCGSTAB iterations {its}; parity err u {eu:.2e} u_prev {ep:.2e}")
    assert eu <= tol(precision) and ep <= tol(precision)


def test_seismic_plans_are_rejected():
    require_gpu()
    from paper_2311_13049_amd import vofl as V
    shape, lo, hi = (16, 16), (-2.0, -2.0), (2.0, 2.0)
    x = dev(np.zeros(shape), "fp64")
    y = dev(np.zeros(shape), "fp64")
    p = V.Plan(shape, lo, hi, precision="fp64", Q=np.full(shape, 30.0), M=4, dt=1e-3)
    with pytest.raises(V.VoflError) as ei:
        p.cnfp_step(x, y, 1)
    assert ei.value.code == V.VOFL_ERR_UNSUPPORTED


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape,per_solve", [((256,), True), ((32, 48), True), ((32, 48), False)])
def test_batched_solves_vs_oracle(shape, per_solve, precision):
    """Three solves in one plan, each with its own s(x) (or one shared s),
    advanced one after another by vofl_cnfp_step; every solve against the
    oracle run on its own."""
    L = 32.0 if len(shape) == 1 else 8.0   # h = 1/4 in 1D: FFT rounding amplified by |mu_max|^{2s} stays small
    lo = (-L,) * len(shape)
    hi = (L,) * len(shape)
    X = mesh(shape, lo, hi)
    ss = [1.0 + a * np.sin(np.pi * X[0] / 8) * (np.cos(np.pi * X[-1] / 8) if len(shape) > 1 else 1.0)
          for a in (0.3, -0.2, 0.1)]
    if not per_solve:
        ss = [ss[0]] * 3
    phis = [gaussian_pulse(shape, lo, hi, [c] * len(shape)) for c in (0.0, 1.0, -1.5)]
    dt, M, steps = 5e-3, 8, 6
    say(f"cnfp batch 3 {shape} per_solve={per_solve} {precision}")
    p = _plan(shape, lo, hi, precision, s=np.stack(ss) if per_solve else ss[0], kappa=0.8, lam=0.4, M=M, dt=dt,
              batch=3, coef_per_solve=per_solve)
    up, u, its = _run(p, np.stack(phis), np.zeros((3,) + shape), precision, steps,
                      1e-14 if precision == "fp64" else 1e-6)
    hu = host(u).reshape((3,) + shape)
    hp = host(up).reshape((3,) + shape)
    for b in range(3):
        rp, ru = O.cnfp_generic(as_seen(phis[b], precision), np.zeros(shape), ss[b], 0.8, lo, hi, M, dt, steps,
                                f=lambda w: 0.4 * w ** 3)
        eu, ep = parity_err(hu[b], ru), parity_err(hp[b], rp)
        say(f"  solve {b}: parity err u {eu:.2e} u_prev {ep:.2e}")
        assert eu <= tol(precision) and ep <= tol(precision)
    say(f"  BiCGSTAB iterations (all solves) {its}")
