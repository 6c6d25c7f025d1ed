"""Pins for the oracle's Crank-Nicolson scheme CNFP (3.2)-(3.3) for (1.5).

Expected values: the paper's Table 2 at the two largest steps (where the
reference solution's own error does not matter), the closed-form solution of
the Crank-Nicolson recurrence on one Fourier mode, and second-order
convergence to an independent method-of-lines solution.
"""

import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import cnfp_generic, dense_matrix_1d, weighted_l2
from workloads import grid_1d

GOLD = os.path.join(os.path.dirname(__file__), "golden")
LO, HI = (-32.0,), (32.0,)


def test_single_mode_closed_form():
    """f = 0, constant order: (1 + a w^2)(u^{n+1} + u^{n-1}) = 2 u^n, a = dt^2/2,
    w^2 = kappa |mu|^{2s}; with u^0 = cos(mu x) and the start (3.3b)
    u^1 = (1 - dt^2 w^2 / 2) u^0, u^n = [cos(n t) + B sin(n t)] u^0 with
    cos(t) = 1/(1 + a w^2), B = (u^1/u^0 - cos t)/sin t."""
    n, lo, hi = 64, (-4.0,), (4.0,)
    x = grid_1d(n, lo[0], hi[0])
    k, s, kappa, dt, steps = 5, 1.2, 0.8, 3e-3, 40
    mu = 2 * np.pi * k / (hi[0] - lo[0])
    u0 = np.cos(mu * (x - lo[0]))
    w2 = kappa * mu ** (2 * s)
    c = 1.0 / (1.0 + 0.5 * dt * dt * w2)
    th = math.acos(c)
    g1 = 1.0 - 0.5 * dt * dt * w2
    B = (g1 - c) / math.sin(th)
    _, cur = cnfp_generic(u0, np.zeros(n), np.full(n, s), kappa, lo, hi, 4, dt, steps)
    np.testing.assert_allclose(cur, (math.cos(steps * th) + B * math.sin(steps * th)) * u0, atol=1e-12)


def test_second_order_convergence_to_method_of_lines():
    J, lo, hi = 32, -8.0, 8.0
    x = grid_1d(J, lo, hi)
    s = 1.0 + 0.3 * np.sin(np.pi * x / 8.0)
    kap = 0.9
    L = dense_matrix_1d(s, lo, hi)
    u0 = np.exp(-x * x)

    def rhs(_, y):
        u, v = y[:J], y[J:]
        return np.concatenate([v, -kap * (L @ u) + u ** 3])
    t = 0.5
    ref = solve_ivp(rhs, (0, t), np.concatenate([u0, np.zeros(J)]), method="DOP853",
                    rtol=1e-12, atol=1e-14).y[:J, -1]
    errs = []
    for steps in (50, 100, 200):
        _, u = cnfp_generic(u0, np.zeros(J), s, kap, (lo,), (hi,), 30, t / steps, steps, f=lambda w: w ** 3)
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    rates = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(1.8 < r < 2.3 for r in rates), (errs, rates)


@pytest.mark.slow
def test_table2_largest_steps():
    """Table 2, s = 1 column, tau = 2^-7 and 2^-8 against a CNFP reference with
    tau = 1e-4. (At smaller steps the printed errors sit a nearly constant
    1.9e-8 below these, so the paper's reference differs from this one; see
    the design notes. The largest two steps are insensitive to that.)"""
    tab = json.load(open(os.path.join(GOLD, "table2_cnfp_temporal.json")))
    col = tab["columns"].index("s=1")
    J = 4096
    x = grid_1d(J, LO[0], HI[0])
    phi, s = np.exp(-x * x), np.ones(J)

    def run(dt, steps):
        return cnfp_generic(phi, np.zeros(J), s, 1.0, LO, HI, 15, dt, steps, f=lambda w: w ** 3)[1]
    ref = run(1e-4, 10000)
    for key in ("7", "8"):
        k = int(key)
        printed = float(tab["rows"][key][col])
        err = weighted_l2(run(2.0 ** -k, 2 ** k) - ref, 1.0 / 64)
        assert abs(err - printed) <= 5e-3 * printed, (key, err, printed)
