"""Pins for the oracle's leap-frog scheme for the viscoacoustic model (1.1)
(lffp_seismic) and for per-point phase velocities in tsfp2_seismic.

The paper solves (1.1) with the leap-frog scheme (Example 3) without writing
the discretisation of the damping term out; the oracle takes the backward
difference (u^n - u^{n-1})/dt there and the Taylor start of (3.4c). The
expected values below come from closed forms of the per-mode recurrence and
from a high-order ODE integration of the semi-discrete system, never from the
oracle itself.
"""

import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import (dense_matrix_1d, gamma_from_Q, lffp_seismic, seismic_coefficients,
                    tsfp2_seismic)
from workloads import grid_1d, mesh


def _mode_recurrence(a, b, u0, u1, n):
    """u^n of u^{k+1} = (2 - a - b) u^k - (1 - b) u^{k-1} from its characteristic roots."""
    p, q = 2.0 - a - b, 1.0 - b
    disc = complex(p * p - 4.0 * q)
    r1 = (p + np.sqrt(disc)) / 2.0
    r2 = (p - np.sqrt(disc)) / 2.0
    c2 = (u1 - r1 * u0) / (r2 - r1)
    c1 = u0 - c2
    return (c1 * r1 ** n + c2 * r2 ** n).real


@pytest.mark.parametrize("k", [(1, 0), (2, 3), (5, 1)])
def test_gamma_zero_is_the_classical_leapfrog(k):
    """Q = inf (gamma = 0): A = c0^2, B = 0 and L1 = -Lap, so one mode
    cos(mu.x) with psi = 0 follows u^n = cos(n theta) u^0, cos(theta) =
    1 - dt^2 c0^2 |mu|^2 / 2 (2D)."""
    shape, lo, hi = (16, 24), (-2.0, 0.0), (2.0, 3.0)
    X, Y = mesh(shape, lo, hi)
    mx = 2 * np.pi * k[0] / (hi[0] - lo[0])
    my = 2 * np.pi * k[1] / (hi[1] - lo[1])
    u0 = np.cos(mx * (X - lo[0]) + my * (Y - lo[1]))
    c0, dt, steps = 1.3, 2e-3, 41
    gamma = gamma_from_Q(np.full(shape, np.inf))
    theta = math.acos(1 - 0.5 * dt * dt * c0 * c0 * (mx * mx + my * my))
    prev, cur = lffp_seismic(u0, np.zeros(shape), gamma, c0, 3.0, lo, hi, 4, dt, steps)
    np.testing.assert_allclose(cur, math.cos(steps * theta) * u0, atol=1e-12)
    np.testing.assert_allclose(prev, math.cos((steps - 1) * theta) * u0, atol=1e-12)


@pytest.mark.parametrize("Q,c0,w0,k", [(20.0, 1.0, 1.0, 3), (2.0, 1.4, 2.5, 5), (0.7, 0.8, 0.5, 2)])
def test_constant_gamma_mode_follows_the_damped_recurrence(Q, c0, w0, k):
    """Constant gamma: per mode with P1 = |mu|^{2(1+gamma)}, P2 = |mu|^{1+2 gamma},
    a = dt^2 A P1, b = dt B P2, the scheme is u^{n+1} = (2-a-b) u^n - (1-b) u^{n-1}
    with u^1 = u^0 + dt v^0 - (a/2) u^0 - (dt b/2) v^0 for u^0 = cos, v^0 = psi
    amplitudes; the characteristic roots give u^n in closed form."""
    n, lo, hi = 32, (0.0,), (2 * np.pi,)
    x = grid_1d(n, lo[0], hi[0])
    mode = np.cos(k * x)
    g = float(gamma_from_Q(Q))
    A, B = (float(z) for z in seismic_coefficients(g, c0, w0))
    dt, steps = 4e-3, 60
    P1, P2 = k ** (2 * (1 + g)), k ** (1 + 2 * g)
    a, b = dt * dt * A * P1, dt * B * P2
    for amp_u, amp_v in ((1.0, 0.0), (0.0, 1.0), (0.7, -0.4)):
        u1 = amp_u + dt * amp_v - 0.5 * a * amp_u - 0.5 * dt * b * amp_v
        prev, cur = lffp_seismic(amp_u * mode, amp_v * mode, np.full(n, g), c0, w0, lo, hi, 3, dt, steps)
        np.testing.assert_allclose(cur, _mode_recurrence(a, b, amp_u, u1, steps) * mode, atol=1e-12)
        np.testing.assert_allclose(prev, _mode_recurrence(a, b, amp_u, u1, steps - 1) * mode, atol=1e-12)


def test_zero_and_one_step():
    x = grid_1d(16, -1.0, 1.0)
    phi, psi = np.exp(-x * x), np.sin(np.pi * x)
    prev, cur = lffp_seismic(phi, psi, np.full(16, 0.02), 1.0, 1.0, (-1.0,), (1.0,), 2, 1e-2, 0)
    assert np.array_equal(prev, phi) and np.array_equal(cur, phi)
    prev, cur = lffp_seismic(phi, psi, np.full(16, 0.02), 1.0, 1.0, (-1.0,), (1.0,), 2, 1e-2, 1)
    assert np.array_equal(prev, phi)
    assert np.abs(cur - (phi + 1e-2 * psi)).max() < 1e-3


def _mol(u0, v0, A, B, L1, L2, t):
    n = u0.size

    def rhs(_, y):
        u, v = y[:n], y[n:]
        return np.concatenate([v, -A * (L1 @ u) - B * (L2 @ v)])
    sol = solve_ivp(rhs, (0.0, t), np.concatenate([u0, v0]), method="DOP853", rtol=1e-12, atol=1e-14)
    return sol.y[:n, -1]


def _layered(x, lo, hi):
    """Smooth two-layer phase velocity on the periodic interval: 11/18 and 1."""
    L = hi - lo
    z = (x - lo) / L
    return 1.0 - (1.0 - 11.0 / 18.0) * 0.5 * (np.tanh(8 * (z - 0.25)) - np.tanh(8 * (z - 0.75)))


def test_variable_gamma_and_layered_c0_converge_at_first_order():
    """The damping term's backward difference makes the scheme first order:
    halving dt halves the error against the semi-discrete solution (exact
    discrete operators (2.7); M = 30 leaves no visible expansion error)."""
    J, lo, hi = 32, -8.0, 8.0
    x = grid_1d(J, lo, hi)
    gamma = gamma_from_Q(1.2 + 0.8 * np.sin(np.pi * x / 8.0))
    c0 = _layered(x, lo, hi)
    A, B = seismic_coefficients(gamma, c0, 2.0)
    L1 = dense_matrix_1d(1.0 + gamma, lo, hi)
    L2 = dense_matrix_1d(0.5 + gamma, lo, hi)
    u0, v0 = np.exp(-x * x), 0.3 * np.exp(-(x - 1) ** 2)
    t = 0.5
    ref = _mol(u0, v0, A, B, L1, L2, t)
    errs = []
    for steps in (100, 200, 400, 800):
        _, u = lffp_seismic(u0, v0, gamma, c0, 2.0, (lo,), (hi,), 30, t / steps, steps)
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    rates = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(0.85 < r < 1.3 for r in rates), (errs, rates)
    assert errs[-1] < 2e-3


def test_undamped_layered_medium_converges_at_second_order():
    """gamma = 0 with a layered c0 (B = 0, A = c0(x)^2): the classical
    leap-frog for a variable-speed wave equation, second order in dt."""
    J, lo, hi = 32, -8.0, 8.0
    x = grid_1d(J, lo, hi)
    gamma = np.zeros(J)
    c0 = _layered(x, lo, hi)
    A, B = seismic_coefficients(gamma, c0, 1.0)
    assert np.all(B == 0.0)
    L1 = dense_matrix_1d(np.ones(J), lo, hi)
    u0, v0 = np.exp(-x * x), np.zeros(J)
    t = 0.5
    ref = _mol(u0, v0, A, B, L1, L1, t)
    errs = []
    for steps in (50, 100, 200):
        _, u = lffp_seismic(u0, v0, gamma, c0, 1.0, (lo,), (hi,), 4, t / steps, steps)
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    rates = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(r > 1.9 for r in rates), (errs, rates)


def test_tsfp2_layered_c0_converges_to_method_of_lines():
    """TSFP2 for (1.1) with per-point c0 (exact part at the mean c0) converges
    to the semi-discrete solution with A(x), B(x) from c0(x)."""
    J, lo, hi = 32, -8.0, 8.0
    x = grid_1d(J, lo, hi)
    gamma = gamma_from_Q(1.2 + 0.8 * np.sin(np.pi * x / 8.0))
    c0 = _layered(x, lo, hi)
    A, B = seismic_coefficients(gamma, c0, 2.0)
    L1 = dense_matrix_1d(1.0 + gamma, lo, hi)
    L2 = dense_matrix_1d(0.5 + gamma, lo, hi)
    u0, v0 = np.exp(-x * x), 0.3 * np.exp(-(x - 1) ** 2)
    t = 0.5
    ref = _mol(u0, v0, A, B, L1, L2, t)
    errs = []
    for steps in (50, 100, 200, 400):
        u, _ = tsfp2_seismic(u0, v0, gamma, c0, 2.0, (lo,), (hi,), 30, t / steps, steps)
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    rates = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(r > 0.9 for r in rates), (errs, rates)
    assert errs[-1] < 1e-3


def test_scalar_c0_field_equals_scalar():
    """A constant c0 field gives the same result as the scalar c0 (both schemes)."""
    x = grid_1d(32, -4.0, 4.0)
    gamma = gamma_from_Q(5.0 + 3.0 * np.cos(np.pi * x / 4.0))
    u0 = np.exp(-x * x)
    for fn in (lffp_seismic, tsfp2_seismic):
        a = fn(u0, np.zeros(32), gamma, 1.2, 1.5, (-4.0,), (4.0,), 6, 1e-2, 20)
        b = fn(u0, np.zeros(32), gamma, np.full(32, 1.2), 1.5, (-4.0,), (4.0,), 6, 1e-2, 20)
        for p, q in zip(a, b):
            np.testing.assert_allclose(p, q, rtol=0, atol=1e-15)
