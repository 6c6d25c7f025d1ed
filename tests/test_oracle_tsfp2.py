"""Pins for the oracle's time integrators (TSFP2 for (1.5) and for (1.1)).

Expected values come from the paper's printed tables (tests/golden/), from
closed-form solutions (d'Alembert, matrix exponentials of the mode ODEs), or
from an independent high-order ODE integration of the semi-discrete system.
"""

import json
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

from oracle import (damped_propagator, dense_matrix_1d, gamma_from_Q,
                    seismic_coefficients, tsfp2_generic, tsfp2_seismic,
                    weighted_l2)
from workloads import grid_1d, paper_s1, paper_s2

GOLD = os.path.join(os.path.dirname(__file__), "golden")
LO, HI = (-32.0,), (32.0,)


def _ex1(J, s_fn, dt, steps, M=15):
    """Problem (4.1): kappa = 1, f(u) = u^3, [-32, 32], u0 = exp(-x^2), v0 = 0."""
    x = grid_1d(J, LO[0], HI[0])
    s = s_fn(x) if callable(s_fn) else np.full(J, float(s_fn))
    u, _ = tsfp2_generic(np.exp(-x * x), np.zeros(J), s, 1.0, LO, HI, M, dt, steps,
                         f=lambda u: u ** 3)
    return u


@pytest.fixture(scope="module")
def references():
    """Reference solutions of Tables 4-5: h = 1/64, tau = 1e-4, t = 1."""
    return {"s=1": _ex1(4096, 1.0, 1e-4, 10000), "s1": _ex1(4096, paper_s1, 1e-4, 10000)}


@pytest.mark.slow
def test_table4_temporal_errors(references):
    """Table 4: TSFP2 temporal errors at t = 1, h = 1/64, to the printed digits."""
    tab = json.load(open(os.path.join(GOLD, "table4_tsfp2_temporal.json")))
    cols = tab["columns"]
    for col, s_fn in (("s=1", 1.0), ("s1", paper_s1)):
        for key in ("9", "10", "11"):
            k = int(key)
            printed = float(tab["rows"][key][cols.index(col)])
            u = _ex1(4096, s_fn, 2.0 ** -k, 2 ** k)
            err = weighted_l2(u - references[col], 1.0 / 64)
            assert abs(err - printed) <= 6e-4 * printed, (col, key, err, printed)


@pytest.mark.slow
def test_table5_spatial_errors(references):
    """Table 5: TSFP2 spatial errors at t = 1, tau = 1e-4, h = 1/2 and 1/4."""
    tab = json.load(open(os.path.join(GOLD, "table5_tsfp2_spatial.json")))
    cols = tab["columns"]
    for col, s_fn in (("s=1", 1.0), ("s1", paper_s1)):
        for key in ("0.5", "0.25"):
            h = float(key)
            J = int(round(64 / h))
            printed = float(tab["rows"][key][cols.index(col)])
            u = _ex1(J, s_fn, 1e-4, 10000)
            err = weighted_l2(u - references[col][:: 4096 // J], h)
            assert abs(err - printed) <= 6e-4 * printed, (col, key, err, printed)


def test_table4_unstable_entries():
    """Table 4: 'unstable' for s1 at tau = 2^-7, 2^-8 and for s2 at 2^-7; s2 at 2^-8 stays finite."""
    def blows_up(s_fn, k):
        u = _ex1(4096, s_fn, 2.0 ** -k, 2 ** k)
        return (not np.all(np.isfinite(u))) or np.max(np.abs(u)) > 1e3
    assert blows_up(paper_s1, 7)
    assert blows_up(paper_s1, 8)
    assert blows_up(paper_s2, 7)
    assert not blows_up(paper_s2, 8)


def test_constant_order_linear_is_exact_in_time():
    """Remark 3.1: constant order, f = 0: only (3.7) remains, so the step size does not matter."""
    J, lo, hi = 128, (-10.0,), (10.0,)
    x = grid_1d(J, lo[0], hi[0])
    u0 = np.exp(-x * x)
    v0 = 0.5 * x * np.exp(-x * x)
    s = np.full(J, 0.7)
    a = tsfp2_generic(u0, v0, s, 1.3, lo, hi, 5, 0.8, 1)
    b = tsfp2_generic(u0, v0, s, 1.3, lo, hi, 5, 0.01, 80)
    np.testing.assert_allclose(a[0], b[0], atol=1e-12)
    np.testing.assert_allclose(a[1], b[1], atol=1e-12)


def test_seismic_gamma_zero_is_dalembert():
    """(1.1) with gamma = 0 is the acoustic wave equation: u = (u0(x-ct) + u0(x+ct))/2."""
    J, lo, hi = 512, (-20.0,), (20.0,)
    x = grid_1d(J, lo[0], hi[0])
    c0, t, steps = 1.3, 3.0, 30
    u0 = np.exp(-x * x)
    u, v = tsfp2_seismic(u0, np.zeros(J), np.zeros(J), c0, 2.0, lo, hi, 6, t / steps, steps)
    L = hi[0] - lo[0]

    def g(y):
        y = (y - lo[0]) % L + lo[0]
        return np.exp(-y * y)

    def dg(y):
        y = (y - lo[0]) % L + lo[0]
        return -2 * y * np.exp(-y * y)
    np.testing.assert_allclose(u, 0.5 * (g(x - c0 * t) + g(x + c0 * t)), atol=1e-12)
    np.testing.assert_allclose(v, 0.5 * c0 * (-dg(x - c0 * t) + dg(x + c0 * t)), atol=1e-11)


@pytest.mark.parametrize("gamma", [0.02, 0.2, 0.45])
def test_seismic_constant_gamma_modes_match_expm(gamma):
    """Constant gamma: every mode is a damped oscillator; compare with expm of the mode ODE."""
    J, lo, hi = 64, (-4.0,), (6.0,)
    x = grid_1d(J, lo[0], hi[0])
    c0, w0 = 1.4, 3.0
    c = c0 * np.cos(np.pi * gamma / 2)
    eta = -c0 ** (2 * gamma) * w0 ** (-2 * gamma) * np.cos(np.pi * gamma)
    tau = -c0 ** (2 * gamma - 1) * w0 ** (-2 * gamma) * np.sin(np.pi * gamma)
    kap, bet = -c * c * eta, -c * c * tau
    t, steps = 0.9, 9
    u0 = np.zeros(J)
    v0 = np.zeros(J)
    expect_u = np.zeros(J)
    expect_v = np.zeros(J)
    for k, a, b in ((0, 0.3, 0.2), (1, 1.0, 0.5), (5, -0.4, 1.0), (13, 0.7, -0.3)):
        mu = 2 * np.pi * k / (hi[0] - lo[0])
        ph = np.cos(mu * (x - lo[0]))
        u0 += a * ph
        v0 += b * ph
        mu2 = mu * mu
        G = expm(t * np.array([[0.0, 1.0],
                               [-kap * mu2 ** (1 + gamma), -bet * mu2 ** (0.5 + gamma)]]))
        expect_u += (G[0, 0] * a + G[0, 1] * b) * ph
        expect_v += (G[1, 0] * a + G[1, 1] * b) * ph
    u, v = tsfp2_seismic(u0, v0, np.full(J, gamma), c0, w0, lo, hi, 8, t / steps, steps)
    np.testing.assert_allclose(u, expect_u, atol=1e-12)
    np.testing.assert_allclose(v, expect_v, atol=1e-11)


def test_damped_propagator_against_expm_and_semigroup():
    rng = np.random.default_rng(7)
    P1 = np.concatenate([[0.0], rng.uniform(0.01, 50, 20)])
    P2 = np.concatenate([[0.0], rng.uniform(0.01, 50, 20)])
    for kap, bet in ((1.0, 0.0), (0.8, 0.3), (0.5, 4.0)):  # undamped, underdamped, overdamped modes
        for t in (0.05, 0.7):
            g = damped_propagator(P1, P2, kap, bet, t)
            for i in range(P1.size):
                G = expm(t * np.array([[0.0, 1.0], [-kap * P1[i], -bet * P2[i]]]))
                got = np.array([[g[0][i], g[1][i]], [g[2][i], g[3][i]]])
                np.testing.assert_allclose(got, G, rtol=1e-11, atol=1e-13)
        ga = damped_propagator(P1, P2, kap, bet, 0.3)
        gb = damped_propagator(P1, P2, kap, bet, 0.45)
        gab = damped_propagator(P1, P2, kap, bet, 0.75)
        comp = (gb[0] * ga[0] + gb[1] * ga[2], gb[0] * ga[1] + gb[1] * ga[3],
                gb[2] * ga[0] + gb[3] * ga[2], gb[2] * ga[1] + gb[3] * ga[3])
        for a, b in zip(comp, gab):
            np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)


def _mol_reference(u0, v0, A, B, L1, L2, t):
    """High-order ODE integration of u' = v, v' = -A L1 u - B L2 v (dense operators)."""
    n = u0.size

    def rhs(_, y):
        u, v = y[:n], y[n:]
        return np.concatenate([v, -A * (L1 @ u) - B * (L2 @ v)])
    sol = solve_ivp(rhs, (0.0, t), np.concatenate([u0, v0]), method="DOP853",
                    rtol=1e-12, atol=1e-14)
    return sol.y[:n, -1], sol.y[n:, -1]


def test_seismic_variable_gamma_converges_to_method_of_lines():
    """Variable gamma: TSFP2 (reading for (1.1)) converges in dt to the semi-discrete solution.

    The semi-discrete system uses the exact discrete operators (2.7)/(2.12); at
    M = 30 the expansion error is negligible, so what remains is the splitting
    error, which must decrease at an order of at least one.
    """
    J, lo, hi = 32, -8.0, 8.0
    x = grid_1d(J, lo, hi)
    Q = 1.2 + 0.8 * np.sin(np.pi * x / 8.0)
    gamma = gamma_from_Q(Q)
    c0, w0 = 1.1, 2.0
    A, B = seismic_coefficients(gamma, c0, w0)
    L1 = dense_matrix_1d(1.0 + gamma, lo, hi)
    L2 = dense_matrix_1d(0.5 + gamma, lo, hi)
    u0 = np.exp(-x * x)
    v0 = 0.3 * np.exp(-(x - 1) ** 2)
    t = 0.5
    ur, vr = _mol_reference(u0, v0, A, B, L1, L2, t)
    errs = []
    for steps in (50, 100, 200, 400):
        u, v = tsfp2_seismic(u0, v0, gamma, c0, w0, (lo,), (hi,), 30, t / steps, steps)
        errs.append(np.linalg.norm(u - ur) / np.linalg.norm(ur))
    rates = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(r > 0.9 for r in rates), (errs, rates)
    assert errs[-1] < 1e-3


def test_generic_variable_order_converges_second_order_to_method_of_lines():
    """TSFP2 (3.13) for (1.5) with f = u^3 converges at second order in dt (Tables 2-4 claim)."""
    J, lo, hi = 32, -8.0, 8.0
    x = grid_1d(J, lo, hi)
    s = 1.0 + 0.3 * np.sin(np.pi * x / 8.0)
    kap = 0.9
    L = dense_matrix_1d(s, lo, hi)
    u0 = np.exp(-x * x)
    v0 = np.zeros(J)

    def rhs(_, y):
        u, v = y[:J], y[J:]
        return np.concatenate([v, -kap * (L @ u) + u ** 3])
    t = 0.5
    ref = solve_ivp(rhs, (0, t), np.concatenate([u0, v0]), method="DOP853",
                    rtol=1e-12, atol=1e-14).y[:J, -1]
    errs = []
    for steps in (50, 100, 200):
        u, _ = tsfp2_generic(u0, v0, s, kap, (lo,), (hi,), 30, t / steps, steps, f=lambda u: u ** 3)
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    rates = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(1.8 < r < 2.3 for r in rates), (errs, rates)


def test_seismic_reflection_symmetry():
    """Even gamma and even data about the centre stay even (Section 4.1 remark on symmetry)."""
    J, lo, hi = 64, (-8.0,), (8.0,)
    x = grid_1d(J, lo[0], hi[0])
    gamma = 0.1 + 0.08 * np.cos(np.pi * x / 8.0)
    u, v = tsfp2_seismic(np.exp(-x * x), np.zeros(J), gamma, 1.0, 1.0, lo, hi, 10, 0.01, 50)
    idx = (-np.arange(J)) % J
    np.testing.assert_allclose(u, u[idx], atol=1e-13)
    np.testing.assert_allclose(v, v[idx], atol=1e-12)


def test_fourth_order_composition_converges_at_order_four():
    """The composed splitting (three TSFP2 steps w1, w0, w1) for (1.5) with
    f = u^3 converges at fourth order to the semi-discrete solution."""
    from oracle import tsfp4_generic
    J, lo, hi = 32, -8.0, 8.0
    x = grid_1d(J, lo, hi)
    s = 1.0 + 0.3 * np.sin(np.pi * x / 8.0)
    kap = 0.9
    L = dense_matrix_1d(s, lo, hi)
    u0 = np.exp(-x * x)
    v0 = np.zeros(J)

    def rhs(_, y):
        u, v = y[:J], y[J:]
        return np.concatenate([v, -kap * (L @ u) + u ** 3])
    t = 0.5
    ref = solve_ivp(rhs, (0, t), np.concatenate([u0, v0]), method="DOP853",
                    rtol=1e-13, atol=1e-15).y[:J, -1]
    errs = []
    for steps in (10, 20, 40):
        u, _ = tsfp4_generic(u0, v0, s, kap, (lo,), (hi,), 30, t / steps, steps, f=lambda u: u ** 3)
        errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    rates = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(3.7 < r < 4.4 for r in rates), (errs, rates)


def test_fourth_order_composition_constant_order_linear_is_exact():
    """Constant order, f = 0: every sub-step is exact (Remark 3.1), so is the composition."""
    from oracle import tsfp4_generic
    J, lo, hi = 64, (-8.0,), (8.0,)
    x = grid_1d(J, lo[0], hi[0])
    u0, v0 = np.exp(-x * x), 0.2 * np.sin(np.pi * x / 4)
    a, va = tsfp4_generic(u0, v0, np.full(J, 1.2), 1.3, lo, hi, 5, 0.05, 7)
    b, vb = tsfp2_generic(u0, v0, np.full(J, 1.2), 1.3, lo, hi, 5, 0.35, 1)
    np.testing.assert_allclose(a, b, atol=1e-12)
    np.testing.assert_allclose(va, vb, atol=1e-12)
