"""Pins for the oracle's leap-frog scheme LFFP (3.4) for (1.5).

Expected values come from the paper's Table 3 (tests/golden/) and from the
closed-form solution of the leap-frog recurrence on one Fourier mode.
"""

import json
import math
import os

import numpy as np
import pytest

from oracle import lffp_generic, weighted_l2
from workloads import grid_1d, paper_s1

GOLD = os.path.join(os.path.dirname(__file__), "golden")
LO, HI = (-32.0,), (32.0,)


def _ex1(J, s_fn, dt, steps, M=15):
    """Problem (4.1) with LFFP: kappa = 1, f(u) = u^3, [-32, 32], u0 = exp(-x^2), v0 = 0."""
    x = grid_1d(J, LO[0], HI[0])
    s = s_fn(x) if callable(s_fn) else np.full(J, float(s_fn))
    return lffp_generic(np.exp(-x * x), np.zeros(J), s, 1.0, LO, HI, M, dt, steps,
                        f=lambda u: u ** 3)[1]


@pytest.mark.parametrize("kappa,s,k", [(1.0, 1.0, 3), (2.5, 0.6, 7), (0.7, 1.4, 1)])
def test_single_mode_follows_the_chebyshev_recurrence(kappa, s, k):
    """f = 0, constant order, u^0 = cos(mu x), psi = 0: the scheme is
    u^{n+1} = 2 c u^n - u^{n-1} with c = 1 - tau^2 w^2 / 2, w^2 = kappa |mu|^{2s},
    and (3.4c) gives u^1 = c u^0, so u^n = cos(n theta) u^0 with cos(theta) = c."""
    n, lo, hi = 64, (-4.0,), (4.0,)
    x = grid_1d(n, lo[0], hi[0])
    mu = 2 * np.pi * k / (hi[0] - lo[0])
    u0 = np.cos(mu * (x - lo[0]))
    dt, steps = 1e-3, 37
    w2 = kappa * mu ** (2 * s)
    theta = math.acos(1 - 0.5 * dt * dt * w2)
    prev, cur = lffp_generic(u0, np.zeros(n), np.full(n, s), kappa, lo, hi, 6, dt, steps)
    np.testing.assert_allclose(cur, math.cos(steps * theta) * u0, atol=1e-12)
    np.testing.assert_allclose(prev, math.cos((steps - 1) * theta) * u0, atol=1e-12)


def test_single_mode_velocity_start():
    """u^0 = 0, psi = cos(mu x): u^1 = tau psi and u^n = tau sin(n theta)/sin(theta) psi."""
    n, lo, hi = 32, (0.0,), (2 * np.pi,)
    x = grid_1d(n, lo[0], hi[0])
    k, s, kappa, dt, steps = 2, 0.8, 1.3, 2e-3, 50
    psi = np.cos(k * x)
    theta = math.acos(1 - 0.5 * dt * dt * kappa * k ** (2 * s))
    _, cur = lffp_generic(np.zeros(n), psi, np.full(n, s), kappa, lo, hi, 3, dt, steps)
    np.testing.assert_allclose(cur, dt * math.sin(steps * theta) / math.sin(theta) * psi, atol=1e-13)


def test_zero_and_one_step():
    x = grid_1d(16, -1.0, 1.0)
    phi, psi = np.exp(-x * x), np.sin(np.pi * x)
    prev, cur = lffp_generic(phi, psi, np.full(16, 1.0), 1.0, (-1.0,), (1.0,), 2, 1e-2, 0)
    assert np.array_equal(prev, phi) and np.array_equal(cur, phi)
    prev, cur = lffp_generic(phi, psi, np.full(16, 1.0), 1.0, (-1.0,), (1.0,), 2, 1e-2, 1)
    assert np.array_equal(prev, phi)
    # s = 1: the operator is -Laplacian, u^1 = phi + tau psi + tau^2/2 phi''
    k = np.fft.fftfreq(16, d=2.0 / 16) * 2 * np.pi
    lap = np.real(np.fft.ifft(-(k ** 2) * np.fft.fft(phi)))
    np.testing.assert_allclose(cur, phi + 1e-2 * psi + 0.5e-4 * lap, atol=1e-13)


@pytest.fixture(scope="module")
def references():
    """Reference solutions of Table 3: LFFP with h = 1/64, tau = 1e-4, t = 1."""
    return {"s=1": _ex1(4096, 1.0, 1e-4, 10000), "s1": _ex1(4096, paper_s1, 1e-4, 10000)}


@pytest.mark.slow
def test_table3_temporal_errors(references):
    """Table 3: LFFP temporal errors at t = 1, h = 1/64, to the printed digits."""
    tab = json.load(open(os.path.join(GOLD, "table3_lffp_temporal.json")))
    cols = tab["columns"]
    for col, s_fn in (("s=1", 1.0), ("s1", paper_s1)):
        for key in ("9", "10", "11"):
            k = int(key)
            printed = float(tab["rows"][key][cols.index(col)])
            u = _ex1(4096, s_fn, 2.0 ** -k, 2 ** k)
            err = weighted_l2(u - references[col], 1.0 / 64)
            assert abs(err - printed) <= 6e-4 * printed, (col, key, err, printed)


@pytest.mark.slow
def test_table3_unstable_entries():
    """Table 3: 'unstable' for s1 at tau = 2^-7 and 2^-8."""
    for k in (7, 8):
        u = _ex1(4096, paper_s1, 2.0 ** -k, 2 ** k)
        assert (not np.all(np.isfinite(u))) or np.max(np.abs(u)) > 1e3
