"""Physics pin of the oracle's coefficient map for (1.1): Q -> gamma -> A, B.

The model of Section 1 (the coefficient formulas below (1.1)) says that c0
is the phase velocity at the reference frequency omega0 and that Q is the
quality factor, with gamma = arctan(1/Q)/pi. For a constant gamma every
Fourier mode of (1.1) is a damped oscillator u'' + b2 u' + a2 u = 0 with
eigenvalues -b +- i w. At the wavenumber |mu| = omega0/c0 the mode's phase
velocity w/|mu| must equal c0, and its quality factor w/(2b) must equal Q,
both up to O(1/Q^2) (the constant-Q model is exact at the reference
frequency to first order in 1/Q).

The test measures w and b from the oracle's own time stepper (exact in time
for constant gamma), through its propagator matrix for one mode, so it pins
gamma_from_Q, seismic_coefficients and the exact sub-step together. A wrong
exponent of c0 or omega0 in the coefficients, a factor 2 in gamma, or a
wrong trigonometric factor moves one of the two ratios by far more than
1/Q^2.
"""

import numpy as np
import pytest

from oracle import gamma_from_Q, tsfp2_seismic


def _mode_eigenvalues(gamma, c0, omega0, t):
    """Eigenvalues of the oracle's one-mode propagator over time t, as rates."""
    J, m = 32, 3
    L = 2.0 * np.pi * m * c0 / omega0            # bin m sits at |mu| = omega0 / c0
    lo, hi = (-0.25 * L,), (0.75 * L,)
    x = lo[0] + L * np.arange(J) / J
    mode = np.cos(2.0 * np.pi * m * (x - lo[0]) / L)
    G = np.zeros((2, 2))
    for col, (u0, v0) in enumerate(((mode, 0 * mode), (0 * mode, mode))):
        u, v = tsfp2_seismic(u0, v0, np.full(J, gamma), c0, omega0, lo, hi, 6, t, 1)
        G[0, col] = 2.0 / J * np.dot(u, mode)
        G[1, col] = 2.0 / J * np.dot(v, mode)
    lam = np.log(np.linalg.eigvals(G).astype(complex)) / t
    return lam, omega0 / c0


@pytest.mark.parametrize("Q", [10.0, 100.0])
@pytest.mark.parametrize("c0,omega0", [(1.0, 1.0), (1.4, 3.0), (0.6, 0.5)])
def test_constant_Q_phase_velocity_and_quality_factor(Q, c0, omega0):
    gamma = float(gamma_from_Q(Q))
    t = 0.5 / omega0                                    # w t < pi: the log is on its main branch
    lam, k = _mode_eigenvalues(gamma, c0, omega0, t)
    lam = lam[np.argmax(lam.imag)]
    w, b = lam.imag, -lam.real
    v_phase = w / k
    Q_eff = w / (2.0 * b)
    assert abs(v_phase / c0 - 1.0) <= 1.0 / Q ** 2, (v_phase, c0)
    assert abs(Q_eff / Q - 1.0) <= 1.0 / Q ** 2, (Q_eff, Q)


def test_infinite_Q_is_lossless_at_c0():
    """Q = inf: gamma = 0, no damping, phase velocity c0 at every wavenumber."""
    c0, omega0 = 1.7, 2.0
    gamma = float(gamma_from_Q(np.inf))
    assert gamma == 0.0
    lam, k = _mode_eigenvalues(gamma, c0, omega0, 0.4 / omega0)
    assert np.max(np.abs(lam.real)) <= 1e-12
    assert abs(np.max(lam.imag) / k / c0 - 1.0) <= 1e-12
