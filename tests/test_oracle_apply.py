"""Pins for the oracle's operator evaluations (dense (2.12) and M-term (2.13)).

Every expected value here comes from a closed form or an independent
computation, never from the oracle's own formulas retyped.
"""

import math

import numpy as np
import pytest

from oracle import (dense_apply, dense_dft, dense_matrix_1d, mterm_apply, mterm_apply_at,
                    rel_l2, seismic_op_order)
from workloads import c1_inputs, grid_1d, mesh, paper_s1


def _trig_poly(shape, lo, hi, modes):
    """sum of a_k cos(2 pi k.x'/L + phi), x' = x - lo; returns (u, list of (k, a, phi))."""
    X = mesh(shape, lo, hi)
    u = np.zeros(shape)
    for k, a, phi in modes:
        arg = sum(2 * np.pi * ki * (Xi - li) / (hi_ - li)
                  for ki, Xi, li, hi_ in zip(k, X, lo, hi))
        u += a * np.cos(arg + phi)
    return u, X


def _kabs2(k, lo, hi):
    return sum((2 * np.pi * ki / (b - a)) ** 2 for ki, a, b in zip(k, lo, hi))


@pytest.mark.parametrize("shape", [(32,), (12, 16), (6, 8, 10)])
@pytest.mark.parametrize("s", [0.3, 1.0, 1.7])
def test_constant_order_is_fourier_multiplier(shape, s):
    """(1.3): each mode e^{i mu.x} is scaled by |mu|^{2s}; DC goes to zero."""
    lo = tuple(-3.0 - i for i in range(len(shape)))
    hi = tuple(5.0 + 2 * i for i in range(len(shape)))
    rng = np.random.default_rng(1)
    modes = []
    for _ in range(4):
        k = tuple(int(rng.integers(-n // 2 + 1, n // 2)) for n in shape)
        if all(ki == 0 for ki in k):
            continue
        modes.append((k, rng.uniform(0.5, 2.0), rng.uniform(0, 2 * np.pi)))
    u, X = _trig_poly(shape, lo, hi, modes)
    u = u + 3.0  # DC part must vanish
    expect = np.zeros(shape)
    for k, a, phi in modes:
        arg = sum(2 * np.pi * ki * (Xi - li) / (h_ - li) for ki, Xi, li, h_ in zip(k, X, lo, hi))
        expect += a * _kabs2(k, lo, hi) ** s * np.cos(arg + phi)
    got_dense = dense_apply(u, np.full(shape, s), lo, hi)
    assert np.max(np.abs(got_dense - expect)) <= 1e-11 * np.max(np.abs(expect))
    for M in (0, 3):
        got = mterm_apply(u, np.full(shape, s), lo, hi, M)
        assert np.max(np.abs(got - expect)) <= 1e-11 * np.max(np.abs(expect))


def test_order_one_is_minus_laplacian():
    """s = 1: the operator is -Laplacian; on sin*cos it is an analytic second derivative."""
    shape, lo, hi = (24, 20), (0.0, -1.0), (3.0, 4.0)
    X, Y = mesh(shape, lo, hi)
    a, b = 2 * np.pi * 3 / 3.0, 2 * np.pi * 2 / 5.0
    u = np.sin(a * X) * np.cos(b * (Y + 1.0))
    lap = -(a * a + b * b) * u
    got = dense_apply(u, np.ones(shape), lo, hi)
    np.testing.assert_allclose(got, -lap, atol=1e-11 * np.abs(lap).max())


@pytest.mark.parametrize("k", [1, 5, 16])
def test_single_mode_variable_order_pointwise(k):
    """(2.12) on one real mode gives |mu_k|^{2 s(x_j)} cos(mu_k (x_j - a)) at every point."""
    n, lo, hi = 48, (-8.0,), (8.0,)
    x = grid_1d(n, lo[0], hi[0])
    s = 0.6 + 0.5 * np.sin(np.pi * x / 8.0) ** 2
    mu = 2 * np.pi * k / 16.0
    u = np.cos(mu * (x - lo[0]))
    got = dense_apply(u, s, lo, hi)
    expect = np.abs(mu) ** (2 * s) * u
    np.testing.assert_allclose(got, expect, atol=1e-11 * np.abs(expect).max())


@pytest.mark.parametrize("M", [0, 1, 2, 4, 8])
def test_single_mode_mterm_is_truncated_exponential(M):
    """(2.13) on one mode: |mu|^{2 s0} sum_{m<=M} z^m/m! with z = delta ln|mu|^2.

    The error against the exact pointwise symbol obeys the Taylor remainder
    bound |mu|^{2 s0} |z|^{M+1} e^{|z|}/(M+1)!, and for z > 0 the truncated
    series equals e^z Q(M+1, z) (regularised upper incomplete gamma).
    """
    from scipy.special import gammaincc
    n, lo, hi = 64, (-8.0,), (8.0,)
    x = grid_1d(n, lo[0], hi[0])
    s = 1.0 + 0.3 * np.sin(np.pi * x / 8.0)
    k = 7
    mu = 2 * np.pi * k / 16.0
    u = np.cos(mu * (x - lo[0]))
    got = mterm_apply(u, s, lo, hi, M)
    s0 = s.mean()
    z = (s - s0) * np.log(mu * mu)
    exact = np.abs(mu) ** (2 * s) * u
    bound = np.abs(mu) ** (2 * s0) * np.abs(z) ** (M + 1) * np.exp(np.abs(z)) / math.factorial(M + 1)
    assert np.all(np.abs(got - exact) <= bound * np.abs(u) + 1e-12 * np.abs(exact).max())
    pos = z > 1e-3
    series = np.exp(z[pos]) * gammaincc(M + 1, z[pos])
    np.testing.assert_allclose(got[pos], np.abs(mu) ** (2 * s0) * series * u[pos],
                               atol=1e-11 * np.abs(exact).max())


def test_mterm_converges_to_dense_as_M_grows():
    """Section 4.2 (Figure 5a statement): the truncation error decays quickly with M."""
    n, lo, hi = 128, (-32.0,), (32.0,)
    x = grid_1d(n, lo[0], hi[0])
    s = paper_s1(x)
    u = np.exp(-x * x)
    ref = dense_apply(u, s, lo, hi)
    errs = [rel_l2(mterm_apply(u, s, lo, hi, M), ref) for M in (0, 2, 4, 8, 16, 30)]
    assert all(b < a for a, b in zip(errs, errs[1:5]))
    assert errs[-1] < 1e-12


def test_matrix_form_1d_and_closed_form_reading():
    """(2.7): the dense matrix times u equals (2.12); the closed form of (2.7),
    read as (1/J)[(-1)^{j-l}|mu_{J/2}|^{2 s_j} + 2 sum_{k=1}^{J/2-1} |mu_k|^{2 s_j}
    cos(mu_k (x_j - x_l))], equals the sum form."""
    n, lo, hi = 40, -5.0, 5.0
    x = grid_1d(n, lo, hi)
    s = 0.8 + 0.4 * np.cos(2 * np.pi * x / 10.0)
    A = dense_matrix_1d(s, lo, hi)
    u = np.exp(-x * x) * (1 + 0.3 * x)
    np.testing.assert_allclose(A @ u, dense_apply(u, s, (lo,), (hi,)), atol=1e-11 * np.abs(A @ u).max())
    j = np.arange(n)
    d = j[:, None] - j[None, :]
    muN = np.pi * n / (hi - lo)
    closed = ((-1.0) ** d) * muN ** (2 * s)[:, None]
    for k in range(1, n // 2):
        mk = 2 * np.pi * k / (hi - lo)
        closed = closed + 2 * (mk ** (2 * s))[:, None] * np.cos(mk * (x[:, None] - x[None, :]))
    closed /= n
    np.testing.assert_allclose(A, closed, atol=1e-10 * np.abs(A).max())


def test_dense_dft_matches_library_fft():
    rng = np.random.default_rng(3)
    u = rng.standard_normal((6, 10, 4))
    np.testing.assert_allclose(dense_dft(u), np.fft.fftn(u) / u.size, atol=1e-14)


def test_c1_single_apply_mterm_vs_dense():
    """1D workload n=256, M=8: the truncation is far below 1e-12 for both orders."""
    c = c1_inputs()
    for op in (1, 2):
        s = seismic_op_order(c["gamma"], op)
        ref = dense_apply(c["u0"], s, c["lo"], c["hi"])
        got = mterm_apply(c["u0"], s, c["lo"], c["hi"], c["M"])
        assert rel_l2(got, ref) < 1e-12


def test_reflection_symmetry_of_operator():
    """Even u and even s (about the box centre) give an even result (Section 4.1, Figure 4 remarks)."""
    n, lo, hi = 64, (-8.0,), (8.0,)
    x = grid_1d(n, lo[0], hi[0])
    s = 1.0 + 0.3 * np.cos(np.pi * x / 8.0)
    u = np.exp(-x * x)
    out = mterm_apply(u, s, lo, hi, 12)
    # x_j -> -x_j maps index j to (n - j) mod n on this grid
    np.testing.assert_allclose(out, out[(-np.arange(n)) % n], atol=1e-12 * np.abs(out).max())


def test_pointwise_evaluation_matches_full_field_and_single_mode():
    """mterm_apply_at (used to sample huge grids) agrees with mterm_apply and,
    on one mode, with the truncated exponential series at those points."""
    shape, lo, hi = (8, 12, 10), (-1.0, -2.0, -1.5), (1.0, 2.0, 1.5)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(shape)
    s = 1.0 + 0.2 * rng.random(shape)
    full = mterm_apply(u, s, lo, hi, 7)
    pts = [(0, 0, 0), (3, 5, 7), (7, 11, 9)]
    got = mterm_apply_at(u, s, lo, hi, 7, pts)
    np.testing.assert_allclose(got, [full[p] for p in pts], atol=1e-12 * np.abs(full).max())
    X = mesh(shape, lo, hi)
    mu = (2 * np.pi * 2 / 2.0, 2 * np.pi * 3 / 4.0, 0.0)
    mode = np.cos(mu[0] * (X[0] - lo[0]) + mu[1] * (X[1] - lo[1]))
    vals = mterm_apply_at(mode, s, lo, hi, 3, pts)
    s0 = s.mean()
    m2 = mu[0] ** 2 + mu[1] ** 2
    for v, p in zip(vals, pts):
        z = (s[p] - s0) * np.log(m2)
        series = sum(z ** m / math.factorial(m) for m in range(4))
        assert abs(v - m2 ** s0 * series * mode[p]) <= 1e-12 * m2 ** 2
