"""GPU parity: libvofl (through the C ABI) against the FP64 oracle, element by
element, on seeded inputs at sizes the oracle finishes in seconds (several
tiles per axis and ragged tiles included)."""

import numpy as np
import pytest

import oracle as O
from gpu_helpers import as_seen, dev, host, parity_err, require_gpu, say, tol
from workloads import c1_inputs, gaussian_pulse, grf_Q, grid_1d, mesh, paper_s1, rng_for

pytestmark = pytest.mark.gpu


def _plan(shape, lo, hi, precision, **kw):
    require_gpu()
    from paper_2311_13049_amd import vofl as V
    return V.Plan(shape, lo, hi, precision=precision, **kw)


# --------------------------------------------------------------------------
# apply (2.13)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_apply_1d_c1_vs_dense_and_mterm(precision):
    c = c1_inputs()
    say(f"apply 1D n=256 M=8 {precision}")
    p = _plan(c["shape"], c["lo"], c["hi"], precision, gamma=c["gamma"], M=c["M"], dt=c["dt"])
    u = dev(c["u0"], precision)
    u_in = as_seen(c["u0"], precision)
    for op in (1, 2):
        out = host(p.apply(op, u))
        s = O.seismic_op_order(c["gamma"], op)
        ref_m = O.mterm_apply(u_in, s, c["lo"], c["hi"], c["M"])
        ref_d = O.dense_apply(u_in, s, c["lo"], c["hi"])
        assert parity_err(out, ref_m) <= tol(precision), (op, parity_err(out, ref_m))
        assert parity_err(out, ref_d) <= tol(precision) + 1e-13, (op, parity_err(out, ref_d))


CASES_ND = [
    ((32, 128), (-4.0, -6.0), (4.0, 6.0)),         # 2D, several tiles along the last axis
    ((16, 8), (-2.0, -1.0), (2.0, 1.0)),           # 2D, inner < tile width (ragged tile)
    ((64, 128), (-8.0, -8.0), (8.0, 8.0)),         # 2D, larger
    ((16, 8, 32), (-2.0, -1.0, -4.0), (2.0, 1.0, 4.0)),  # 3D mixed sizes
    ((8, 16, 16), (-1.0, -2.0, -2.0), (1.0, 2.0, 2.0)),  # 3D, single-stage axis 0
    ((32, 32, 32), (-4.0,) * 3, (4.0,) * 3),       # 3D cube
    ((48, 96), (-3.0, -6.0), (3.0, 6.0)),          # radix-3 lengths (48 = 3*16, 96 = 3*32)
    ((96, 16, 48), (-6.0, -1.0, -3.0), (6.0, 1.0, 3.0)),  # radix 3 on axes 0 and 2
    ((1000, 16), (-62.5, -1.0), (62.5, 1.0)),      # radix 5 on axis 0 (1000 = 2^3 5^3), h = 1/8
    ((16, 1000), (-1.0, -62.5), (1.0, 62.5)),      # radix 5 on the last axis
    ((8, 1000, 8), (-0.5, -62.5, -0.5), (0.5, 62.5, 0.5)),  # radix 5 on the middle axis
]


def _grf_gamma(shape, lo, hi, seed):
    Q = grf_Q(shape, lo, hi, rng_for(90, seed), corr_len=1.0, qmin=1.0, qmax=30.0)
    return Q, O.gamma_from_Q(Q)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(len(CASES_ND)))
@pytest.mark.parametrize("M", [0, 5, 12])
def test_apply_nd_vs_mterm(case, precision, M):
    shape, lo, hi = CASES_ND[case]
    Q, gamma = _grf_gamma(shape, lo, hi, case)
    rng = rng_for(91, case)
    u0 = gaussian_pulse(shape, lo, hi, [0.3 * (b - a) / 4 for a, b in zip(lo, hi)], width=1.0)
    u0 = u0 + 0.1 * rng.standard_normal(shape)
    say(f"apply {shape} M={M} {precision}")
    p = _plan(shape, lo, hi, precision, Q=Q, M=M, dt=1e-3, max_batch=2)
    u = dev(u0, precision)
    for op in (1, 2):
        out = host(p.apply(op, u))
        ref = O.mterm_apply(as_seen(u0, precision), O.seismic_op_order(gamma, op), lo, hi, M)
        assert parity_err(out, ref) <= tol(precision), (op, parity_err(out, ref))


def test_apply_batch_of_fields_fp64():
    shape, lo, hi = (32, 16, 16), (-4.0, -2.0, -2.0), (4.0, 2.0, 2.0)
    Q, gamma = _grf_gamma(shape, lo, hi, 7)
    rng = rng_for(92, 0)
    U = rng.standard_normal((3,) + shape)
    say("apply batch of 3 fields 3D fp64")
    p = _plan(shape, lo, hi, "fp64", Q=Q, M=6, dt=1e-3, max_batch=3)
    out = host(p.apply(2, dev(U, "fp64"))).reshape(U.shape)
    for f in range(3):
        ref = O.mterm_apply(U[f], O.seismic_op_order(gamma, 2), lo, hi, 6)
        assert parity_err(out[f], ref) <= 1e-12


def test_apply_small_grid_vs_dense():
    shape, lo, hi = (8, 8, 16), (-2.0, -2.0, -3.0), (2.0, 2.0, 3.0)
    Q, gamma = _grf_gamma(shape, lo, hi, 3)
    u0 = gaussian_pulse(shape, lo, hi, (0.2, -0.1, 0.4))
    p = _plan(shape, lo, hi, "fp64", Q=Q, M=24, dt=1e-3)
    out = host(p.apply(1, dev(u0, "fp64")))
    ref = O.dense_apply(u0, O.seismic_op_order(gamma, 1), lo, hi)
    assert parity_err(out, ref) <= 1e-12


def test_apply_constant_order_single_mode_exact():
    """(1.3): constant gamma, one mode -> |mu|^{2s} times the mode, any M."""
    shape, lo, hi = (16, 32), (0.0, 0.0), (2.0, 3.0)
    X, Y = mesh(shape, lo, hi)
    k = (3, 5)
    mu = (2 * np.pi * 3 / 2.0, 2 * np.pi * 5 / 3.0)
    u0 = np.cos(mu[0] * X + mu[1] * Y)
    g = 0.2
    for precision in ("fp64", "fp32"):
        p = _plan(shape, lo, hi, precision, gamma=np.full(shape, g), M=3, dt=1e-3)
        out = host(p.apply(1, dev(u0, precision)))
        expect = (mu[0] ** 2 + mu[1] ** 2) ** (1 + g) * as_seen(u0, precision)
        assert parity_err(out, expect) <= tol(precision), k


# --------------------------------------------------------------------------
# step (3.13) for (1.1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [96, 768, 1000])
def test_apply_and_step_1d_mixed_radix(n):
    # h = 1/8 as in the 1D workload: the operator's amplification of FFT
    # rounding (|mu_max|^{2s}) stays where FP64 parity of 1e-12 is meaningful
    L = n / 16.0
    lo, hi = (-L,), (L,)
    x = grid_1d(n, lo[0], hi[0])
    gamma = 0.1 + 0.08 * np.sin(np.pi * x / L)
    u0 = np.exp(-x * x)
    p = _plan((n,), lo, hi, "fp64", gamma=gamma, M=10, dt=2e-3)
    out = host(p.apply(1, dev(u0, "fp64")))
    assert parity_err(out, O.mterm_apply(u0, 1.0 + gamma, lo, hi, 10)) <= 1e-12
    u, v = dev(u0, "fp64"), dev(np.zeros(n), "fp64")
    p.step(u, v, 20)
    ru, _ = O.tsfp2_seismic(u0, np.zeros(n), gamma, 1.0, 1.0, lo, hi, 10, 2e-3, 20)
    assert parity_err(host(u), ru) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_step_1d_c1(precision):
    c = c1_inputs()
    say(f"step 1D C1 100 steps {precision}")
    p = _plan(c["shape"], c["lo"], c["hi"], precision, gamma=c["gamma"], M=c["M"], dt=c["dt"])
    u, v = dev(c["u0"], precision), dev(c["v0"], precision)
    p.step(u, v, c["steps"])
    assert p.sync_status() == 0
    ru, rv = O.tsfp2_seismic(as_seen(c["u0"], precision), c["v0"], c["gamma"], c["c0"], c["omega0"],
                             c["lo"], c["hi"], c["M"], c["dt"], c["steps"])
    eu, ev = parity_err(host(u), ru), parity_err(host(v), rv)
    say(f"  parity err u {eu:.2e} v {ev:.2e}")
    assert eu <= tol(precision), eu
    assert ev <= tol(precision), ev


STEP_CASES = [
    ((64, 32), (-8.0, -4.0), (8.0, 4.0), 8, 12),
    ((96, 48), (-6.0, -3.0), (6.0, 3.0), 6, 7),
    ((48, 32, 96), (-3.0, -2.0, -6.0), (3.0, 2.0, 6.0), 5, 3),
    ((16, 8), (-2.0, -1.0), (2.0, 1.0), 4, 5),
    ((16, 16, 32), (-2.0, -2.0, -4.0), (2.0, 2.0, 4.0), 6, 6),
    ((8, 32, 8), (-1.0, -4.0, -1.0), (1.0, 4.0, 1.0), 3, 4),
    ((1000, 32), (-62.5, -2.0), (62.5, 2.0), 6, 5),   # radix 5 on axis 0
    ((32, 1000), (-2.0, -62.5), (2.0, 62.5), 6, 5),   # radix 5 on the last axis
    ((8, 1000, 16), (-0.5, -62.5, -1.0), (0.5, 62.5, 1.0), 4, 3),  # radix 5 on the middle axis
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(len(STEP_CASES)))
def test_step_nd_vs_oracle(case, precision):
    shape, lo, hi, M, steps = STEP_CASES[case]
    Q, gamma = _grf_gamma(shape, lo, hi, 20 + case)
    u0 = gaussian_pulse(shape, lo, hi, [0.0] * len(shape))
    v0 = 0.3 * gaussian_pulse(shape, lo, hi, [0.5] * len(shape))
    dt = 2e-3
    say(f"step {shape} M={M} steps={steps} {precision}")
    p = _plan(shape, lo, hi, precision, Q=Q, M=M, dt=dt, c0=1.2, omega0=2.0)
    u, v = dev(u0, precision), dev(v0, precision)
    p.step(u, v, steps)
    assert p.sync_status() == 0
    ru, rv = O.tsfp2_seismic(as_seen(u0, precision), as_seen(v0, precision), gamma, 1.2, 2.0, lo, hi,
                             M, dt, steps)
    eu, ev = parity_err(host(u), ru), parity_err(host(v), rv)
    say(f"  parity err u {eu:.2e} v {ev:.2e}")
    assert eu <= tol(precision), eu
    assert ev <= tol(precision), ev


def test_step_zero_steps_is_identity():
    shape, lo, hi = (16, 16), (-2.0, -2.0), (2.0, 2.0)
    p = _plan(shape, lo, hi, "fp64", gamma=np.full(shape, 0.1), M=2, dt=1e-3)
    u0 = gaussian_pulse(shape, lo, hi, (0, 0))
    u, v = dev(u0, "fp64"), dev(np.zeros(shape), "fp64")
    p.step(u, v, 0)
    assert np.array_equal(host(u), u0)


def test_step_split_calls_equal_one_call():
    """Two calls of k steps equal one call of 2k steps (half steps merge)."""
    shape, lo, hi = (32, 16), (-4.0, -2.0), (4.0, 2.0)
    Q, gamma = _grf_gamma(shape, lo, hi, 31)
    u0 = gaussian_pulse(shape, lo, hi, (0, 0))
    p = _plan(shape, lo, hi, "fp64", Q=Q, M=6, dt=1e-3)
    u1, v1 = dev(u0, "fp64"), dev(np.zeros(shape), "fp64")
    p.step(u1, v1, 10)
    u2, v2 = dev(u0, "fp64"), dev(np.zeros(shape), "fp64")
    p.step(u2, v2, 4)
    p.step(u2, v2, 6)
    assert parity_err(host(u2), host(u1)) <= 1e-13


@pytest.mark.parametrize("ndim", [1, 2])
def test_step_batch_per_solve_coefficients(ndim):
    """batch = 3 solves, each with its own Q: each equals its own oracle run."""
    shape = (128,) if ndim == 1 else (32, 16)
    lo = (-8.0,) * ndim
    hi = (8.0,) * ndim
    Qs, gs, us = [], [], []
    for i in range(3):
        Q, g = _grf_gamma(shape, lo, hi, 40 + i)
        Qs.append(Q)
        gs.append(g)
        us.append(gaussian_pulse(shape, lo, hi, [0.5 * i] * ndim))
    say(f"batched step ndim={ndim}")
    p = _plan(shape, lo, hi, "fp64", Q=np.stack(Qs), M=5, dt=2e-3, batch=3, coef_per_solve=True)
    u, v = dev(np.stack(us), "fp64"), dev(np.zeros((3,) + shape), "fp64")
    p.step(u, v, 7)
    hu = host(u).reshape((3,) + shape)
    for i in range(3):
        ru, _ = O.tsfp2_seismic(us[i], np.zeros(shape), gs[i], 1.0, 1.0, lo, hi, 5, 2e-3, 7)
        assert parity_err(hu[i], ru) <= 1e-12


# --------------------------------------------------------------------------
# generic model (1.5) with f(u) = u^3
# --------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_generic_1d_example_41(precision):
    J, lo, hi = 512, (-32.0,), (32.0,)
    x = grid_1d(J, lo[0], hi[0])
    s = paper_s1(x)
    u0, v0 = np.exp(-x * x), np.zeros(J)
    dt, steps, M = 2.0 ** -9, 64, 15
    say(f"generic 1D J=512 {precision}")
    p = _plan((J,), lo, hi, precision, model="generic", s=s, kappa=1.0, lam=1.0, M=M, dt=dt)
    u, v = dev(u0, precision), dev(v0, precision)
    p.step(u, v, steps)
    ru, rv = O.tsfp2_generic(as_seen(u0, precision), v0, s, 1.0, lo, hi, M, dt, steps, f=lambda w: w ** 3)
    assert parity_err(host(u), ru) <= tol(precision)


@pytest.mark.parametrize("shape", [(32, 64), (16, 16, 16)])
def test_generic_nd(shape):
    lo = (-8.0,) * len(shape)
    hi = (8.0,) * len(shape)
    X = mesh(shape, lo, hi)
    s = 1.0 - 0.4 * np.cos(np.pi * X[0] / 4) * np.cos(np.pi * X[1] / 4)
    u0 = gaussian_pulse(shape, lo, hi, [0.0] * len(shape))
    p = _plan(shape, lo, hi, "fp64", model="generic", s=s, kappa=0.7, lam=0.5, M=10, dt=1e-3)
    u, v = dev(u0, "fp64"), dev(np.zeros(shape), "fp64")
    p.step(u, v, 9)
    ru, _ = O.tsfp2_generic(u0, np.zeros(shape), s, 0.7, lo, hi, 10, 1e-3, 9, f=lambda w: 0.5 * w ** 3)
    assert parity_err(host(u), ru) <= 1e-12


def test_unstable_flag_table4_entry():
    """Table 4: s1 at tau = 2^-7 is unstable; the device flag reports it."""
    from paper_2311_13049_amd import vofl as V
    J, lo, hi = 4096, (-32.0,), (32.0,)
    x = grid_1d(J, lo[0], hi[0])
    p = _plan((J,), lo, hi, "fp64", model="generic", s=paper_s1(x), kappa=1.0, lam=1.0, M=15,
              dt=2.0 ** -7)
    u, v = dev(np.exp(-x * x), "fp64"), dev(np.zeros(J), "fp64")
    p.step(u, v, 128)
    assert p.sync_status() == V.VOFL_ERR_UNSTABLE
    assert p.sync_status() == 0  # flag cleared by the read


# --------------------------------------------------------------------------
# every selectable axis-0 kernel variant (the autotuner may pick any of them)
# --------------------------------------------------------------------------

VARIANT_CASES = [
    ((64, 8, 48), (-4.0, -1.0, -3.0), (4.0, 1.0, 3.0)),   # 3D, 384 columns
    ((128, 8), (-8.0, -1.0), (8.0, 1.0)),                 # 2D, fewer columns than a tile
    ((256, 8, 16), (-16.0, -1.0, -2.0), (16.0, 1.0, 2.0)),  # axis 0 of the 256^3 workload
    ((64, 1000), (-4.0, -62.5), (4.0, 62.5)),             # 1000 columns: a partial last tile group
]


@pytest.mark.parametrize("variant", [0, 2, 5, 6, 11, 12, 13, 14])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(len(VARIANT_CASES)))
def test_axis0_variants_apply_and_step(case, precision, variant):
    import os
    shape, lo, hi = VARIANT_CASES[case]
    Q, gamma = _grf_gamma(shape, lo, hi, 60 + case)
    u0 = gaussian_pulse(shape, lo, hi, [0.3] * len(shape))
    say(f"axis-0 variant {variant} {shape} {precision}")
    os.environ["VOFL_C2R_VARIANT"] = str(variant)
    try:
        p = _plan(shape, lo, hi, precision, Q=Q, M=6, dt=2e-3, max_batch=2)
    finally:
        del os.environ["VOFL_C2R_VARIANT"]
    assert p.info()["c2r_variant"] == variant
    u_in = as_seen(u0, precision)
    out = host(p.apply(1, dev(u0, precision))).reshape(shape)
    ref = O.mterm_apply(u_in, 1.0 + gamma, lo, hi, 6)
    assert parity_err(out, ref) <= tol(precision), parity_err(out, ref)
    u, v = dev(u0, precision), dev(np.zeros(shape), precision)
    p.step(u, v, 4)
    assert p.sync_status() == 0
    ru, rv = O.tsfp2_seismic(u_in, np.zeros(shape), gamma, 1.0, 1.0, lo, hi, 6, 2e-3, 4)
    eu, ev = parity_err(host(u), ru), parity_err(host(v), rv)
    say(f"  parity err u {eu:.2e} v {ev:.2e}")
    assert eu <= tol(precision), eu
    assert ev <= tol(precision), ev


@pytest.mark.parametrize("mid_variant", [0, 1, 2])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mid_variants_apply_and_step(precision, mid_variant):
    """Every middle-axis tile width (the 256-point axis 1 with a ragged last
    axis of 96 columns) against the oracle."""
    import os
    shape, lo, hi = (16, 256, 96), (-2.0, -16.0, -6.0), (2.0, 16.0, 6.0)
    Q, gamma = _grf_gamma(shape, lo, hi, 77)
    u0 = gaussian_pulse(shape, lo, hi, [0.2, -1.0, 0.5])
    say(f"mid variant {mid_variant} {shape} {precision}")
    os.environ["VOFL_MID_VARIANT"] = str(mid_variant)
    try:
        p = _plan(shape, lo, hi, precision, Q=Q, M=4, dt=2e-3, max_batch=2)
    finally:
        del os.environ["VOFL_MID_VARIANT"]
    assert p.info()["mid_variant"] == mid_variant
    u_in = as_seen(u0, precision)
    out = host(p.apply(2, dev(u0, precision))).reshape(shape)
    ref = O.mterm_apply(u_in, 0.5 + gamma, lo, hi, 4)
    assert parity_err(out, ref) <= tol(precision), parity_err(out, ref)
    u, v = dev(u0, precision), dev(np.zeros(shape), precision)
    p.step(u, v, 3)
    assert p.sync_status() == 0
    ru, rv = O.tsfp2_seismic(u_in, np.zeros(shape), gamma, 1.0, 1.0, lo, hi, 4, 2e-3, 3)
    eu, ev = parity_err(host(u), ru), parity_err(host(v), rv)
    say(f"  parity err u {eu:.2e} v {ev:.2e}")
    assert eu <= tol(precision), eu
    assert ev <= tol(precision), ev


@pytest.mark.parametrize("contig_variant", [0, 1])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(8, 16, 256), (16, 512), (8, 1024)])
def test_last_axis_schedules_apply_and_step(shape, precision, contig_variant):
    """Both last-axis radix schedules (4 or 8 elements per thread) the
    autotuner chooses between, against the oracle."""
    import os
    lo = tuple(-0.125 * n for n in shape)
    hi = tuple(0.125 * n for n in shape)
    Q, gamma = _grf_gamma(shape, lo, hi, 88)
    u0 = gaussian_pulse(shape, lo, hi, [0.1] * len(shape))
    say(f"last-axis schedule {contig_variant} {shape} {precision}")
    os.environ["VOFL_CONTIG_VARIANT"] = str(contig_variant)
    try:
        p = _plan(shape, lo, hi, precision, Q=Q, M=5, dt=2e-3, max_batch=2)
    finally:
        del os.environ["VOFL_CONTIG_VARIANT"]
    assert p.info()["contig_variant"] == contig_variant
    u_in = as_seen(u0, precision)
    out = host(p.apply(1, dev(u0, precision))).reshape(shape)
    assert parity_err(out, O.mterm_apply(u_in, 1.0 + gamma, lo, hi, 5)) <= tol(precision)
    u, v = dev(u0, precision), dev(np.zeros(shape), precision)
    p.step(u, v, 3)
    assert p.sync_status() == 0
    ru, rv = O.tsfp2_seismic(u_in, np.zeros(shape), gamma, 1.0, 1.0, lo, hi, 5, 2e-3, 3)
    eu, ev = parity_err(host(u), ru), parity_err(host(v), rv)
    say(f"  parity err u {eu:.2e} v {ev:.2e}")
    assert eu <= tol(precision) and ev <= tol(precision), (eu, ev)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(16, 32, 64), (32, 512), (64, 1000)])
def test_half_row_padding_does_not_change_results(shape, precision):
    """The padded stride of the half spectra's axis-0 rows is a layout choice
    only: plans with the default padding, with none and with a larger one
    give bit-identical applies, TSFP2 steps and leap-frog steps."""
    import os
    lo = tuple(-0.125 * n for n in shape)
    hi = tuple(0.125 * n for n in shape)
    Q, gamma = _grf_gamma(shape, lo, hi, 91)
    u0 = gaussian_pulse(shape, lo, hi, [0.1] * len(shape))
    X = mesh(shape, lo, hi)
    s = 1.0 + 0.2 * np.sin(np.pi * X[0] / 4)
    results, sizes = [], []
    for pad in (None, "0", "24"):
        say(f"half-row padding {pad} {shape} {precision}")
        if pad is not None:
            os.environ["VOFL_HALF_ROW_PAD"] = pad
        try:
            p = _plan(shape, lo, hi, precision, Q=Q, M=5, dt=2e-3, max_batch=2)
            pg = _plan(shape, lo, hi, precision, model="generic", s=s, kappa=1.0, lam=0.5, M=5, dt=2e-3)
        finally:
            os.environ.pop("VOFL_HALF_ROW_PAD", None)
        sizes.append(p.info()["device_bytes"])
        out = host(p.apply(1, dev(u0, precision)))
        u, v = dev(u0, precision), dev(np.zeros(shape), precision)
        p.step(u, v, 3)
        up, uc = pg.lffp_start(dev(u0, precision), dev(np.zeros(shape), precision))
        pg.lffp_step(up, uc, 3)
        assert p.sync_status() == 0 and pg.sync_status() == 0
        results.append((out, host(u), host(v), host(uc), host(up)))
        p.close()
        pg.close()
    assert sizes[1] < sizes[2]  # no pad < a 24-element pad
    for r in results[1:]:
        for a, b in zip(results[0], r):
            assert np.array_equal(a, b)
