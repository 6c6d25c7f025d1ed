"""Seeded input recipes for the workloads of the benchmark and the tests.

Every array is float64, C-ordered (last index fastest), sampled at the grid
points x_j = lo + j*h, j = 0..n-1, of a periodic box [lo, hi) per axis
(Section 2, the grid below eq. (2.1); Section 2.3 for d > 1).

Recipes (all seeds are explicit):

* ``c1``     1D n=256 on [-16,16): gamma(x) = 0.1 + 0.05 sin(pi x/16),
             u0 = exp(-x^2), v0 = 0.
* ``grf_Q``  Gaussian random field: white noise, smoothed by the spectral
             filter exp(-|k|^2 l^2/4) (covariance exp(-r^2/(2 l^2))),
             min-max mapped onto [qmin, qmax].
* ``two_layer_Q``  Q(z) = 60 - 40 tanh(z/w) tanh((L/2-|z|)/w) along the first
             axis (about 20 for z>0 and 100 for z<0, smooth at 0 and at the
             periodic wrap), times (1 + 0.05 U(-1,1)) per point.
* ``gaussian_pulse``  exp(-|x - xs|^2) with periodic minimum-image distance.
* paper test functions of Section 4.1: s1, s2 and the initial data of (4.1).
* ``ex3``    Example 3 of Section 4 (two-layer attenuating medium) on the
             periodic box [0,2)^2: gamma = a1 + a2 tanh(100 (y - 1)), phase
             velocity 11/18 for y > 1 and 1 for y <= 1, Ricker initial
             displacement (4.3) with nu0 = 25 centred at (1, 0.85), zero
             initial velocity, dt = 1e-4. The paper's mesh h = 0.002 gives
             n = 1000 per axis; omega0 = 1 and M = 8 are not given there.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "BASE_SEED", "rng_for", "grid_1d", "mesh", "gaussian_pulse", "grf_Q",
    "two_layer_Q", "c1_inputs", "c2_inputs", "c3_inputs", "c4_inputs",
    "c5_requests", "c5_request_inputs", "paper_s1", "paper_s2", "paper_ex1_initial",
    "ricker", "ex3_inputs", "probe_field",
]

BASE_SEED = 13049


def rng_for(config_id: int, *spawn_key: int) -> np.random.Generator:
    """Generator for a config (and optionally a shot/request index)."""
    ss = np.random.SeedSequence(BASE_SEED + int(config_id), spawn_key=tuple(int(k) for k in spawn_key))
    return np.random.default_rng(ss)


def grid_1d(n: int, lo: float, hi: float) -> np.ndarray:
    """Sample points lo + j*(hi-lo)/n, j = 0..n-1."""
    return lo + (hi - lo) * np.arange(n, dtype=np.float64) / n


def mesh(shape, lo, hi):
    """Coordinate arrays (indexing='ij') for a box given per axis."""
    axes = [grid_1d(n, a, b) for n, a, b in zip(shape, lo, hi)]
    return np.meshgrid(*axes, indexing="ij")


def gaussian_pulse(shape, lo, hi, center, width: float = 1.0) -> np.ndarray:
    """exp(-|x - xs|^2 / width^2) with periodic minimum-image distance."""
    X = mesh(shape, lo, hi)
    r2 = np.zeros(tuple(shape))
    for Xi, a, b, c in zip(X, lo, hi, center):
        L = b - a
        d = Xi - c
        d = d - L * np.round(d / L)
        r2 = r2 + d * d
    return np.exp(-r2 / (width * width))


def grf_Q(shape, lo, hi, rng: np.random.Generator, corr_len: float = 4.0,
          qmin: float = 10.0, qmax: float = 200.0) -> np.ndarray:
    """Quality-factor field from a smoothed Gaussian random field."""
    shape = tuple(int(n) for n in shape)
    noise = rng.standard_normal(shape)
    spec = np.fft.fftn(noise)
    k2 = np.zeros(shape)
    for ax, (n, a, b) in enumerate(zip(shape, lo, hi)):
        kk = 2.0 * np.pi * np.fft.fftfreq(n, d=(b - a) / n)
        sh = [1] * len(shape)
        sh[ax] = n
        k2 = k2 + (kk ** 2).reshape(sh)
    field = np.fft.ifftn(spec * np.exp(-k2 * corr_len ** 2 / 4.0)).real
    fmin, fmax = field.min(), field.max()
    unit = (field - fmin) / (fmax - fmin)
    return qmin + (qmax - qmin) * unit


def two_layer_Q(shape, lo, hi, rng: np.random.Generator, width: float = 1.0,
                noise: float = 0.05) -> np.ndarray:
    """Two-layer Q along the first axis (Q~20 above 0, Q~100 below), with noise."""
    shape = tuple(int(n) for n in shape)
    L = hi[0] - lo[0]
    z = mesh(shape, lo, hi)[0]
    q = 60.0 - 40.0 * np.tanh(z / width) * np.tanh((L / 2.0 - np.abs(z)) / width)
    return q * (1.0 + noise * rng.uniform(-1.0, 1.0, size=shape))


def c1_inputs(n: int = 256):
    """1D workload: gamma given directly, Gaussian displacement, zero velocity."""
    lo, hi = (-16.0,), (16.0,)
    x = grid_1d(n, lo[0], hi[0])
    gamma = 0.1 + 0.05 * np.sin(np.pi * x / 16.0)
    u0 = np.exp(-x * x)
    v0 = np.zeros(n)
    return dict(shape=(n,), lo=lo, hi=hi, gamma=gamma, u0=u0, v0=v0,
                c0=1.0, omega0=1.0, M=8, dt=1e-3, steps=100)


def c2_inputs(n: int = 1024, seed_offset: int = 0):
    """2D workload: GRF Q in [10,200], Gaussian pulse at the centre."""
    lo, hi = (-32.0, -32.0), (32.0, 32.0)
    rng = rng_for(2, seed_offset)
    Q = grf_Q((n, n), lo, hi, rng, corr_len=4.0)
    u0 = gaussian_pulse((n, n), lo, hi, (0.0, 0.0))
    return dict(shape=(n, n), lo=lo, hi=hi, Q=Q, u0=u0, v0=np.zeros_like(u0),
                c0=1.0, omega0=1.0, M=16, dt=5e-4, steps=1000)


def c3_inputs(n: int = 256, seed_offset: int = 0):
    """3D workload: two-layer Q with 5% noise, Gaussian pulse at the centre."""
    lo, hi = (-16.0,) * 3, (16.0,) * 3
    rng = rng_for(3, seed_offset)
    Q = two_layer_Q((n, n, n), lo, hi, rng)
    u0 = gaussian_pulse((n, n, n), lo, hi, (0.0, 0.0, 0.0))
    return dict(shape=(n, n, n), lo=lo, hi=hi, Q=Q, u0=u0, v0=np.zeros_like(u0),
                c0=1.0, omega0=1.0, M=16, dt=1e-3, steps=500)


def c4_inputs(n_small: int = 512, n_large: int = 768, shots_small: int = 64,
              shots_large: int = 16):
    """Batched shots: shared-Q group plus a group with one Q per shot."""
    lo, hi = (-32.0, -32.0), (32.0, 32.0)
    rng = rng_for(4, 0)
    Q_shared = grf_Q((n_small, n_small), lo, hi, rng)
    shots = []
    for i in range(shots_small):
        r = rng_for(4, 1, i)
        xs = r.uniform(lo[0], hi[0], size=2)
        shots.append(dict(shape=(n_small, n_small), Q=Q_shared,
                          u0=gaussian_pulse((n_small, n_small), lo, hi, xs)))
    for i in range(shots_large):
        r = rng_for(4, 2, i)
        Q = grf_Q((n_large, n_large), lo, hi, r)
        xs = r.uniform(lo[0], hi[0], size=2)
        shots.append(dict(shape=(n_large, n_large), Q=Q,
                          u0=gaussian_pulse((n_large, n_large), lo, hi, xs)))
    return dict(lo=lo, hi=hi, shots=shots, c0=1.0, omega0=1.0, M=12, dt=5e-4, steps=200)


def c5_requests(count: int = 200, rate: float = 200.0, grids=None, seed_offset: int = 0):
    """Poisson request stream: arrival time, grid, M, steps, precision, seed."""
    if grids is None:
        grids = [(128, 128), (256, 256), (512, 512), (1024, 1024), (128, 128, 128), (256, 256, 256)]
    rng = rng_for(5, seed_offset)
    t = 0.0
    reqs = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        g = grids[int(rng.integers(len(grids)))]
        reqs.append(dict(index=i, arrival=t, shape=tuple(g),
                         M=int(rng.choice([8, 16])),
                         steps=int(rng.integers(100, 2001)),
                         precision=("fp32" if rng.random() < 0.5 else "fp64"),
                         seed=int(rng.integers(1 << 31))))
    return reqs


def c5_request_inputs(req):
    """Box, time step, Q field and initial data of one request of the stream.

    2D grids live on [-32,32)^2 with dt = 5e-4, 3D grids on [-16,16)^3 with
    dt = 1e-3; Q is a Gaussian random field (correlation length 4, Q in
    [10, 200]); u0 is a unit Gaussian pulse at a uniform random centre, v0 = 0.
    """
    shape = tuple(int(n) for n in req["shape"])
    d = len(shape)
    half = 32.0 if d == 2 else 16.0
    lo, hi = (-half,) * d, (half,) * d
    rng = rng_for(5, 1, int(req["seed"]))
    Q = grf_Q(shape, lo, hi, rng, corr_len=4.0)
    xs = rng.uniform(-half, half, size=d)
    u0 = gaussian_pulse(shape, lo, hi, xs)
    return dict(shape=shape, lo=lo, hi=hi, dt=(5e-4 if d == 2 else 1e-3), Q=Q, u0=u0,
                v0=np.zeros_like(u0), c0=1.0, omega0=1.0)


def paper_s1(x):
    """s1(x) = 1 + 0.3 sin(pi x / 8) (Tables 2-5, Section 4.1)."""
    return 1.0 + 0.3 * np.sin(np.pi * x / 8.0)


def paper_s2(x):
    """s2(x) = 1 + 0.2 tanh(cos(pi x / 8)) (Tables 2-5, Section 4.1)."""
    return 1.0 + 0.2 * np.tanh(np.cos(np.pi * x / 8.0))


def paper_ex1_initial(x):
    """Initial data of problem (4.1): u(x,0) = exp(-x^2), u_t(x,0) = 0."""
    return np.exp(-x * x), np.zeros_like(x)


def ricker(shape, lo, hi, center, nu0: float) -> np.ndarray:
    """(1 - 2 pi^2 nu0^2 r^2) exp(-pi^2 nu0^2 r^2), r = |x - xc| (initial data (4.3))."""
    X = mesh(shape, lo, hi)
    r2 = np.zeros(tuple(shape))
    for Xi, c in zip(X, center):
        r2 = r2 + (Xi - c) ** 2
    a = (np.pi * nu0) ** 2 * r2
    return (1.0 - 2.0 * a) * np.exp(-a)


def ex3_inputs(n: int = 1000, case: int = 0):
    """Example 3 (Section 4): case 0 has (a1, a2) = (0.0065, 0.0035), case 1
    (0.02, 0.01); y is the last axis."""
    a1, a2 = ((0.0065, 0.0035), (0.02, 0.01))[case]
    shape, lo, hi = (n, n), (0.0, 0.0), (2.0, 2.0)
    _, Y = mesh(shape, lo, hi)
    gamma = a1 + a2 * np.tanh(100.0 * (Y - 1.0))
    c0 = np.where(Y > 1.0, 11.0 / 18.0, 1.0)
    phi = ricker(shape, lo, hi, (1.0, 0.85), 25.0)
    return dict(shape=shape, lo=lo, hi=hi, gamma=gamma, c0=c0, omega0=1.0, M=8, dt=1e-4,
                phi=phi, psi=np.zeros(shape), a1=a1, a2=a2)


def probe_field(shape, index: int) -> np.ndarray:
    """Seeded standard-normal field number ``index``: test vectors onto which
    stored results are projected (the projections of an error field estimate
    its L2 norm; nothing of the method is computed here)."""
    return rng_for(90, int(index)).standard_normal(tuple(int(n) for n in shape))
