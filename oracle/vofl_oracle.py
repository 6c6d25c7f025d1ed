"""Plain, slow FP64 reference for the matrix-free variable-order fractional
Laplacian and the second-order time-splitting Fourier pseudospectral solver
of Zhang, Zhao and Zhou, "Fourier pseudospectral methods for the
variable-order space fractional wave equations" (arXiv 2311.13049).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the product package.

Conventions (fixed by the paper, with the readings noted where it is silent):

* Grid: n_i points per axis (even), h_i = L_i/n_i, x_j = a + j h (Section 2,
  below (2.1); Section 2.3). Arrays are C-ordered, last axis fastest.
* Wavenumbers: k_i in [-n_i/2, n_i/2 - 1], mu = 2 pi k / L (eq. (2.2)); the
  symbol uses |mu|^2 = sum_i mu_i^2 (eq. (2.12)). The symbol is written in the
  angular convention |mu|^{2s}: eq. (1.2) prints exp(2 pi i x.xi) with
  |xi|^{2s}, which disagrees with the discrete (2.3); the discrete form is
  taken. The Nyquist index -n/2 is part of the sum, once.
* u_hat_k = (1/N) sum_j u_j exp(-i mu_k.(x_j - a)) (eqs. (2.2), (2.11)); the
  phase is a sum over axes (the product printed below (2.11) is read as the
  dot product it stands for).
* s0 is the grid mean of s (the integral mean of Section 2.2, rectangle rule).
* M is the upper index of the expansion: terms m = 0..M (eq. (2.13)).
* k = 0 is excluded from every sum with a power of |mu| (eq. (2.9) note).

Functions and what pins each one (tests/test_oracle_*.py):

  dense_apply         exact discrete operator (2.12) by explicit O(N^2) sums.
                      Pinned: trig polynomials under constant order (closed
                      form (1.3)); single Fourier mode under variable order
                      (pointwise |mu|^{2 s(x)} e^{i mu x}); s = 1 gives the
                      analytic second derivative; matrix form (2.7) in 1D.
  mterm_apply         M-term matrix-free scheme (2.10)/(2.13). Pinned: equals
                      dense_apply for constant order at every M; single mode
                      gives the truncated exponential series (remainder bound);
                      converges to dense_apply as M grows.
  tsfp2_generic       TSFP2 (3.13)-(3.14) for model (1.5). Pinned: Tables 4
                      and 5 of the paper reproduced to the printed digits
                      (including the 'unstable' entries); constant-order
                      linear case exact in time (Remark 3.1).
  damped_propagator   exact solution of the constant-coefficient part of the
                      split seismic model. Pinned: matrix exponential of the
                      mode ODE; semigroup property.
  lffp_seismic        leap-frog (3.4) for (1.1) (reading: backward difference
                      in the damping term, Taylor start). Pinned: gamma = 0 is
                      the classical leap-frog (closed-form cos(n theta) per
                      mode); constant gamma follows the closed-form roots of
                      the per-mode two-term recurrence; variable gamma and a
                      layered c0 converge at first order to a high-order ODE
                      integration of the semi-discrete system.
  tsfp2_seismic       TSFP2 extended to the viscoacoustic model (1.1) (reading
                      below). Pinned: gamma = 0 reduces to d'Alembert's
                      solution of the acoustic wave equation; constant gamma
                      reduces to per-mode damped oscillators (matrix
                      exponential); variable gamma converges in dt to a
                      high-order ODE integration of the semi-discrete system
                      built from dense_apply; reflection symmetry.

Reading used for (1.1) (the paper applies TSFP2 only to (1.5)): with
v = u_t, (1.1) becomes u_t = v, v_t = -A(x) L1 u - B(x) L2 v where
L1 = (-Lap)^{1+gamma(x)}, L2 = (-Lap)^{1/2+gamma(x)}, A = -c^2 eta and
B = -c^2 tau (coefficients of (1.1)). The exactly solved part uses the
constant orders 1+gbar, 1/2+gbar and coefficients kappa0 = A(gbar),
beta0 = B(gbar) (gbar = grid mean of gamma); the kick holds u and v at their
half-step values and adds dt times the remainder. With A = kappa, B = 0 this
is exactly the paper's scheme (3.13), whose kick sign follows (3.8) and
whose tilde operator is the m >= 1 part of (2.13).
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "fft_bins", "wavenumbers", "mu_squared", "gamma_from_Q",
    "seismic_coefficients", "dense_dft", "dense_apply", "dense_matrix_1d",
    "mterm_apply", "seismic_op_order", "tsfp2_generic", "tsfp4_generic", "lffp_generic", "cnfp_generic",
    "damped_propagator", "lffp_seismic",
    "tsfp2_seismic", "weighted_l2", "rel_l2", "mterm_apply_at", "set_fft_workers",
]

# FFT backend: numpy's pocketfft by default; set_fft_workers(n) switches to
# scipy.fft with n threads (same transform, a library primitive either way).
_FFT_WORKERS = 0


def set_fft_workers(n: int) -> None:
    """Use scipy.fft with n worker threads for the oracle's FFTs (0: numpy)."""
    global _FFT_WORKERS
    _FFT_WORKERS = int(n)


def _fftn(x):
    if _FFT_WORKERS:
        import scipy.fft
        return scipy.fft.fftn(x, workers=_FFT_WORKERS)
    return np.fft.fftn(x)


def _ifftn(x):
    if _FFT_WORKERS:
        import scipy.fft
        return scipy.fft.ifftn(x, workers=_FFT_WORKERS)
    return np.fft.ifftn(x)


# ---------------------------------------------------------------------------
# Grid and symbol (Section 2, eqs. (2.2), (2.11)-(2.12))
# ---------------------------------------------------------------------------

def fft_bins(n: int) -> np.ndarray:
    """Integer wavenumbers k in [-n/2, n/2-1], stored at index k mod n (eq. (2.2))."""
    if n % 2:
        raise ValueError("the grid size must be even (Section 2)")
    k = np.arange(n)
    return np.where(k < n // 2, k, k - n)


def wavenumbers(n: int, lo: float, hi: float) -> np.ndarray:
    """mu_k = 2 pi k / (b - a) in FFT bin order (eq. (2.2))."""
    return 2.0 * np.pi * fft_bins(n) / (hi - lo)


def mu_squared(shape, lo, hi) -> np.ndarray:
    """|mu_k|^2 = sum over axes of mu_{k_i}^2 (eq. (2.12)), FFT bin order."""
    shape = tuple(shape)
    out = np.zeros(shape)
    for ax, n in enumerate(shape):
        mu = wavenumbers(n, lo[ax], hi[ax])
        sh = [1] * len(shape)
        sh[ax] = n
        out = out + (mu * mu).reshape(sh)
    return out


def gamma_from_Q(Q) -> np.ndarray:
    """gamma = arctan(1/Q)/pi (Section 1, coefficients of (1.1)); Q = inf gives 0."""
    Q = np.asarray(Q, dtype=np.float64)
    return np.arctan2(1.0, Q) / np.pi


def seismic_coefficients(gamma, c0: float, omega0: float):
    """Coefficients of (1.1) and the first-order form used here.

    c = c0 cos(pi gamma/2), eta = -c0^{2 gamma} omega0^{-2 gamma} cos(pi gamma),
    tau = -c0^{2 gamma - 1} omega0^{-2 gamma} sin(pi gamma). Dividing (1.1) by
    1/c^2 gives u_tt = -A (-Lap)^{1+gamma} u - B (-Lap)^{1/2+gamma} u_t with
    A = -c^2 eta and B = -c^2 tau. Returns (A, B).
    """
    g = np.asarray(gamma, dtype=np.float64)
    c = c0 * np.cos(np.pi * g / 2.0)
    eta = -(c0 ** (2.0 * g)) * omega0 ** (-2.0 * g) * np.cos(np.pi * g)
    tau = -(c0 ** (2.0 * g - 1.0)) * omega0 ** (-2.0 * g) * np.sin(np.pi * g)
    return -c * c * eta, -c * c * tau


def seismic_op_order(gamma, op: int) -> np.ndarray:
    """Order s(x) of the two operators of (1.1): op 1 -> 1+gamma, op 2 -> 1/2+gamma."""
    g = np.asarray(gamma, dtype=np.float64)
    if op == 1:
        return 1.0 + g
    if op == 2:
        return 0.5 + g
    raise ValueError("op must be 1 or 2")


# ---------------------------------------------------------------------------
# O1: exact discrete operator by explicit sums (eqs. (2.3), (2.6), (2.12))
# ---------------------------------------------------------------------------

def _phase_tables(shape):
    """Per axis: exp(2 pi i (k j mod n)/n) for k in bin order, j = 0..n-1."""
    tabs = []
    for n in shape:
        k = fft_bins(n)
        j = np.arange(n)
        r = np.mod(np.outer(k, j), n)
        tabs.append(np.exp(2j * np.pi * r / n))
    return tabs


def _phase_block(tabs, shape, jflat):
    """E[k, j] = exp(i mu_k.(x_j - a)) for all k (flat) and the given flat j."""
    N = int(np.prod(shape))
    kidx = np.unravel_index(np.arange(N), shape)
    jidx = np.unravel_index(jflat, shape)
    E = np.ones((N, len(jflat)), dtype=np.complex128)
    for ax in range(len(shape)):
        E *= tabs[ax][kidx[ax][:, None], jidx[ax][None, :]]
    return E


def dense_dft(u) -> np.ndarray:
    """u_hat_k = (1/N) sum_j u_j exp(-i mu_k.(x_j - a)) by explicit sums (eq. (2.11))."""
    u = np.asarray(u, dtype=np.float64)
    shape = u.shape
    N = u.size
    tabs = _phase_tables(shape)
    uflat = u.reshape(-1)
    uhat = np.zeros(N, dtype=np.complex128)
    chunk = max(1, min(N, 4_000_000 // N))
    for j0 in range(0, N, chunk):
        jj = np.arange(j0, min(N, j0 + chunk))
        E = _phase_block(tabs, shape, jj)
        uhat += np.conj(E) @ uflat[jj]
    return (uhat / N).reshape(shape)


def dense_apply(u, s, lo, hi) -> np.ndarray:
    """Exact discrete variable-order operator (eq. (2.12)), O(N^2).

    out_j = sum_{k != 0} |mu_k|^{2 s(x_j)} u_hat_k exp(i mu_k.(x_j - a)), real part.
    Use on tiny grids only (N up to a few thousand points).
    """
    u = np.asarray(u, dtype=np.float64)
    s = np.broadcast_to(np.asarray(s, dtype=np.float64), u.shape)
    shape = u.shape
    N = u.size
    uhat = dense_dft(u).reshape(-1)
    mu2 = mu_squared(shape, lo, hi).reshape(-1)
    nz = mu2 > 0.0
    tabs = _phase_tables(shape)
    sflat = s.reshape(-1)
    out = np.empty(N)
    chunk = max(1, min(N, 4_000_000 // N))
    for j0 in range(0, N, chunk):
        jj = np.arange(j0, min(N, j0 + chunk))
        E = _phase_block(tabs, shape, jj)[nz, :]          # (K, J)
        W = mu2[nz][:, None] ** sflat[jj][None, :]         # |mu_k|^{2 s_j}
        out[jj] = np.real(np.sum(W * E * uhat[nz][:, None], axis=0))
    return out.reshape(shape)


def dense_matrix_1d(s, lo: float, hi: float) -> np.ndarray:
    """Matrix A_{s(x)} of eq. (2.7), entries from the sum over k (first line of (2.7)).

    a_jl = (1/J) sum_k |mu_k|^{2 s(x_j)} exp(i mu_k (x_j - x_l)), real part.
    """
    s = np.asarray(s, dtype=np.float64)
    J = s.size
    k = fft_bins(J)
    mu = 2.0 * np.pi * k / (hi - lo)
    j = np.arange(J)
    A = np.zeros((J, J))
    for kk, m in zip(k, mu):
        if kk == 0:
            continue
        ph = np.exp(2j * np.pi * np.mod(kk * (j[:, None] - j[None, :]), J) / J)
        A += np.real((np.abs(m) ** (2.0 * s))[:, None] * ph)
    return A / J


# ---------------------------------------------------------------------------
# O2: M-term matrix-free scheme (eqs. (2.8)-(2.10), (2.13))
# ---------------------------------------------------------------------------

def mterm_apply(u, s, lo, hi, M: int) -> np.ndarray:
    """Matrix-free approximation (2.13) with terms m = 0..M.

    out_j = sum_m [s(x_j) - s0]^m sum_{k != 0} (ln|mu_k|^2)^m / m! |mu_k|^{2 s0}
            u_hat_k exp(i mu_k.(x_j - a)), with s0 the grid mean of s.
    """
    u = np.asarray(u, dtype=np.float64)
    s = np.broadcast_to(np.asarray(s, dtype=np.float64), u.shape)
    N = u.size
    s0 = float(np.mean(s))
    delta = s - s0
    uhat = _fftn(u) / N
    mu2 = mu_squared(u.shape, lo, hi)
    nz = mu2 > 0.0
    lnmu2 = np.zeros_like(mu2)
    lnmu2[nz] = np.log(mu2[nz])
    base = np.zeros_like(mu2)
    base[nz] = mu2[nz] ** s0                                # |mu_k|^{2 s0}
    out = np.zeros(u.shape)
    for m in range(M + 1):
        coef = lnmu2 ** m / math.factorial(m) * base        # zero at k = 0
        inner = np.real(_ifftn(coef * uhat)) * N             # sum over k
        out += delta ** m * inner
    return out


def mterm_apply_at(u, s, lo, hi, M: int, points) -> np.ndarray:
    """(2.13) at selected grid points, each computed on its own.

    For a point x_j: sum_m delta_j^m sum_{k != 0} l_m(k) |mu_k|^{2 s0} u_hat_k
    exp(i mu_k.(x_j - a)), the inner sum taken over all k explicitly. points
    is a sequence of index tuples.
    """
    u = np.asarray(u, dtype=np.float64)
    s = np.broadcast_to(np.asarray(s, dtype=np.float64), u.shape)
    shape = u.shape
    N = u.size
    s0 = float(np.mean(s))
    uhat = _fftn(u) / N
    mu2 = mu_squared(shape, lo, hi)
    nz = mu2 > 0.0
    lnmu2 = np.zeros_like(mu2)
    lnmu2[nz] = np.log(mu2[nz])
    base = np.zeros_like(mu2)
    base[nz] = mu2[nz] ** s0
    out = []
    for j in points:
        ph = np.ones(shape, dtype=np.complex128)
        for ax, n in enumerate(shape):
            k = fft_bins(n)
            e = np.exp(2j * np.pi * np.mod(k * j[ax], n) / n)
            sh = [1] * len(shape)
            sh[ax] = n
            ph = ph * e.reshape(sh)
        w = base * uhat * ph
        d = s[tuple(j)] - s0
        val = 0.0
        for m in range(M + 1):
            inner = np.real(np.sum(lnmu2 ** m / math.factorial(m) * w))
            val += d ** m * inner
        out.append(val)
    return np.array(out)


# ---------------------------------------------------------------------------
# O3: TSFP2 for model (1.5) (eqs. (3.6)-(3.14))
# ---------------------------------------------------------------------------

def _to_spec(u):
    return _fftn(u) / u.size


def _to_phys(uhat):
    return np.real(_ifftn(uhat)) * uhat.size


def tsfp2_generic(phi, psi, s, kappa: float, lo, hi, M: int, dt: float,
                  nsteps: int, f=None):
    """TSFP2 (3.13) for u_tt = -kappa (-Lap)^{s(x)} u + f(u) on a periodic box.

    Sub-problem (3.7) with the constant order s0 is solved exactly per mode by
    (3.10)-(3.11) with w_k = sqrt(kappa) |mu_k|^{s0} (the ODE above (3.10)
    carries |mu_k|^{2 s0}); sub-problem (3.8) is the kick
    v <- v + dt (-kappa T u + f(u)), T = sum_{m=1..M} of (2.13).
    Returns (u, v) after nsteps steps; non-finite values are propagated.
    """
    u = np.asarray(phi, dtype=np.float64)
    v = np.asarray(psi, dtype=np.float64)
    s = np.broadcast_to(np.asarray(s, dtype=np.float64), u.shape)
    s0 = float(np.mean(s))
    delta = s - s0
    mu2 = mu_squared(u.shape, lo, hi)
    nz = mu2 > 0.0
    lnmu2 = np.zeros_like(mu2)
    lnmu2[nz] = np.log(mu2[nz])
    base = np.zeros_like(mu2)
    base[nz] = mu2[nz] ** s0
    w = np.sqrt(kappa) * np.sqrt(base)                       # sqrt(kappa) |mu|^{s0}

    def exact_part(uh, vh, t):
        c = np.cos(w * t)
        sn = np.sin(w * t)
        ws = np.where(nz, w, 1.0)
        u_new = np.where(nz, uh * c + vh * sn / ws, uh + t * vh)        # (3.10), (3.11)
        v_new = np.where(nz, -w * uh * sn + vh * c, vh)
        return u_new, v_new

    # loop-invariant factors of (2.13): l_m |mu|^{2 s0} and delta^m, m = 1..M
    coefs = [lnmu2 ** m / math.factorial(m) * base for m in range(M + 1)]
    dpow = [delta ** m for m in range(M + 1)]
    uh, vh = _to_spec(u), _to_spec(v)
    with np.errstate(all="ignore"):
        for _ in range(nsteps):
            uh, vh = exact_part(uh, vh, dt / 2.0)
            u1 = _to_phys(uh)
            v1 = _to_phys(vh)
            tilde = np.zeros(u.shape)
            for m in range(1, M + 1):
                tilde += dpow[m] * _to_phys(coefs[m] * uh)
            rhs = -kappa * tilde
            if f is not None:
                rhs = rhs + f(u1)
            v2 = v1 + dt * rhs
            uh, vh = exact_part(_to_spec(u1), _to_spec(v2), dt / 2.0)
    return _to_phys(uh), _to_phys(vh)


def tsfp4_generic(phi, psi, s, kappa: float, lo, hi, M: int, dt: float,
                  nsteps: int, f=None):
    """Higher-order splitting for (1.5) (named after (3.13), with the
    higher-order split-step references there): each step is the symmetric
    composition of three TSFP2 steps of lengths w1 dt, w0 dt, w1 dt with
    w1 = 1/(2 - 2^{1/3}), w0 = 1 - 2 w1 (the symmetric triple jump, order 4
    for a symmetric second-order base step). Returns (u, v)."""
    w1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
    w0 = 1.0 - 2.0 * w1
    u = np.asarray(phi, dtype=np.float64)
    v = np.asarray(psi, dtype=np.float64)
    for _ in range(nsteps):
        for w in (w1, w0, w1):
            u, v = tsfp2_generic(u, v, s, kappa, lo, hi, M, w * dt, 1, f=f)
    return u, v


def lffp_generic(phi, psi, s, kappa: float, lo, hi, M: int, dt: float,
                 nsteps: int, f=None):
    """Leap-frog Fourier pseudospectral scheme (3.4) for u_tt = -kappa
    (-Lap)^{s(x)} u + f(u) on a periodic box, with (2.13) as the operator.

    u^0 = phi, u^1 = phi + dt psi + dt^2/2 F(phi) (the start (3.4b, c), as
    in (3.3)), then u^{n+1} = 2 u^n - u^{n-1} + dt^2 F(u^n), where
    F(w) = -kappa (-Lap)^{s(x)}_{h,M} w + f(w). Returns (u^{nsteps-1},
    u^{nsteps}) (with u^{-1} taken as phi for nsteps = 0); non-finite values
    are propagated.
    """
    u = np.asarray(phi, dtype=np.float64)
    s = np.broadcast_to(np.asarray(s, dtype=np.float64), u.shape)
    s0 = float(np.mean(s))
    delta = s - s0
    mu2 = mu_squared(u.shape, lo, hi)
    nz = mu2 > 0.0
    lnmu2 = np.zeros_like(mu2)
    lnmu2[nz] = np.log(mu2[nz])
    base = np.zeros_like(mu2)
    base[nz] = mu2[nz] ** s0
    # loop-invariant factors of (2.13): l_m |mu|^{2 s0} and delta^m, m = 0..M
    coefs = [lnmu2 ** m / math.factorial(m) * base for m in range(M + 1)]
    dpow = [delta ** m for m in range(M + 1)]

    def F(w):
        wh = _to_spec(w)
        lw = np.zeros(w.shape)
        for m in range(M + 1):
            lw += dpow[m] * _to_phys(coefs[m] * wh)
        out = -kappa * lw
        if f is not None:
            out = out + f(w)
        return out

    if nsteps == 0:
        return u.copy(), u.copy()
    with np.errstate(all="ignore"):
        prev = u
        cur = u + dt * np.asarray(psi, dtype=np.float64) + 0.5 * dt * dt * F(u)
        for _ in range(nsteps - 1):
            prev, cur = cur, 2.0 * cur - prev + dt * dt * F(cur)
    return prev, cur


def cnfp_generic(phi, psi, s, kappa: float, lo, hi, M: int, dt: float,
                 nsteps: int, f=None, tol: float = 1e-14, max_outer: int = 100):
    """Crank-Nicolson Fourier pseudospectral scheme (3.2) with the start (3.3)
    for u_tt = -kappa (-Lap)^{s(x)} u + f(u), (2.13) as the operator L.

    Each step solves for w = u^{n+1}:
      w + a L w - b f(w) = 2 u^n - u^{n-1} - a L u^{n-1} + b f(u^{n-1}),
    a = kappa dt^2/2, b = dt^2/2, by fixed-point iteration on f(w); every
    linear solve with I + a L uses the library's GMRES, preconditioned by the
    exact inverse of I + a (-Lap)^{s0} (a Fourier multiplier), to a relative
    residual of tol. Returns (u^{nsteps-1}, u^{nsteps}).
    """
    from scipy.sparse.linalg import LinearOperator, gmres
    u = np.asarray(phi, dtype=np.float64)
    shape = u.shape
    N = u.size
    s = np.broadcast_to(np.asarray(s, dtype=np.float64), shape)
    s0 = float(np.mean(s))
    delta = s - s0
    mu2 = mu_squared(shape, lo, hi)
    nz = mu2 > 0.0
    lnmu2 = np.zeros_like(mu2)
    lnmu2[nz] = np.log(mu2[nz])
    base = np.zeros_like(mu2)
    base[nz] = mu2[nz] ** s0
    # constant order: delta = 0, so only the m = 0 term is nonzero
    nterms = M + 1 if np.any(delta != 0.0) else 1
    coefs = [lnmu2 ** m / math.factorial(m) * base for m in range(nterms)]
    dpow = [delta ** m for m in range(nterms)]

    def L(w):
        wh = _to_spec(w)
        out = np.zeros(shape)
        for m in range(nterms):
            out += dpow[m] * _to_phys(coefs[m] * wh)
        return out

    def fv(w):
        return f(w) if f is not None else np.zeros(shape)

    a = kappa * dt * dt / 2.0
    b = dt * dt / 2.0
    A = LinearOperator((N, N), matvec=lambda x: (x.reshape(shape) + a * L(x.reshape(shape))).ravel(),
                       dtype=np.float64)
    inv0 = 1.0 / (1.0 + a * base)
    P = LinearOperator((N, N), matvec=lambda x: _to_phys(inv0 * _to_spec(x.reshape(shape))).ravel(),
                       dtype=np.float64)
    if nsteps == 0:
        return u.copy(), u.copy()
    prev = u
    cur = u + dt * np.asarray(psi, dtype=np.float64) + b * (-kappa * L(u) + fv(u))
    for _ in range(nsteps - 1):
        r = 2.0 * cur - prev - a * L(prev) + b * fv(prev)
        w = 2.0 * cur - prev
        for _ in range(max_outer):
            rhs = r + b * fv(w)
            x, info = gmres(A, rhs.ravel(), x0=w.ravel(), rtol=tol, atol=0.0, restart=50, maxiter=200, M=P)
            if info != 0:
                raise RuntimeError(f"GMRES did not converge (info {info})")
            wn = x.reshape(shape)
            done = np.linalg.norm(wn - w) <= tol * max(np.linalg.norm(wn), 1e-300)
            w = wn
            if done:
                break
        prev, cur = cur, w
    return prev, cur


# ---------------------------------------------------------------------------
# O4: TSFP2 for the viscoacoustic model (1.1)
# ---------------------------------------------------------------------------

def damped_propagator(P1, P2, kappa0: float, beta0: float, t: float):
    """Exact flow of u' = v, v' = -kappa0 P1 u - beta0 P2 v over time t, per mode.

    Returns (g11, g12, g21, g22) with (u, v)(t) = [[g11, g12], [g21, g22]] (u, v)(0).
    With b = beta0 P2 / 2, q = kappa0 P1, w^2 = q - b^2:
      u(t) = e^{-bt} [(C + b S) u0 + S v0],  v(t) = e^{-bt} [-q S u0 + (C - b S) v0],
    C = cos(wt), S = sin(wt)/w (w^2 > 0); cosh/sinh for w^2 < 0; C = 1, S = t at w = 0.
    For beta0 = 0 this is (3.10), and for P1 = P2 = 0 it is (3.11).
    """
    P1 = np.asarray(P1, dtype=np.float64)
    P2 = np.asarray(P2, dtype=np.float64)
    b = 0.5 * beta0 * P2
    q = kappa0 * P1
    w2 = q - b * b
    C = np.ones_like(w2)
    S = np.full_like(w2, float(t))
    pos = w2 > 0.0
    neg = w2 < 0.0
    wp = np.sqrt(w2[pos])
    C[pos] = np.cos(wp * t)
    S[pos] = np.sin(wp * t) / wp
    wn = np.sqrt(-w2[neg])
    C[neg] = np.cosh(wn * t)
    S[neg] = np.sinh(wn * t) / wn
    e = np.exp(-b * t)
    return e * (C + b * S), e * S, -e * q * S, e * (C - b * S)


def tsfp2_seismic(u0, v0, gamma, c0: float, omega0: float, lo, hi, M: int,
                  dt: float, nsteps: int):
    """TSFP2 for (1.1), steps taken one by one in physical/spectral form.

    c0 is a number or a field of per-point phase velocities (a layered
    medium); A and B are formed point by point, and the exact part uses
    kappa0 = A(gbar, cbar), beta0 = B(gbar, cbar) with cbar the grid mean of c0.

    Per step: exact part over dt/2, kick, exact part over dt/2, where the kick is
      v <- v + dt [(kappa0 - A) t1_0 - A sum_{m>=1} delta^m t1_m
                   + (beta0 - B) t2_0 - B sum_{m>=1} delta^m t2_m],
    t1_m = IDFT(l_m |mu|^{2(1+gbar)} u_hat), t2_m = IDFT(l_m |mu|^{2(1/2+gbar)} v_hat),
    l_m = (ln|mu|^2)^m / m!, delta = gamma - gbar (eq. (2.13) for both orders).
    Returns (u, v).
    """
    u = np.asarray(u0, dtype=np.float64)
    v = np.asarray(v0, dtype=np.float64)
    gamma = np.broadcast_to(np.asarray(gamma, dtype=np.float64), u.shape)
    gbar = float(np.mean(gamma))
    delta = gamma - gbar
    c0 = np.broadcast_to(np.asarray(c0, dtype=np.float64), u.shape)
    A, B = seismic_coefficients(gamma, c0, omega0)
    # exact part: coefficients at the mean order and the mean phase velocity
    kappa0, beta0 = (float(x) for x in seismic_coefficients(gbar, float(np.mean(c0)), omega0))
    mu2 = mu_squared(u.shape, lo, hi)
    nz = mu2 > 0.0
    lnmu2 = np.zeros_like(mu2)
    lnmu2[nz] = np.log(mu2[nz])
    P1 = np.zeros_like(mu2)
    P2 = np.zeros_like(mu2)
    P1[nz] = mu2[nz] ** (1.0 + gbar)
    P2[nz] = mu2[nz] ** (0.5 + gbar)
    g = damped_propagator(P1, P2, kappa0, beta0, dt / 2.0)

    def exact_part(uh, vh):
        return g[0] * uh + g[1] * vh, g[2] * uh + g[3] * vh

    # loop-invariant factors: l_m |mu|^{2 sigma} for both orders, and delta^m
    c1 = [lnmu2 ** m / math.factorial(m) * P1 for m in range(M + 1)]
    c2 = [lnmu2 ** m / math.factorial(m) * P2 for m in range(M + 1)]
    dpow = [delta ** m for m in range(M + 1)]
    uh, vh = _to_spec(u), _to_spec(v)
    with np.errstate(all="ignore"):
        for _ in range(nsteps):
            uh, vh = exact_part(uh, vh)
            u1 = _to_phys(uh)
            v1 = _to_phys(vh)
            t1 = [_to_phys(c1[m] * uh) for m in range(M + 1)]
            t2 = [_to_phys(c2[m] * vh) for m in range(M + 1)]
            tilde1 = np.zeros(u.shape)
            tilde2 = np.zeros(u.shape)
            for m in range(1, M + 1):
                tilde1 += dpow[m] * t1[m]
                tilde2 += dpow[m] * t2[m]
            dv = (kappa0 - A) * t1[0] - A * tilde1 + (beta0 - B) * t2[0] - B * tilde2
            v2 = v1 + dt * dv
            uh, vh = exact_part(_to_spec(u1), _to_spec(v2))
    return _to_phys(uh), _to_phys(vh)


def lffp_seismic(phi, psi, gamma, c0, omega0: float, lo, hi, M: int, dt: float,
                 nsteps: int):
    """Leap-frog scheme (3.4) carried over to the viscoacoustic model (1.1)
    (the scheme of Example 3; the paper does not write it out, reading below).

    With A = -c^2 eta and B = -c^2 tau (seismic_coefficients; c0 may be a
    field of per-point phase velocities), (1.1) reads
    u_tt = -A L1 u - B L2 u_t, L1 = (-Lap)^{1+gamma(x)}, L2 = (-Lap)^{1/2+gamma(x)},
    both by the M-term expansion (2.13) about their grid-mean orders. The
    time derivative inside the damping term is the backward difference
    (u^n - u^{n-1})/dt, which keeps the scheme explicit; the start is the
    Taylor step of (3.4c) with u_t(0) = psi:
      u^1     = phi + dt psi + dt^2/2 (-A L1 phi - B L2 psi),
      u^{n+1} = 2 u^n - u^{n-1} + dt^2 (-A L1 u^n - B L2 (u^n - u^{n-1})/dt).
    Returns (u^{nsteps-1}, u^{nsteps}) (both phi for nsteps = 0).
    """
    u = np.asarray(phi, dtype=np.float64)
    gamma = np.broadcast_to(np.asarray(gamma, dtype=np.float64), u.shape)
    c0 = np.broadcast_to(np.asarray(c0, dtype=np.float64), u.shape)
    gbar = float(np.mean(gamma))
    delta = gamma - gbar
    A, B = seismic_coefficients(gamma, c0, omega0)
    mu2 = mu_squared(u.shape, lo, hi)
    nz = mu2 > 0.0
    lnmu2 = np.zeros_like(mu2)
    lnmu2[nz] = np.log(mu2[nz])
    P1 = np.zeros_like(mu2)
    P2 = np.zeros_like(mu2)
    P1[nz] = mu2[nz] ** (1.0 + gbar)
    P2[nz] = mu2[nz] ** (0.5 + gbar)
    c1 = [lnmu2 ** m / math.factorial(m) * P1 for m in range(M + 1)]
    c2 = [lnmu2 ** m / math.factorial(m) * P2 for m in range(M + 1)]
    dpow = [delta ** m for m in range(M + 1)]

    def op(w, cm):
        wh = _to_spec(w)
        out = np.zeros(w.shape)
        for m in range(M + 1):
            out += dpow[m] * _to_phys(cm[m] * wh)
        return out

    def F(w, wt):
        return -A * op(w, c1) - B * op(wt, c2)

    if nsteps == 0:
        return u.copy(), u.copy()
    with np.errstate(all="ignore"):
        prev = u
        cur = u + dt * np.asarray(psi, dtype=np.float64) + 0.5 * dt * dt * F(u, np.asarray(psi, dtype=np.float64))
        for _ in range(nsteps - 1):
            prev, cur = cur, 2.0 * cur - prev + dt * dt * F(cur, (cur - prev) / dt)
    return prev, cur


# ---------------------------------------------------------------------------
# Norms (Tables 2-5)
# ---------------------------------------------------------------------------

def weighted_l2(e, h) -> float:
    """(prod(h) sum e^2)^{1/2}: the l2 norm of the error tables (reading, fits Tables 4-5)."""
    e = np.asarray(e, dtype=np.float64)
    return float(np.sqrt(np.prod(np.atleast_1d(h)) * np.sum(e * e)))


def rel_l2(a, ref) -> float:
    """||a - ref||_2 / ||ref||_2 (unweighted)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((a - ref).ravel()) / (den if den > 0 else 1.0))
