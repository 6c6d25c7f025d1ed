"""Shared helpers of the GPU tests: device transfer and plan construction."""

import numpy as np

TOL_FP64 = 1e-12   # parity_err bound, FP64 path vs FP64 oracle
TOL_FP32 = 1e-5    # parity_err bound, FP32 path (FP64 coefficients/state) vs FP64 oracle


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device (no CPU fallback exists)"
    return torch


def dev(x, precision):
    import torch
    dt = torch.float32 if precision == "fp32" else torch.float64
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float64))).to("cuda", dt)


def as_seen(x, precision):
    """The values a plan of this precision receives: x rounded to FP32 for
    FP32 plans (the oracle is run on exactly these inputs)."""
    x = np.asarray(x, dtype=np.float64)
    return x.astype(np.float32).astype(np.float64) if precision == "fp32" else x


def host(t):
    return t.detach().double().cpu().numpy()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_rel(a, b):
    """Largest element-wise error over the reference's largest modulus."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) if b.size else 0.0


def parity_err(a, b):
    """The error every GPU parity test bounds: the larger of the relative L2
    error over the whole field and the element-wise error max|a - b| over
    max|b|. A bound on it holds both ways, so an error confined to a few
    planes, a Nyquist line or one tile column cannot hide inside the norm."""
    return max(rel_l2(a, b), max_rel(a, b))


def tol(precision):
    return TOL_FP32 if precision == "fp32" else TOL_FP64


def say(msg):
    print(msg, flush=True)
