"""Serving on the GPU: continuous batching of wave solves of different grids,
Q fields, M and precisions (request stream with Poisson arrivals).

Checks: every result served in the mix equals the same request solved alone
(bit for bit, hence within the stated tolerance), sampled results agree with
the FP64 oracle, the memory budget bounds what is admitted at once, requests
that can never fit are rejected without blocking the rest, and the latency
record is consistent.
"""

import numpy as np
import pytest

import oracle as O
from gpu_helpers import TOL_FP32, TOL_FP64, as_seen, parity_err, require_gpu, say
from workloads import c5_requests

pytestmark = pytest.mark.gpu

GRIDS = [(64, 64), (128, 128), (256, 256), (32, 32, 32), (64, 64, 64)]


def _serve():
    require_gpu()
    from paper_2311_13049_amd import serve as S
    return S


def _trace(count, seed_offset=0, step_scale=0.03):
    S = _serve()
    recs = c5_requests(count=count, rate=2000.0, grids=GRIDS, seed_offset=seed_offset)
    return S.requests_from_stream(recs, step_scale=step_scale)


def test_mix_equals_alone_and_oracle():
    S = _serve()
    reqs = _trace(12)
    say(f"serve mix: {len(reqs)} requests, steps {[r.steps for r in reqs]}")
    mix, stats = S.Server(slots=6, chunk=8).run(reqs, realtime=True)
    say(f"  mix stats: {stats}")
    assert stats["completed"] == len(reqs) and stats["peak_active"] > 1
    # alone: one request at a time, same chunking, eager launches
    alone, _ = S.Server(slots=1, chunk=8, graphs=False).run(reqs, realtime=False)
    # plain path: one request at a time, the whole solve in one vofl_step call
    # (chunk boundaries split a merged half-step, so equal only to rounding)
    whole, _ = S.Server(slots=1, chunk=0, graphs=False).run(reqs, realtime=False)
    for r in reqs:
        a, b, c = mix[r.index], alone[r.index], whole[r.index]
        assert a.status == "ok" and b.status == "ok" and c.status == "ok"
        assert np.array_equal(a.u, b.u) and np.array_equal(a.v, b.v), f"request {r.index}"
        assert parity_err(a.u, c.u) <= (TOL_FP32 if r.precision == "fp32" else TOL_FP64)
    for prec in ("fp64", "fp32"):
        r = next(q for q in reqs if q.precision == prec)
        say(f"  oracle check request {r.index} {r.shape} M={r.M} steps={r.steps} {prec}")
        ru, rv = O.tsfp2_seismic(as_seen(r.u0, prec), np.zeros(r.shape), O.gamma_from_Q(r.Q),
                                 r.c0, r.omega0, r.lo, r.hi, r.M, r.dt, r.steps)
        e = parity_err(mix[r.index].u, ru)
        say(f"    parity err {e:.3e}")
        assert e <= (TOL_FP32 if prec == "fp32" else TOL_FP64)


def test_time_sliced_mix_equals_alone():
    """Default server (chunks sized to about 2 ms of device time, least
    remaining work issued first) against the same requests one at a time."""
    S = _serve()
    reqs = _trace(10, seed_offset=3, step_scale=0.05)
    say(f"serve time-sliced mix: {len(reqs)} requests")
    mix, stats = S.Server(slots=8).run(reqs, realtime=True)
    say(f"  stats: {stats}")
    alone, _ = S.Server(slots=1).run(reqs, realtime=False)
    for r in reqs:
        assert mix[r.index].status == "ok"
        assert np.array_equal(mix[r.index].u, alone[r.index].u), f"request {r.index}"
        assert np.array_equal(mix[r.index].v, alone[r.index].v), f"request {r.index}"


def test_budget_bounds_concurrency_and_rejects_oversize():
    S = _serve()
    reqs = _trace(8, seed_offset=1)
    sizes = [S.footprint(r, r.precision) for r in reqs]
    budget = int(1.2 * max(sizes))
    big = max(range(len(reqs)), key=lambda i: sizes[i])
    # one request that can never fit: a 3D grid far above the budget
    huge = S.Request(index=99, arrival=0.0, shape=(256, 256, 256), M=16, steps=1, precision="fp64",
                     lo=(-16.0,) * 3, hi=(16.0,) * 3, dt=1e-3, Q=np.full((256,) * 3, 50.0),
                     u0=np.zeros((256,) * 3))
    say(f"serve with budget {budget} bytes (largest request {sizes[big]})")
    res, stats = S.Server(slots=8, budget=budget, chunk=4).run(reqs + [huge], realtime=False)
    say(f"  stats: {stats}")
    assert res[99].status == "rejected"
    assert stats["peak_bytes"] <= budget
    assert stats["completed"] == len(reqs)
    for r in reqs:
        x = res[r.index]
        assert x.finished >= x.started >= x.admitted
        assert np.isfinite(x.u).all()


def test_zero_step_request_returns_initial_data():
    S = _serve()
    r = _trace(1, seed_offset=2)[0]
    r.steps = 0
    res, _ = S.Server(slots=2, chunk=4).run([r], realtime=False)
    x = res[r.index]
    assert x.status == "ok"
    np.testing.assert_array_equal(x.u, as_seen(r.u0, r.precision))
    np.testing.assert_array_equal(x.v, np.zeros(r.shape))
