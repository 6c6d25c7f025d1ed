"""The remaining C-ABI calls on the GPU: vofl_solve (copy + steps, aliased
and separate outputs), vofl_plan_info (the plan's scalars against the
oracle's coefficient formulas and vofl_plan_footprint), and the per-class
kernel timing of vofl_set_timing / vofl_kernel_times (launch counts of one
vofl_step call)."""

import numpy as np
import pytest

import oracle as O
from gpu_helpers import dev, host, require_gpu, say
from workloads import gaussian_pulse, grf_Q, rng_for

pytestmark = pytest.mark.gpu

SHAPE, LO, HI = (32, 48), (-4.0, -6.0), (4.0, 6.0)


def _plan(precision="fp64", **kw):
    require_gpu()
    from paper_2311_13049_amd import vofl as V
    Q = grf_Q(SHAPE, LO, HI, rng_for(95), corr_len=1.5, qmin=2.0, qmax=40.0)
    return V.Plan(SHAPE, LO, HI, precision=precision, Q=Q, M=6, dt=2e-3, c0=1.3, omega0=0.8, **kw), Q


def test_solve_equals_copy_then_step():
    import torch
    p, _ = _plan()
    u0 = dev(gaussian_pulse(SHAPE, LO, HI, (0.5, -1.0)), "fp64")
    v0 = dev(0.2 * gaussian_pulse(SHAPE, LO, HI, (-1.0, 0.5)), "fp64")
    say("vofl_solve vs copy + vofl_step, separate and aliased outputs")
    u, v = p.solve(u0, v0, 9)                    # new output tensors
    ue, ve = u0.clone(), v0.clone()
    p.step(ue, ve, 9)
    ua, va = u0.clone(), v0.clone()
    p.solve(ua, va, 9, u=ua, v=va)               # inputs are the outputs
    torch.cuda.synchronize()
    assert p.sync_status() == 0
    assert torch.equal(u, ue) and torch.equal(v, ve)
    assert torch.equal(ua, ue) and torch.equal(va, ve)
    assert not torch.equal(u0, u)                # the inputs are left alone


def test_plan_info_matches_coefficients_and_footprint():
    from paper_2311_13049_amd import vofl as V
    p, Q = _plan(precision="fp32")
    info = p.info()
    gbar = float(np.mean(O.gamma_from_Q(Q)))
    k0, b0 = (float(x) for x in O.seismic_coefficients(gbar, 1.3, 0.8))
    say(f"plan info {info}")
    assert info["N"] == SHAPE[0] * SHAPE[1]
    assert abs(info["mean_order_offset"] - gbar) <= 1e-15
    assert abs(info["kappa0"] - k0) <= 1e-14 * abs(k0)
    assert abs(info["beta0"] - b0) <= 1e-14 * abs(b0)
    d, keep = V.make_desc(SHAPE, LO, HI, Q=Q, M=6, dt=2e-3, c0=1.3, omega0=0.8, precision="fp32")
    assert info["device_bytes"] == V.vofl_plan_footprint(d)


def test_kernel_times_count_the_launches_of_one_step_call():
    import torch
    p, _ = _plan()
    u = dev(gaussian_pulse(SHAPE, LO, HI, (0.0, 0.0)), "fp64")
    v = torch.zeros_like(u)
    p.set_timing(True)
    p.step(u, v, 5)
    torch.cuda.synchronize()
    kt = p.kernel_times()
    p.set_timing(False)
    say(f"kernel classes {sorted(kt)}")
    launches = {k: n for k, (_, n) in kt.items()}
    # 2D: forward transforms of u and v, the first exact half step with the
    # terms, then per step the kick pair of passes, and the final export
    assert launches["r2c0"] == 2
    assert launches["contig_init"] == 1
    assert launches["c2r0_kick"] == 5
    assert launches["contig_kick"] == 5
    assert launches["c2r0_export"] == 1
    assert all(ms > 0.0 for ms, _ in kt.values())
    # timing off: no further records
    p.step(u, v, 2)
    torch.cuda.synchronize()
    assert p.kernel_times()["c2r0_kick"][1] == 5


def test_stream_probe_streams_move_the_bytes_they_name():
    """The measurement probe: a copy reproduces its source, a write fills the
    documented pattern, a read leaves the destination alone; every kind with
    a ragged tail (bytes not a multiple of one trip), both depths and both
    cache policies."""
    import torch
    require_gpu()
    from paper_2311_13049_amd import vofl as V
    cur = torch.cuda.current_stream().cuda_stream
    nvec = 3 * 256 * 16 * 7 + 13          # 16-byte vectors: several trips and a tail
    src = torch.randn(nvec * 4, device="cuda")
    for flags in (0, V.VOFL_PROBE_NONTEMPORAL, V.VOFL_PROBE_DEEP, V.VOFL_PROBE_NONTEMPORAL | V.VOFL_PROBE_DEEP):
        for blocks in (1, 5, 64):
            say(f"stream probe nvec={nvec} blocks={blocks} flags={flags}")
            dst = torch.full_like(src, -3.0)
            V.vofl_stream_probe(V.VOFL_PROBE_READ, src.data_ptr(), dst.data_ptr(), nvec * 16, blocks, flags, cur)
            torch.cuda.synchronize()
            assert bool((dst == -3.0).all())
            V.vofl_stream_probe(V.VOFL_PROBE_COPY, src.data_ptr(), dst.data_ptr(), nvec * 16, blocks, flags, cur)
            torch.cuda.synchronize()
            assert torch.equal(dst, src)
            V.vofl_stream_probe(V.VOFL_PROBE_WRITE, 0, dst.data_ptr(), nvec * 16, blocks, flags, cur)
            torch.cuda.synchronize()
            i = torch.arange(nvec, device="cuda") & 1023
            want = (i.float()[:, None] + torch.arange(4, device="cuda").float()[None, :]).reshape(-1)
            assert torch.equal(dst, want)


def test_arguments_outside_their_domain_are_refused_and_leave_outputs_alone():
    """Calls with a field count outside [1, max_batch], a negative step count
    or an unknown operator return VOFL_ERR_INVALID before any launch, and the
    caller's buffers keep their values; zero steps is a no-op."""
    import torch
    from paper_2311_13049_amd import vofl as V
    p, _ = _plan(max_batch=2)
    lib = V.load_library()
    u = dev(gaussian_pulse(SHAPE, LO, HI, (0.0, 0.0)), "fp64")
    v = torch.zeros_like(u)
    out = torch.full((3,) + SHAPE, 7.0, dtype=torch.float64, device="cuda")
    u3 = torch.stack([u, u, u]).contiguous()
    s = torch.cuda.current_stream().cuda_stream
    h = p.handle
    say("domain checks of vofl_apply / vofl_step")
    assert lib.vofl_apply(h, V.VOFL_OP_S1, u3.data_ptr(), out.data_ptr(), 0, s) == V.VOFL_ERR_INVALID
    assert lib.vofl_apply(h, V.VOFL_OP_S1, u3.data_ptr(), out.data_ptr(), 3, s) == V.VOFL_ERR_INVALID
    assert lib.vofl_apply(h, 3, u3.data_ptr(), out.data_ptr(), 1, s) == V.VOFL_ERR_INVALID
    assert lib.vofl_step(h, u.data_ptr(), v.data_ptr(), -1, s) == V.VOFL_ERR_INVALID
    u_before = u.clone()
    assert lib.vofl_step(h, u.data_ptr(), v.data_ptr(), 0, s) == V.VOFL_OK
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    assert torch.equal(u, u_before) and bool((v == 0).all())
    assert p.sync_status() == 0
