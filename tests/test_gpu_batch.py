"""Batched shots on the GPU: 64 solves on 512^2 sharing one random-field Q and
16 solves on 768^2 with their own Q (M = 12, FP32 transforms, dt = 5e-4),
run as two batched plans, through vofl_step_batch, through captured graphs
(vofl_step_graph) and with autotuned kernel variants.

Checks: sampled shots against the FP64 oracle (TSFP2 (3.13) for (1.1)),
each batched shot bit for bit equal to the same shot solved alone, the
multi-plan batch equal to the plans run one after another, every graph
replay equal to the eager steps, and tuned plans within the FP32 bound.
"""

import os

import numpy as np
import pytest

import oracle as O
from gpu_helpers import TOL_FP32, as_seen, dev, host, parity_err, require_gpu, say
from workloads import c4_inputs

pytestmark = pytest.mark.gpu

PREC = "fp32"
ORACLE_STEPS = 30


@pytest.fixture(scope="module")
def c4():
    return c4_inputs()


def _V():
    require_gpu()
    from paper_2311_13049_amd import vofl as V
    return V


def _group(c4, big):
    shots = [s for s in c4["shots"] if (s["shape"][0] == 768) == big]
    return shots


def _plan(c4, shots, shared, **kw):
    V = _V()
    shape = shots[0]["shape"]
    Q = shots[0]["Q"] if shared else np.stack([s["Q"] for s in shots])
    return V.Plan(shape, c4["lo"], c4["hi"], Q=Q, M=c4["M"], dt=c4["dt"], precision=PREC,
                  c0=c4["c0"], omega0=c4["omega0"], batch=len(shots),
                  coef_per_solve=not shared, **kw)


def _fields(shots):
    import torch
    u = dev(np.stack([s["u0"] for s in shots]), PREC)
    v = torch.zeros_like(u)
    return u, v


def _oracle(c4, shot, nsteps):
    O.set_fft_workers(min(8, os.cpu_count() or 1))
    try:
        u, v = O.tsfp2_seismic(as_seen(shot["u0"], PREC), np.zeros(shot["shape"]),
                               O.gamma_from_Q(shot["Q"]), c4["c0"], c4["omega0"], c4["lo"],
                               c4["hi"], c4["M"], c4["dt"], nsteps)
    finally:
        O.set_fft_workers(0)
    return u, v


def _step_batch(plans, us, vs, nsteps):
    import torch
    V = _V()
    V.vofl_step_batch([p.handle for p in plans], [u.data_ptr() for u in us],
                      [v.data_ptr() for v in vs], list(nsteps),
                      torch.cuda.current_stream().cuda_stream)


def test_c4_batch_sampled_shots_vs_oracle(c4):
    """Both groups in one vofl_step_batch call; shots 0 and 37 of the 512^2
    group and 0 and 11 of the 768^2 group against the oracle."""
    import torch
    small, big = _group(c4, False), _group(c4, True)
    assert len(small) == 64 and len(big) == 16
    say(f"c4 batch: {len(small)} x 512^2 shared Q + {len(big)} x 768^2 own Q, {ORACLE_STEPS} steps")
    pa, pb = _plan(c4, small, True), _plan(c4, big, False)
    ua, va = _fields(small)
    ub, vb = _fields(big)
    _step_batch([pa, pb], [ua, ub], [va, vb], [ORACLE_STEPS, ORACLE_STEPS])
    torch.cuda.synchronize()
    assert pa.sync_status() == 0 and pb.sync_status() == 0
    hua = host(ua).reshape((64, 512, 512))
    hva = host(va).reshape((64, 512, 512))
    hub = host(ub).reshape((16, 768, 768))
    for grp, idx, hu, hv in (("512", 0, hua, hva), ("512", 37, hua, hva),
                             ("768", 0, hub, None), ("768", 11, hub, None)):
        shots = small if grp == "512" else big
        say(f"  oracle shot {grp}^2 #{idx}")
        ru, rv = _oracle(c4, shots[idx], ORACLE_STEPS)
        eu = parity_err(hu[idx], ru)
        say(f"    parity err u {eu:.3e}")
        assert eu <= TOL_FP32
        if hv is not None:
            ev = parity_err(hv[idx], rv)
            say(f"    parity err v {ev:.3e}")
            assert ev <= TOL_FP32


def test_c4_full_run_batched_equals_alone(c4):
    """All 200 steps: sampled shots of each batched group are bit-identical to
    the same shot solved alone by a batch-1 plan (no cross-shot coupling)."""
    import torch
    steps = c4["steps"]
    small, big = _group(c4, False), _group(c4, True)
    pa, pb = _plan(c4, small, True), _plan(c4, big, False)
    ua, va = _fields(small)
    ub, vb = _fields(big)
    say(f"c4 full run {steps} steps, batched")
    _step_batch([pa, pb], [ua, ub], [va, vb], [steps, steps])
    torch.cuda.synchronize()
    assert pa.sync_status() == 0 and pb.sync_status() == 0
    for grp, shots, u, v, idx in (("512", small, ua, va, 63), ("768", big, ub, vb, 5)):
        say(f"  alone {grp}^2 #{idx}")
        p1 = _plan(c4, [shots[idx]], True)
        u1, v1 = _fields([shots[idx]])
        p1.step(u1, v1, steps)
        torch.cuda.synchronize()
        assert torch.equal(u[idx].reshape(-1), u1.reshape(-1))
        assert torch.equal(v[idx].reshape(-1), v1.reshape(-1))
        assert bool(torch.isfinite(u1).all())
        p1.close()


def test_step_batch_equals_plans_in_sequence(c4):
    """vofl_step_batch over uneven step counts equals each plan's vofl_step."""
    import torch
    small, big = _group(c4, False)[:8], _group(c4, True)[:3]
    pa, pb = _plan(c4, small, True), _plan(c4, big, False)
    ua, va = _fields(small)
    ub, vb = _fields(big)
    ua2, va2, ub2, vb2 = ua.clone(), va.clone(), ub.clone(), vb.clone()
    say("step_batch (8 x 512^2 for 7 steps, 3 x 768^2 for 4 steps) vs sequence")
    _step_batch([pa, pb], [ua, ub], [va, vb], [7, 4])
    pa.step(ua2, va2, 7)
    pb.step(ub2, vb2, 4)
    torch.cuda.synchronize()
    for x, y in ((ua, ua2), (va, va2), (ub, ub2), (vb, vb2)):
        assert torch.equal(x, y)


def test_graph_replays_equal_eager_steps(c4):
    """A captured 5-step graph, replayed 3 times with other device work and
    host synchronisation in between; every replay equals the eager steps."""
    import torch
    small = _group(c4, False)[:16]
    big = _group(c4, True)[:4]
    for shots, shared in ((small, True), (big, False)):
        p = _plan(c4, shots, shared)
        ug, vg = _fields(shots)
        ue, ve = ug.clone(), vg.clone()
        scratch = torch.randn(1 << 20, device="cuda")
        for rep in range(3):
            say(f"graph replay {rep} ({len(shots)} x {shots[0]['shape']})")
            p.step_graph(ug, vg, 5)
            scratch.mul_(1.0001).add_(0.5)  # unrelated eager work between replays
            p.step(ue, ve, 5)
            torch.cuda.synchronize()
            assert torch.equal(ug, ue) and torch.equal(vg, ve)
        assert p.sync_status() == 0
        p.close()


def test_step_batch_captured_as_one_graph_equals_eager(c4):
    """vofl_step_batch of both groups (forked onto the plans' streams and
    joined) captured into one graph by the caller, replayed 3 times with other
    device work and host synchronisation in between: every replay equals the
    same steps run eagerly."""
    import torch
    small, big = _group(c4, False)[:8], _group(c4, True)[:3]
    pa, pb = _plan(c4, small, True), _plan(c4, big, False)
    ua, va = _fields(small)
    ub, vb = _fields(big)
    ea, fa, eb, fb = ua.clone(), va.clone(), ub.clone(), vb.clone()
    _step_batch([pa, pb], [ea, eb], [fa, fb], [1, 1])  # first call: internal streams exist
    _step_batch([pa, pb], [ua, ub], [va, vb], [1, 1])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    say("capture vofl_step_batch (8 x 512^2 and 3 x 768^2, 4 and 3 steps)")
    with torch.cuda.graph(g, stream=cap):
        _step_batch([pa, pb], [ua, ub], [va, vb], [4, 3])
    torch.cuda.synchronize()
    # the capture ran nothing: the fields still hold the 1-step state
    assert torch.equal(ua, ea) and torch.equal(ub, eb)
    scratch = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        say(f"one-graph replay {rep}")
        g.replay()
        scratch.mul_(1.0001).add_(0.5)
        _step_batch([pa, pb], [ea, eb], [fa, fb], [4, 3])
        torch.cuda.synchronize()
        for x, y in ((ua, ea), (va, fa), (ub, eb), (vb, fb)):
            assert torch.equal(x, y)
    assert pa.sync_status() == 0 and pb.sync_status() == 0
    del g
    pa.close()
    pb.close()


def test_graph_cache_keys_on_buffers_and_steps(c4):
    """Different (u, v, nsteps) get their own graphs; more than the cache holds
    still gives correct results (oldest graphs are dropped)."""
    import torch
    shots = _group(c4, False)[:2]
    p = _plan(c4, shots, True)
    ue, ve = _fields(shots)
    bufs = [_fields(shots) for _ in range(3)]
    say("graph cache: 3 buffer pairs x nsteps 1..4")
    total = 0
    for k in range(1, 5):
        for (u, v) in bufs:
            p.step_graph(u, v, k)
        p.step(ue, ve, k)
        total += k
    torch.cuda.synchronize()
    for (u, v) in bufs:
        assert torch.equal(u, ue) and torch.equal(v, ve)
    p.close()


def test_autotuned_plans_pick_listed_variants_and_stay_accurate(c4, tmp_path):
    """tune_steps > 0 times the axis-0 kernel variants inside vofl_plan; the
    chosen variant is reported, written to the cache file, read back by a
    second plan, and the tuned run agrees with the oracle."""
    import torch
    os.environ["VOFL_TUNE_CACHE"] = str(tmp_path / "tune.txt")
    try:
        for big in (False, True):
            shots = _group(c4, big)[:4]
            say(f"autotune {shots[0]['shape']} x {len(shots)}")
            p = _plan(c4, shots, not big, tune_steps=3)
            info = p.info()
            assert info["c2r_variant"] in (0, 2, 5, 6, 11, 12, 13, 14)
            assert info["contig_variant"] in (0, 1)
            q = _plan(c4, shots, not big, tune_steps=3)  # served from the cache file
            assert q.info()["c2r_variant"] == info["c2r_variant"]
            assert q.info()["contig_variant"] == info["contig_variant"]
            u, v = _fields(shots)
            p.step(u, v, 10)
            torch.cuda.synchronize()
            ru, _ = _oracle(c4, shots[1], 10)
            e = parity_err(host(u).reshape((4,) + shots[0]["shape"])[1], ru)
            say(f"  variant {info['c2r_variant']}: parity err {e:.3e}")
            assert e <= TOL_FP32
            p.close()
            q.close()
        lines = open(tmp_path / "tune.txt").read().splitlines()
        assert len(lines) == 2 and all(" | " in ln for ln in lines)
    finally:
        del os.environ["VOFL_TUNE_CACHE"]
