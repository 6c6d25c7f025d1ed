"""Benchmark: TSFP2 steps of the viscoacoustic model (1.1) on a 256^3 grid,
M = 16, one MI355X. The headline line is the FP64 path (the paper's
arithmetic); the FP32 form (FP32 transforms with FP64 expansion
coefficients, multipliers, propagator and spectral state) is measured in the
same run and reported beside it with its own roofline.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--precision fp64|fp32]
                [--workload c3|c2|c4|c5|lffp|ex3]

The default workload (c3) is the 256^3 grid below. Two more measurements
print their own JSON line: c4, the batched shots (64 x 512^2 sharing one Q
and 16 x 768^2 with their own Q, M = 12, FP32) as eager batched steps and as
graph replays, against the plain FP64 path solving one shot at a time; c5,
the request server on a Poisson request stream against the same plain path
serving one request at a time.

One step is the whole hot path: the exact damped-oscillator sub-steps and
the kick, which applies both variable-order operators (2.13) (L1 to u and L2
to v, 2(M+1) inverse transforms) and transforms the kick back. "applies/s"
counts those two operator applies per step. Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import itertools
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
WORKLOAD = ("3D periodic [-16,16)^3, 256^3, M=16, two-layer Q (20 above / 100 below, tanh width 1) "
            "x (1 +- 5% seeded noise), Gaussian pulse u0, v0 = 0, c0 = omega0 = 1, dt = 1e-3")


# device-code sources of the solver's kernels and their launch shapes (host
# code, the allocation-free 1D entry point and the streaming probe do not
# change what a step kernel reads or writes)
KERNEL_SOURCES = ("fft_engine.hpp", "kernels.hpp", "launch.hpp", "launch_impl.hpp",
                  "kernels_f32.hip", "kernels_f64.hip")


def kernel_source_hash() -> str:
    """Hash of the step kernels' device-code sources, comments and blank
    lines left out (they do not change the code a profile measured)."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2311_13049_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()[:16]


def algorithmic_rw(cls: str, n: int, M: int, elt: int) -> tuple:
    """(read, write) bytes one launch of a kernel class must move at least.

    N real points, H = (n/2+1) n^2 complex half-spectrum elements, complex of
    2*elt bytes; state FP64 complex (16 B); delta FP64, A and B elt bytes.
    """
    N = n ** 3
    H = (n // 2 + 1) * n * n
    c = 2 * elt
    nterm = 2 * (M + 1)
    table = {
        # kick axis-0 pass: read 2(M+1) term slots + delta, A, B; write dv half
        "c2r0_kick": (nterm * H * c + N * (8 + 2 * elt), H * c),
        # middle-axis pass over the 2(M+1) term slots (in place)
        "mid_terms": (nterm * H * c, nterm * H * c),
        "mid_dv": (H * c, H * c),
        # last-axis pass: read dv half + state (u_hat, v_hat), write state + 2(M+1) slots
        "contig_kick": (H * c + 2 * H * 16, 2 * H * 16 + nterm * H * c),
    }
    r, w = table.get(cls, (0, 0))
    return float(r), float(w)


def algorithmic_bytes(cls: str, n: int, M: int, elt: int) -> float:
    """Bytes one launch of a kernel class must move at least (read + write once)."""
    return sum(algorithmic_rw(cls, n, M, elt))


# probe settings that reached the highest rates on this GPU (a sweep over
# grid sizes, depth and cache policy: bench.py --stream-probe)
STREAM_CONFIGS = {"read": [(512, 1), (1024, 1)], "write": [(8192, 0), (4096, 2)], "copy": [(512, 0), (8192, 1)]}


def measure_streams(torch, V, dev, nbytes=4 << 30, reps=10):
    """Best measured read, write and copy stream rates (GB/s) of the library's
    probe kernels over 4 GiB, HIP events on the current stream."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    cur = torch.cuda.current_stream().cuda_stream
    kinds = {"read": V.VOFL_PROBE_READ, "write": V.VOFL_PROBE_WRITE, "copy": V.VOFL_PROBE_COPY}
    out = {}
    for name, cfgs in STREAM_CONFIGS.items():
        best = 0.0
        for blocks, flags in cfgs:
            for _ in range(2):
                V.vofl_stream_probe(kinds[name], src.data_ptr(), dst.data_ptr(), nbytes, blocks, flags, cur)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                V.vofl_stream_probe(kinds[name], src.data_ptr(), dst.data_ptr(), nbytes, blocks, flags, cur)
            e1.record()
            torch.cuda.synchronize()
            moved = 2 * nbytes if name == "copy" else nbytes
            best = max(best, moved / (e0.elapsed_time(e1) / reps) / 1e6)
        out[f"{name}_GBps"] = best
    del src, dst
    torch.cuda.empty_cache()
    out["note"] = ("best rates of plain read, write and copy streams over 4 GiB (vofl_stream_probe); a pass "
                   "moving R read and W written bytes is set against (R + W) / (R / read + W / write)")
    return out


def mix_bound(rw, streams):
    """Rate (GB/s) of a stream of R read and W written bytes when reads and
    writes run at the measured stream rates one after the other."""
    r, w = rw
    return (r + w) / (r / streams["read_GBps"] + w / streams["write_GBps"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--M", type=int, default=16)
    ap.add_argument("--precision", default=None,
                    help="c3 (default fp64, the paper's arithmetic): the headline path, with the other precision "
                         "measured beside it; lffp, ex3 (default fp32)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="c3: skip the step-time spread and the b = 1, 4 apply rates (profiling runs)")
    ap.add_argument("--workload", default="c3", choices=("c3", "c2", "c4", "c5", "lffp", "ex3"))
    ap.add_argument("--requests", type=int, default=200, help="c5: requests in the trace")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 1 GiB five times (HBM counter calibration)")
    ap.add_argument("--stream-probe", action="store_true",
                    help="only measure the read, write and copy stream rates of the library's probe kernels")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the workload is one grid per device, and this "
              "build has no multi-GPU path (pass --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2311_13049_amd import vofl as V
    from workloads import c3_inputs

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    if args.precision is None:
        args.precision = "fp64" if args.workload == "c3" else "fp32"
    if args.calibrate_copy:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        # rate of torch's device copy kernel on the same bytes (HIP events on
        # the current stream), reported beside the counter calibration
        reps = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"copy_bytes_read_per_launch": nbytes, "copy_bytes_written_per_launch": nbytes,
                          "launches": 5 + reps, "copy_ms": ms, "copy_GBps_read_plus_write": 2 * nbytes / ms / 1e6}),
              flush=True)
        return
    if args.stream_probe:
        return stream_probe(torch, V, dev)
    if args.workload == "c4":
        return bench_c4(args, torch, V, dev)
    if args.workload == "c5":
        return bench_c5(args, torch, V, dev)
    if args.workload == "lffp":
        return bench_lffp(args, torch, V, dev)
    if args.workload == "ex3":
        return bench_ex3(args, torch, V, dev)
    if args.workload == "c2":
        return bench_c2(args, torch, V, dev)
    n, M = args.n, args.M
    c = c3_inputs(n=n)
    if args.precision not in ("fp64", "fp32"):
        raise SystemExit("--precision must be fp64 or fp32")
    other = "fp32" if args.precision == "fp64" else "fp64"
    head = _c3_measure(args, torch, V, dev, c, args.precision, extras=not args.no_extras)
    side = None if args.no_extras else _c3_measure(args, torch, V, dev, c, other, extras=True)
    N = n ** 3
    streams = None
    if not args.no_extras:
        # each kernel against a stream of its own read/write mix at the
        # measured read and write rates of this GPU
        streams = measure_streams(torch, V, dev)
        for res in (head, side):
            elt = 4 if res["precision"] == "fp32" else 8
            res["kernel_of_stream_mix_bound"] = {
                k: gbps / mix_bound(algorithmic_rw(k, n, M, elt), streams) for k, gbps in res["kernel_GBps"].items()}
            rf = res["roofline"]
            rf["stream_mix_bound_GBps"] = mix_bound(algorithmic_rw(rf["kernel"], n, M, elt), streams)
            rf["of_stream_mix_bound"] = rf["achieved"] / rf["stream_mix_bound_GBps"]

    cpu = None
    cpu_mt = None
    accuracy = None
    if not args.no_cpu:
        import oracle as O
        gamma = O.gamma_from_Q(c["Q"])
        x = c["u0"]
        t0 = time.perf_counter()
        O.mterm_apply(x, 1.0 + gamma, c["lo"], c["hi"], M)
        cpu_s = time.perf_counter() - t0
        cpu = {"value": 1.0 / cpu_s, "unit": "applies/s", "cores": 1, "kind": "oracle",
               "sample": f"one oracle apply (2.13) of L1 on the {n}^3 M={M} field, FP64 numpy "
                         f"(pocketfft, single thread): {cpu_s:.1f} s"}
        # accuracy of the benchmarked plans: L1 of the workload's initial field
        # (rounded to FP32, so that both precisions see the same values)
        # against the FP64 oracle evaluated point by point
        x_seen = c["u0"].astype(np.float32).astype(np.float64)
        rng = np.random.default_rng(np.random.SeedSequence(13049 + 3, spawn_key=(95,)))
        pts = [tuple(k // 2 for k in c["shape"])] + [tuple(int(rng.integers(k)) for k in c["shape"]) for _ in range(5)]
        t0 = time.perf_counter()
        ref = O.mterm_apply_at(x_seen, 1.0 + gamma, c["lo"], c["hi"], M, pts)
        acc_s = time.perf_counter() - t0
        accuracy = {"points": len(pts), "operator": "L1 = (-Lap)^{1+gamma(x)} by (2.13)",
                    "reference": f"FP64 oracle evaluated point by point ({acc_s:.1f} s)"}
        for prec in ("fp64", "fp32"):
            tdt = torch.float32 if prec == "fp32" else torch.float64
            plan = V.Plan(c["shape"], c["lo"], c["hi"], Q=c["Q"], M=M, dt=c["dt"], precision=prec,
                          c0=c["c0"], omega0=c["omega0"])
            lu = plan.apply(V.VOFL_OP_S1, torch.from_numpy(x_seen).to(dev, tdt)).double().cpu().numpy()
            lu = lu.reshape(c["shape"])
            plan.close()
            got = np.array([lu[j] for j in pts])
            accuracy[f"max_abs_err_over_max_abs_out_{prec}"] = float(np.max(np.abs(got - ref)) / np.max(np.abs(lu)))
        if not args.no_extras:
            workers = max(1, min(16, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))))
            O.set_fft_workers(workers)
            try:
                t0 = time.perf_counter()
                O.mterm_apply(x, 1.0 + gamma, c["lo"], c["hi"], M)
                mt_s = time.perf_counter() - t0
            finally:
                O.set_fft_workers(0)
            cpu_mt = {"value": 1.0 / mt_s, "unit": "applies/s", "cores": workers, "kind": "oracle",
                      "sample": f"the same apply with scipy.fft on {workers} worker threads: {mt_s:.1f} s"}

    c4x = c5x = None
    if not args.no_extras:
        c4x = _c4_short(args, torch, V, dev)
        c5x = _c5_short(args, torch, V, dev)

    prec = args.precision
    out = {
        "metric": f"variable-order applies/s at {n}^3, M={M} (two operator applies per TSFP2 step)",
        "value": head["applies_per_s"],
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD.replace("256^3", f"{n}^3").replace("M=16", f"M={M}"),
                   "grid": [n, n, n], "M": M, "precision": prec, "solver": "TSFP2 (3.13)"},
        "gpts_M_per_s": head["gpts_M_per_s"],
        "apply_only_b2": head["apply_only"].get("b2"),
        "apply_only": head["apply_only"],
        "step_time_spread": head["spread"],
        "resumable_chunk": head["resumable_chunk"],
        "roofline": head["roofline"],
        "whole_step": head["whole_step"],
        "kernel_ms_per_step": head["kernel_ms_per_step"],
        "kernel_GBps": head["kernel_GBps"],
        "kernel_of_stream_mix_bound": head.get("kernel_of_stream_mix_bound"),
        "streams": streams,
        "status": head["status"],
        f"{other}_path": side,
        "accuracy": accuracy,
        "cpu_baseline": cpu,
        "cpu_oracle_multicore": cpu_mt,
        "c4_batched_shots": c4x,
        "c5_served_short": c5x,
    }
    if side:
        out["fp32_speedup_over_fp64"] = (side if prec == "fp64" else head)["applies_per_s"] / \
            (head if prec == "fp64" else side)["applies_per_s"]
    print(json.dumps(out), flush=True)


def _c3_measure(args, torch, V, dev, c, prec, extras):
    """TSFP2 steps of the 256^3 workload in one precision: K timed steps in one
    vofl_step call with per-kernel-class HIP events, the dominant kernel's
    roofline, the whole step's fused bytes over its time, and (extras) the
    per-step spread and the apply-only rates of 1, 2 and 4 fields."""
    n, M = c["shape"][0], args.M
    elt = 4 if prec == "fp32" else 8
    tdt = torch.float32 if prec == "fp32" else torch.float64
    plan = V.Plan(c["shape"], c["lo"], c["hi"], Q=c["Q"], M=M, dt=c["dt"], precision=prec,
                  c0=c["c0"], omega0=c["omega0"], max_batch=4)
    u = torch.from_numpy(c["u0"]).to(dev, tdt)
    v = torch.from_numpy(c["v0"]).to(dev, tdt)

    # warmup (untimed)
    plan.step(u, v, args.warmup)
    torch.cuda.synchronize()

    # timed: exactly K steps in one call, with per-kernel-class HIP events
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step(u, v, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ktimes = plan.kernel_times()
    plan.set_timing(False)
    status = plan.sync_status()
    step_s = (t1 - t0) / args.steps
    N = n ** 3

    # dominant kernel class (largest share of device time)
    dom_name, (dom_ms, dom_launches) = max(ktimes.items(), key=lambda kv: kv[1][0])
    avg_s = dom_ms / dom_launches / 1e3
    alg = algorithmic_bytes(dom_name, n, M, elt)
    achieved = alg / avg_s / 1e9 if alg > 0 else None
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{dom_name}_256cube_M16_{prec}.json")
    if n == 256 and M == 16 and os.path.exists(tfile):
        with open(tfile) as f:
            tr = json.load(f)
        if tr.get("source_hash") == kernel_source_hash():
            traffic = tr.get("bytes_per_launch")
    # whole step: the fused kernels' algorithmic bytes per step over the step time
    step_classes = ("mid_terms", "c2r0_kick", "mid_dv", "contig_kick")
    step_bytes = sum(algorithmic_bytes(k, n, M, elt) for k in step_classes)

    spread = None
    apply_rates = {}
    chunk = None
    if extras:
        # resumable run: the cost of a 1-step chunk (vofl_step_advance(1),
        # eager and graph replay) against a steady-state step of vofl_step
        plan.begin(u, v)
        plan.advance(2)
        plan.advance(1, graph=True)  # capture outside the timing
        torch.cuda.synchronize()
        res = {}
        for mode in ("eager", "graph"):
            reps = 20
            t0 = time.perf_counter()
            for _ in range(reps):
                plan.advance(1, graph=(mode == "graph"))
            torch.cuda.synchronize()
            res[f"ms_per_1_step_chunk_{mode}"] = (time.perf_counter() - t0) / reps * 1e3
        plan.end(u, v)
        chunk = dict(res, ms_per_steady_step=step_s * 1e3,
                     ratio_eager=res["ms_per_1_step_chunk_eager"] / (step_s * 1e3),
                     ratio_graph=res["ms_per_1_step_chunk_graph"] / (step_s * 1e3))
        # spread of the per-step time: 20 chunks of 10 steps, each bracketed
        # by HIP events on the stream the plan launches on
        cs, nchunks = 10, 20
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(nchunks + 1)]
        evs[0].record()
        for i in range(nchunks):
            plan.step(u, v, cs)
            evs[i + 1].record()
        torch.cuda.synchronize()
        per_step = sorted(evs[i].elapsed_time(evs[i + 1]) / cs for i in range(nchunks))
        spread = {"chunk_steps": cs, "chunks": nchunks, "median_ms_per_step": float(np.median(per_step)),
                  "p99_ms_per_step": float(np.percentile(per_step, 99)), "min_ms_per_step": per_step[0],
                  "max_ms_per_step": per_step[-1]}
    # apply-only throughput for b = 1, 2 (the L1/L2 pair size) and 4 fields
    for b in ((1, 2, 4) if extras else (2,)):
        ub = torch.stack([u, v] * 2)[:b].contiguous()
        ob = torch.empty_like(ub)
        for _ in range(3):
            plan.apply(V.VOFL_OP_S1, ub, ob)
        torch.cuda.synchronize()
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.apply(V.VOFL_OP_S1, ub, ob)
        torch.cuda.synchronize()
        r = b / ((time.perf_counter() - t0) / reps)
        apply_rates[f"b{b}"] = {"applies_per_s": r, "gpts_M_per_s": N * M * r / 1e9}
        del ub, ob
    plan.close()
    return {
        "precision": prec,
        "applies_per_s": 2.0 / step_s,
        "ms_per_step": step_s * 1e3,
        "gpts_M_per_s": N * M * 2.0 / step_s / 1e9,
        "status": status,
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": traffic, "alg_bytes_per_launch": alg, "avg_launch_ms": avg_s * 1e3},
        "whole_step": {"alg_bytes_per_step": step_bytes, "achieved_GBps": step_bytes / step_s / 1e9,
                       "frac": step_bytes / step_s / 1e9 / HBM_PEAK_GBS,
                       "note": "sum of the fused kernels' algorithmic bytes over the step time"},
        "kernel_ms_per_step": {k: ms / args.steps for k, (ms, _) in ktimes.items()},
        "kernel_GBps": {k: algorithmic_bytes(k, n, M, elt) / (ms / nl / 1e3) / 1e9
                        for k, (ms, nl) in ktimes.items() if algorithmic_bytes(k, n, M, elt) > 0},
        "apply_only": apply_rates,
        "spread": spread,
        "resumable_chunk": chunk,
    }


def _c4_short(args, torch, V, dev):
    """Batched shots (64 x 512^2 with a shared Q + 16 x 768^2 with their own Q,
    M = 12, FP32), default kernel variants: ms per whole-batch step, eager
    vofl_step_batch, 10 timed steps after 2 warm-up steps."""
    from workloads import c4_inputs
    c = c4_inputs()
    plans, us, vs, nshots, Ntot = [], [], [], 0, 0
    for big in (False, True):
        shots = [sh for sh in c["shots"] if (sh["shape"][0] == 768) == big]
        Q = np.stack([sh["Q"] for sh in shots]) if big else shots[0]["Q"]
        plans.append(V.Plan(shots[0]["shape"], c["lo"], c["hi"], Q=Q, M=c["M"], dt=c["dt"], precision="fp32",
                            c0=c["c0"], omega0=c["omega0"], batch=len(shots), coef_per_solve=big))
        us.append(torch.from_numpy(np.stack([sh["u0"] for sh in shots])).to(dev, torch.float32))
        vs.append(torch.zeros_like(us[-1]))
        nshots += len(shots)
        Ntot += len(shots) * int(np.prod(shots[0]["shape"]))
    hs = [p.handle for p in plans]

    def run(k):
        V.vofl_step_batch(hs, [u.data_ptr() for u in us], [v.data_ptr() for v in vs], [k] * len(hs),
                          torch.cuda.current_stream().cuda_stream)
    run(2)
    torch.cuda.synchronize()
    k = 10
    t0 = time.perf_counter()
    run(k)
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / k
    status = [p.sync_status() for p in plans]
    for p in plans:
        p.close()
    return {"ms_per_batch_step": step_s * 1e3, "shot_steps_per_s": nshots / step_s,
            "gpts_M_per_s": Ntot * c["M"] * 2 / step_s / 1e9, "steps": k, "status": status,
            "workload": "64 x 512^2 (shared GRF Q) + 16 x 768^2 (own GRF Q), M=12, FP32, dt=5e-4; "
                        "eager vofl_step_batch, default kernel variants"}


def _c5_short(args, torch, V, dev, count=30, step_scale=0.1):
    """A short request stream: the first `count` requests of the Poisson trace
    (mean 200 req/s) with their step counts scaled by step_scale, served with
    continuous batching, then by the plain FP64 path one request at a time."""
    from paper_2311_13049_amd import serve as S
    from workloads import c5_requests
    reqs = S.requests_from_stream(c5_requests(count=count), step_scale=step_scale)
    _, served = S.Server(slots=16, graphs=True).run(reqs, realtime=True)
    _, plain = S.Server(slots=1, chunk=0, graphs=False, precision="fp64").run(reqs, realtime=True)
    keys = ("requests", "completed", "p50_latency_s", "p99_latency_s", "requests_per_s", "gpts_M_steps_per_s",
            "mean_queue_s", "mean_service_s")
    return {"requests": count, "step_scale": step_scale,
            "served": {k: served.get(k) for k in keys},
            "plain_fp64_single_solve": {k: plain.get(k) for k in keys},
            "workload": f"first {count} requests of the c5 Poisson stream (200 req/s), steps x {step_scale}"}


def stream_probe(torch, V, dev, nbytes=4 << 30, reps=10):
    """Read, write and copy streams of 4 GiB through the library's probe
    kernels, over several grid sizes, 4 or 16 accesses in flight per lane,
    with and without non-temporal accesses;
    HIP events on the current stream. Rates count the bytes each stream
    moves (copy: read + write)."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    cur = torch.cuda.current_stream().cuda_stream
    rows = []
    for kind, name, moved in ((V.VOFL_PROBE_READ, "read", nbytes), (V.VOFL_PROBE_WRITE, "write", nbytes),
                              (V.VOFL_PROBE_COPY, "copy", 2 * nbytes)):
        for blocks, nt, deep in itertools.product((512, 1024, 2048, 4096, 8192), (False, True), (False, True)):
            flags = (V.VOFL_PROBE_NONTEMPORAL if nt else 0) | (V.VOFL_PROBE_DEEP if deep else 0)
            def run():
                V.vofl_stream_probe(kind, src.data_ptr(), dst.data_ptr(), nbytes, blocks, flags, cur)
            run()
            run()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                run()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            rows.append({"stream": name, "blocks": blocks, "nontemporal": nt, "deep": deep, "ms": ms,
                         "GBps": moved / ms / 1e6})
    assert torch.equal(dst, src), "copy stream result differs from its source"
    best = {n: max((r for r in rows if r["stream"] == n), key=lambda r: r["GBps"]) for n in ("read", "write", "copy")}
    print(json.dumps({"stream_probe_bytes": nbytes, "reps": reps, "best": best, "all": rows}), flush=True)


def _fork_join(torch, streams, fns):
    """Run fns[i] on streams[i] after the current stream's work; join back."""
    cur = torch.cuda.current_stream()
    start = torch.cuda.Event()
    start.record(cur)
    for st, fn in zip(streams, fns):
        st.wait_event(start)
        with torch.cuda.stream(st):
            fn(st.cuda_stream)
    for st in streams:
        ev = torch.cuda.Event()
        ev.record(st)
        cur.wait_event(ev)


def bench_c4(args, torch, V, dev):
    """Batched shots: whole-batch steps/s, eager and graph, vs the plain FP64 path."""
    from workloads import c4_inputs
    c = c4_inputs()
    steps, warm = args.steps, args.warmup
    groups = []
    for big in (False, True):
        shots = [s for s in c["shots"] if (s["shape"][0] == 768) == big]
        Q = np.stack([s["Q"] for s in shots]) if big else shots[0]["Q"]
        t0 = time.perf_counter()
        plan = V.Plan(shots[0]["shape"], c["lo"], c["hi"], Q=Q, M=c["M"], dt=c["dt"], precision="fp32",
                      c0=c["c0"], omega0=c["omega0"], batch=len(shots), coef_per_solve=big, tune_steps=5)
        tplan = time.perf_counter() - t0
        u = torch.from_numpy(np.stack([s["u0"] for s in shots])).to(dev, torch.float32)
        v = torch.zeros_like(u)
        groups.append(dict(shots=shots, plan=plan, u=u, v=v, plan_s=tplan, info=plan.info()))
    streams = [torch.cuda.Stream() for _ in groups]
    hs = [g["plan"].handle for g in groups]

    def eager(k):
        V.vofl_step_batch(hs, [g["u"].data_ptr() for g in groups], [g["v"].data_ptr() for g in groups],
                          [k] * len(groups), torch.cuda.current_stream().cuda_stream)

    def graph(k):
        _fork_join(torch, streams, [
            (lambda s, g=g: V.vofl_step_graph(g["plan"].handle, g["u"].data_ptr(), g["v"].data_ptr(), k, s))
            for g in groups])

    timings = {}
    for name, fn in (("eager_batch", eager), ("graph_batch", graph)):
        fn(warm)
        if name == "graph_batch":
            fn(steps)  # capture outside the timed region
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(steps)
        torch.cuda.synchronize()
        timings[name] = time.perf_counter() - t0
    # the whole batched step sequence (both groups, forked onto the plans'
    # streams and joined) captured as one graph and replayed
    one_graph_error = None
    try:
        cap = torch.cuda.Stream()
        cg = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(cg, stream=cap):
            eager(steps)
        cg.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cg.replay()
        torch.cuda.synchronize()
        timings["one_graph_batch"] = time.perf_counter() - t0
    except Exception as exc:  # capture refused by the runtime: report it
        one_graph_error = str(exc)[:300]
    # each group alone on the current stream: eager steps against graph
    # replays of the same steps (the graph's own cost per launch)
    per_group = {}
    cur = torch.cuda.current_stream().cuda_stream
    for g in groups:
        h, up, vp = g["plan"].handle, g["u"].data_ptr(), g["v"].data_ptr()
        res = {}
        for mode in ("eager", "graph"):
            fn = (lambda k: V.vofl_step(h, up, vp, k, cur)) if mode == "eager" else \
                 (lambda k: V.vofl_step_graph(h, up, vp, k, cur))
            fn(steps)  # warm (and capture)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn(steps)
            torch.cuda.synchronize()
            res[f"{mode}_ms_per_step"] = (time.perf_counter() - t0) / steps * 1e3
        per_group[f"{len(g['shots'])} x {g['shots'][0]['shape'][0]}^2"] = res
    status = [g["plan"].sync_status() for g in groups]
    nshots = sum(len(g["shots"]) for g in groups)
    Ntot = sum(len(g["shots"]) * int(np.prod(g["shots"][0]["shape"])) for g in groups)
    # algorithmic bytes of a step of the fused kernels (2D: the kick's axis-0
    # pass and the last-axis pass), per shot with H = (n/2+1) n half-spectrum
    # elements, FP32 complex c = 8 B: c2r0_kick 2(M+1) H c + N (8 + 2*4) + H c,
    # contig_kick H c + 4*16 H + 2(M+1) H c
    bstep = 0
    for g in groups:
        n0 = g["shots"][0]["shape"][0]
        Ns, Hs, cb, nterm = n0 * n0, (n0 // 2 + 1) * n0, 8, 2 * (c["M"] + 1)
        bstep += len(g["shots"]) * (nterm * Hs * cb + Ns * 16 + Hs * cb + Hs * cb + 64 * Hs + nterm * Hs * cb)
    # the unfused model: (2M+3) real-field transforms, one read and
    # one write of the field per axis pass (an effective rate, not HBM bytes)
    bstep_model = (2 * c["M"] + 3) * 2 * 2 * Ntot * 4

    # plain FP64 single-solve path: one shot per plan, eager vofl_step,
    # one shot at a time; timed on two shots of each size, scaled to the batch
    plain = {}
    for g in groups:
        sh = g["shots"][0]
        p = V.Plan(sh["shape"], c["lo"], c["hi"], Q=sh["Q"], M=c["M"], dt=c["dt"], precision="fp64",
                   c0=c["c0"], omega0=c["omega0"])
        ts = []
        for s_ in g["shots"][:2]:
            u = torch.from_numpy(s_["u0"]).to(dev, torch.float64)
            v = torch.zeros_like(u)
            p.step(u, v, warm)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p.step(u, v, steps)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) / steps)
        plain[f"{sh['shape'][0]}^2"] = float(np.mean(ts))
        p.close()
    plain_step = sum(len(g["shots"]) * plain[f"{g['shots'][0]['shape'][0]}^2"] for g in groups)
    best = min(timings, key=timings.get)
    step_s = timings[best] / steps
    out = {
        "metric": "batched shot-steps/s (64 x 512^2 shared Q + 16 x 768^2 own Q, M=12)",
        "value": nshots / step_s, "unit": "shot-steps/s", "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": step_s * 1e3, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "mode": best,
        "config": {"workload": "c4 batched shots: 64 x 512^2 on [-32,32)^2 sharing one GRF Q + 16 x 768^2 "
                               "with their own GRF Q, M=12, FP32, dt=5e-4"},
        "ms_per_step_by_mode": {k: t / steps * 1e3 for k, t in timings.items()},
        "per_group_alone": per_group,
        "one_graph_error": one_graph_error,
        "applies_per_s": 2 * nshots / step_s,
        "gpts_M_per_s": Ntot * c["M"] * 2 / step_s / 1e9,
        "roofline": {"bound": "hbm", "achieved": bstep / step_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": bstep / step_s / 1e9 / HBM_PEAK_GBS, "alg_bytes_per_step": bstep,
                     "note": "fused kernels' algorithmic bytes of a whole batch step over its time"},
        "effective_rate_unfused_model": {"bytes_per_step": bstep_model, "GBps": bstep_model / step_s / 1e9,
                                         "note": "the (2M+3)-transform unfused model; not HBM traffic"},
        "plain_fp64_single_solve": {"ms_per_step_whole_batch": plain_step * 1e3,
                                    "ms_per_shot_step": {k: t * 1e3 for k, t in plain.items()},
                                    "speedup_of_batched": plain_step / step_s,
                                    "sample": "2 shots of each size, solved one at a time, scaled to 64 + 16"},
        "plan_build_s": [g["plan_s"] for g in groups],
        "tuned_variants": [{"c2r": g["info"]["c2r_variant"], "mid": g["info"]["mid_variant"],
                            "last_axis_schedule": g["info"]["contig_variant"]} for g in groups],
        "status": status,
    }
    print(json.dumps(out), flush=True)


def bench_lffp(args, torch, V, dev):
    """Leap-frog scheme (3.4) for the generic model (1.5) on 256^3, M = 16, FP32:
    one operator apply and the update per step."""
    from workloads import gaussian_pulse, mesh
    n, M = args.n, args.M
    shape, lo, hi = (n, n, n), (-16.0,) * 3, (16.0,) * 3
    X = mesh(shape, lo, hi)
    s_field = 1.0 + 0.3 * np.sin(np.pi * X[0] / 8.0) * np.cos(np.pi * X[1] / 8.0)
    phi = gaussian_pulse(shape, lo, hi, (0.0, 0.0, 0.0))
    del X
    tdt = torch.float32 if args.precision == "fp32" else torch.float64
    plan = V.Plan(shape, lo, hi, model="generic", s=s_field, kappa=1.0, lam=1.0, M=M, dt=1e-3,
                  precision=args.precision)
    up, u = plan.lffp_start(torch.from_numpy(phi).to(dev, tdt), torch.zeros(shape, device=dev, dtype=tdt))
    plan.lffp_step(up, u, args.warmup)
    torch.cuda.synchronize()
    plan.set_timing(True)
    t0 = time.perf_counter()
    plan.lffp_step(up, u, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = plan.kernel_times()
    plan.set_timing(False)
    step_s = (t1 - t0) / args.steps
    elt = 4 if args.precision == "fp32" else 8
    H = (n // 2 + 1) * n * n
    # algorithmic bytes of the axis-0 pass with the update: M+1 term slots,
    # delta, and the FP64 state read and written
    alg_c2r = (M + 1) * H * 2 * elt + n ** 3 * 8 + 4 * n ** 3 * 8
    c2r_ms, c2r_n = kt.get("c2r0_lffp", (0.0, 1))
    out = {
        "metric": "leap-frog (3.4) steps/s, generic model (1.5), 256^3, M=16",
        "value": 1.0 / step_s, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": step_s * 1e3, "higher_is_better": True, "data": "synthetic",
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "config": {"workload": f"LFFP on {n}^3 [-16,16)^3, s = 1 + 0.3 sin(pi x/8) cos(pi y/8), kappa = 1, "
                               f"f = u^3, M = {M}, dt = 1e-3"},
        "applies_per_s": 1.0 / step_s,
        "gpts_M_per_s": n ** 3 * M / step_s / 1e9,
        "kernel_ms_per_step": {k: ms / args.steps for k, (ms, _) in kt.items()},
        "roofline_c2r0_lffp": {"bound": "hbm", "achieved": alg_c2r / (c2r_ms / c2r_n / 1e3) / 1e9 if c2r_ms else None,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "alg_bytes_per_launch": alg_c2r},
        "status": plan.sync_status(),
    }
    print(json.dumps(out), flush=True)


def bench_c2(args, torch, V, dev):
    """2D workload: 1024^2 on [-32,32)^2, GRF Q in [10, 200], M = 16, FP64
    (the plain path the workload names), dt = 5e-4; TSFP2 steps and the
    apply of two fields; the FP32 form of the same run beside it."""
    from workloads import c2_inputs
    c = c2_inputs()
    n, M = c["shape"][0], c["M"]

    def run(prec):
        tdt = torch.float64 if prec == "fp64" else torch.float32
        plan = V.Plan(c["shape"], c["lo"], c["hi"], Q=c["Q"], M=M, dt=c["dt"], precision=prec, c0=c["c0"],
                      omega0=c["omega0"], max_batch=2)
        u = torch.from_numpy(c["u0"]).to(dev, tdt)
        v = torch.from_numpy(c["v0"]).to(dev, tdt)
        plan.step(u, v, args.warmup)
        torch.cuda.synchronize()
        plan.set_timing(True)
        t0 = time.perf_counter()
        plan.step(u, v, args.steps)
        torch.cuda.synchronize()
        step_s = (time.perf_counter() - t0) / args.steps
        kt = plan.kernel_times()
        plan.set_timing(False)
        status = plan.sync_status()
        ub = torch.stack([u, v]).contiguous()
        ob = torch.empty_like(ub)
        plan.apply(V.VOFL_OP_S1, ub, ob)
        torch.cuda.synchronize()
        reps = 50
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.apply(V.VOFL_OP_S1, ub, ob)
        torch.cuda.synchronize()
        return step_s, kt, (time.perf_counter() - t0) / reps, status

    step_s, kt, apply_s, status = run("fp64")
    step32, _, apply32, status32 = run("fp32")
    elt = 8
    N, H, cb = n * n, (n // 2 + 1) * n, 2 * elt
    nterm = 2 * (M + 1)
    # 2D: no middle axis; the kick's axis-0 pass and last-axis pass as in 3D
    alg = {"c2r0_kick": nterm * H * cb + N * (8 + 2 * elt) + H * cb,
           "contig_kick": H * cb + 4 * H * 16 + nterm * H * cb}
    dom = max((k for k in alg if k in kt), key=lambda k: kt[k][0])
    avg = kt[dom][0] / kt[dom][1] / 1e3
    out = {
        "metric": "variable-order applies/s at 1024^2, M=16, FP64 (two operator applies per TSFP2 step)",
        "value": 2.0 / step_s, "unit": "applies/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": step_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2D periodic [-32,32)^2, 1024^2, M=16, GRF Q in [10,200] (corr. length 4), "
                               "Gaussian pulse u0, v0 = 0, c0 = omega0 = 1, dt = 5e-4", "grid": [n, n], "M": M,
                   "precision": "fp64"},
        "gpts_M_per_s": N * M * 2.0 / step_s / 1e9,
        "apply_only_b2": {"applies_per_s": 2.0 / apply_s, "ms_per_apply_of_two": apply_s * 1e3},
        "kernel_ms_per_step": {k: ms / args.steps for k, (ms, _) in kt.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": alg[dom] / avg / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": alg[dom] / avg / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": alg[dom], "avg_launch_ms": avg * 1e3},
        "fp32_form": {"ms_per_step": step32 * 1e3, "applies_per_s": 2.0 / step32,
                      "apply_only_b2_applies_per_s": 2.0 / apply32, "status": status32},
        "status": status,
    }
    print(json.dumps(out), flush=True)


def bench_ex3(args, torch, V, dev):
    """Example 3 (Section 4): leap-frog for (1.1) in the two-layer attenuating
    medium at the paper's mesh (1000 x 1000 on [0,2)^2, dt = 1e-4), M = 8."""
    from workloads import ex3_inputs
    ex = ex3_inputs(1000, case=0)
    n, M, prec = ex["shape"][0], ex["M"], args.precision
    N = n * n
    tdt = torch.float32 if prec == "fp32" else torch.float64
    plan = V.Plan(ex["shape"], ex["lo"], ex["hi"], gamma=ex["gamma"], c0_field=ex["c0"], omega0=ex["omega0"],
                  M=M, dt=ex["dt"], precision=prec)
    up, u = plan.lffp_start(torch.from_numpy(ex["phi"]).to(dev, tdt), torch.from_numpy(ex["psi"]).to(dev, tdt))
    plan.lffp_step(up, u, args.warmup)
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.lffp_step(up, u, 3)  # per-kernel times from events around each launch
    torch.cuda.synchronize()
    kt = plan.kernel_times()
    plan.set_timing(False)
    t0 = time.perf_counter()
    plan.lffp_step(up, u, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    status = plan.sync_status()
    step_s = (t1 - t0) / args.steps
    # both media of Example 3 as one batch of two solves (own gamma, same c0)
    ex1 = ex3_inputs(1000, case=1)
    del plan, up, u
    pb = V.Plan(ex["shape"], ex["lo"], ex["hi"], gamma=np.stack([ex["gamma"], ex1["gamma"]]),
                c0_field=np.stack([ex["c0"], ex1["c0"]]), omega0=ex["omega0"], M=M, dt=ex["dt"], precision=prec,
                batch=2, coef_per_solve=True)
    phi2 = torch.from_numpy(np.stack([ex["phi"], ex1["phi"]])).to(dev, tdt)
    ub_prev, ub = pb.lffp_start(phi2, torch.zeros_like(phi2))
    pb.lffp_step(ub_prev, ub, args.warmup)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pb.lffp_step(ub_prev, ub, args.steps)
    torch.cuda.synchronize()
    batch_step_s = (time.perf_counter() - t2) / args.steps
    batch_status = pb.sync_status()
    del pb, ub_prev, ub, phi2
    elt = 4 if prec == "fp32" else 8
    H = (n // 2 + 1) * n
    # algorithmic bytes per step (read + write once): two FP64 forward axis-0
    # passes (u; w formed from u^n and u^{n-1} while loading), the last-axis
    # pass (2 FP64 half spectra in, 2(M+1) term slots out) and the axis-0
    # update pass (2(M+1) slots, delta, A, B, FP64 state in and out)
    alg = {"r2c0": 24 * N + 2 * 16 * H, "contig_lffp": 2 * 16 * H + 2 * (M + 1) * H * 2 * elt,
           "c2r0_lffp": 2 * (M + 1) * H * 2 * elt + 8 * N + 2 * elt * N + 32 * N}
    per_step = {k: ms / 3 for k, (ms, _) in kt.items()}
    c2r_ms = kt["c2r0_lffp"][0] / kt["c2r0_lffp"][1] if "c2r0_lffp" in kt else None  # per launch
    cpu = None
    if not args.no_cpu:
        import oracle as O
        O.set_fft_workers(0)
        t2 = time.perf_counter()
        O.lffp_seismic(ex["phi"], ex["psi"], ex["gamma"], ex["c0"], ex["omega0"], ex["lo"], ex["hi"], M,
                       ex["dt"], 2)
        cpu_s = (time.perf_counter() - t2) / 2
        cpu = {"value": 1.0 / cpu_s, "unit": "steps/s", "cores": 1, "kind": "oracle",
               "sample": "start + 1 leap-frog step of the same 1000^2 Example 3 problem, FP64 numpy, one thread"}
    out = {
        "metric": "leap-frog steps/s, Example 3 two-layer medium (1.1), 1000^2, M=8",
        "value": 1.0 / step_s, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": step_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": "Example 3 on [0,2)^2, 1000 x 1000 (h = 0.002), gamma = 0.0065 + 0.0035 tanh(100(y-1)), "
                               "c0 = 11/18 (y > 1) / 1, omega0 = 1, Ricker start nu0 = 25 at (1, 0.85), "
                               "dt = 1e-4, M = 8", "grid": [n, n], "M": M, "precision": prec},
        "applies_per_s": 2.0 / step_s,
        "kernel_ms_per_step": per_step,
        "alg_bytes_per_step": alg,
        "roofline": {"bound": "hbm", "kernel": "c2r0_lffp",
                     "achieved": alg["c2r0_lffp"] / (c2r_ms / 1e3) / 1e9 if c2r_ms else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg["c2r0_lffp"] / (c2r_ms / 1e3) / 1e9 / HBM_PEAK_GBS if c2r_ms else None,
                     "traffic": None, "alg_bytes_per_launch": alg["c2r0_lffp"]},
        "status": status,
        "batch2_both_media": {"solve_steps_per_s": 2.0 / batch_step_s, "ms_per_batch_step": batch_step_s * 1e3,
                              "status": batch_status},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_c5(args, torch, V, dev):
    """Request server on a Poisson trace vs the plain FP64 path, one request at a time."""
    from paper_2311_13049_amd import serve as S
    from workloads import c5_requests
    t0 = time.perf_counter()
    reqs = S.requests_from_stream(c5_requests(count=args.requests),
                                  progress=lambda i, n: print(f"c5 inputs {i}/{n}", file=sys.stderr, flush=True))
    gen_s = time.perf_counter() - t0
    print(json.dumps({"c5_inputs_ready_s": gen_s, "requests": len(reqs)}), flush=True)
    print("c5 serving the trace", file=sys.stderr, flush=True)
    served, st_served = S.Server(slots=16, graphs=True).run(reqs, realtime=True)
    print(json.dumps({"served": st_served}), flush=True)
    plain, st_plain = S.Server(slots=1, chunk=0, graphs=False, precision="fp64").run(reqs, realtime=True)
    print(json.dumps({"plain_fp64": st_plain}), flush=True)
    print("c5 plain path, each request in its own precision", file=sys.stderr, flush=True)
    _, st_plain_mix = S.Server(slots=1, chunk=0, graphs=False).run(reqs, realtime=True)
    print(json.dumps({"plain_mixed": st_plain_mix}), flush=True)
    print("c5 plain path, all requests in FP32", file=sys.stderr, flush=True)
    _, st_plain32 = S.Server(slots=1, chunk=0, graphs=False, precision="fp32").run(reqs, realtime=True)
    span = max(r.arrival for r in reqs) - min(r.arrival for r in reqs)
    demand = sum(r.service for r in plain.values() if r.status == "ok")
    work = sum(r.N * r.M * r.steps for r in reqs)
    out = {
        "metric": "served requests/s and p50/p99 latency (Poisson stream, mean 200 req/s)",
        "value": st_served.get("requests_per_s"), "unit": "requests/s", "n_gpus": 1,
        "higher_is_better": True, "data": "synthetic", "dtype": "mixed f32/f64 (per request)",
        "config": {"workload": f"c5 request stream: {len(reqs)} requests, grids 128^2..1024^2 and 128^3, "
                               "256^3, M in {8,16}, steps U{100..2000}, FP32 or FP64, GRF Q"},
        "served": st_served,
        "plain_fp64_single_solve": st_plain,
        "plain_single_solve_request_precision": st_plain_mix,
        "plain_fp32_single_solve": st_plain32,
        "note": "served and plain_single_solve_request_precision run each request in its own precision "
                "(half FP32, half FP64); the two other plain runs force one precision on every request",
        "offered_load": demand / max(span, 1e-9),
        "offered_load_note": "GPU-seconds of the plain path per second of trace",
        "work_gpts_M_steps": work / 1e9,
        "speedup_requests_per_s": (st_served.get("requests_per_s") or 0) / max(st_plain.get("requests_per_s") or 1e-30, 1e-30),
        "speedup_over_plain_same_precisions": (st_served.get("requests_per_s") or 0) /
                                              max(st_plain_mix.get("requests_per_s") or 1e-30, 1e-30),
        "p99_latency_ratio_plain_over_served": (st_plain.get("p99_latency_s") or 0) / max(st_served.get("p99_latency_s") or 1e-30, 1e-30),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
