"""Continuous-batching server for wave solves of (1.1) on one GPU.

Requests (grid, Q field, initial data, M, step count, precision) arrive over
time. A request is admitted as soon as a slot is free and its device
footprint (the plan's workspace from vofl_plan_footprint plus the two
wavefields) fits the memory budget, in arrival order. Every admitted request
owns a HIP stream: its plan is built, its fields are uploaded from pinned
host memory, and it is advanced in chunks of TSFP2 steps (each chunk a
captured graph replay, vofl_step_graph) while other requests run on their own
streams, so that their kernels overlap on the device. Wavefields stay
resident in device memory for the whole solve, and the solve's spectral
state stays in its plan between chunks (vofl_step_begin, vofl_step_advance,
vofl_step_end), so a chunk costs only its steps; at the end (u, v) are
written out, copied back asynchronously and the stability flag is read.

One host thread makes every HIP call: graph capture on one thread must not
overlap device-wide calls (allocation, synchronisation, frees) made by
another. Host-heavy work inside vofl_plan (coefficient maps) is spread over
threads by the library itself. Finished plans are destroyed in groups, when
memory is needed or at the end, because a free waits for the device.

Each solve runs the same kernels on its own buffers with no reduction across
solves, so a result does not depend on what else is in flight.

All computation runs in libvofl's HIP kernels; this module schedules.
"""

from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import vofl as V


@dataclasses.dataclass
class Request:
    index: int
    arrival: float          # seconds after the start of the trace
    shape: tuple
    M: int
    steps: int
    precision: str          # "fp32" or "fp64"
    lo: tuple
    hi: tuple
    dt: float
    Q: np.ndarray           # quality factor on the grid (host, float64)
    u0: np.ndarray          # initial displacement (host, float64)
    v0: np.ndarray | None = None
    c0: float = 1.0
    omega0: float = 1.0

    @property
    def N(self) -> int:
        return int(np.prod(self.shape))


@dataclasses.dataclass
class Result:
    index: int
    status: str             # "ok", "unstable", "rejected" or "error"
    message: str
    precision: str
    arrival: float
    admitted: float = float("nan")
    started: float = float("nan")    # plan built and fields resident
    finished: float = float("nan")   # result downloaded
    u: np.ndarray | None = None
    v: np.ndarray | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def queue(self) -> float:
        return self.admitted - self.arrival

    @property
    def service(self) -> float:
        return self.finished - self.admitted


def _plan_kwargs(req: Request, precision: str) -> dict:
    return dict(Q=req.Q, M=req.M, dt=req.dt, precision=precision, c0=req.c0, omega0=req.omega0)


def footprint(req: Request, precision: str) -> int:
    """Device bytes a request holds while admitted: plan workspace + u, v."""
    desc, _keep = V.make_desc(req.shape, req.lo, req.hi, **_plan_kwargs(req, precision))
    elt = 4 if precision == "fp32" else 8
    return V.vofl_plan_footprint(desc) + 2 * req.N * elt


def est_step_seconds(req: Request, precision: str) -> float:
    """Rough device time of one TSFP2 step: 2M+3 real-field transforms, each
    one read and one write of the field per axis pass, at 4 TB/s, plus a
    floor of six kernel launches. Used only to size chunks and order work."""
    elt = 4 if precision == "fp32" else 8
    d = len(req.shape)
    nbytes = (2 * req.M + 3) * 2 * d * req.N * elt
    return nbytes / 4.0e12 + 6 * 4e-6


class Admission:
    """First-come first-served admission under a slot count and a byte budget.

    The head of the queue blocks the ones behind it (no overtaking), so that
    a large request is not starved by a stream of small ones. A request that
    could never fit, even on an idle device, is rejected at once.
    """

    def __init__(self, budget: int, slots: int):
        if slots < 1:
            raise ValueError("slots must be >= 1")
        self.budget = int(budget)
        self.slots = int(slots)
        self.used = 0
        self.active = 0
        self.peak_used = 0
        self.peak_active = 0

    def never_fits(self, nbytes: int) -> bool:
        return nbytes > self.budget

    def try_admit(self, nbytes: int) -> bool:
        if self.active >= self.slots or self.used + nbytes > self.budget:
            return False
        self.used += nbytes
        self.active += 1
        self.peak_used = max(self.peak_used, self.used)
        self.peak_active = max(self.peak_active, self.active)
        return True

    def release(self, nbytes: int) -> None:
        self.release_slot()
        self.release_memory(nbytes)

    def release_slot(self) -> None:
        self.active -= 1
        assert self.active >= 0

    def release_memory(self, nbytes: int) -> None:
        self.used -= nbytes
        assert self.used >= 0


class _Job:
    def __init__(self, req, precision, nbytes, slot, admitted):
        self.req = req
        self.precision = precision
        self.nbytes = nbytes
        self.slot = slot
        self.admitted = admitted
        self.started = float("nan")
        self.state = "running"
        self.plan = None
        self.u = self.v = None
        self.host = None            # pinned staging (upload, then download)
        self.dev = None             # device (u, v) pair
        self.issued = 0
        self.events = collections.deque()   # (event, estimated seconds) per queued chunk
        self.done_ev = None
        self.step_s = est_step_seconds(req, precision)
        self.chunk = 1
        self.resumable = False      # advanced through vofl_step_begin/advance/end

    def remaining_s(self) -> float:
        return (self.req.steps - self.issued) * self.step_s


class Server:
    """Request loop on one GPU (see the module docstring).

    slots        maximum number of requests admitted at once
    budget       device bytes for admitted requests (default: 90% of free memory)
    chunk        TSFP2 steps per launch; 0 issues the whole solve in one call;
                 None sizes each request's chunks to about slice_s of device time
    slice_s      target device time of one chunk (chunk=None)
    queue_s      estimated device time that may be queued over all requests;
                 every running request may still keep one chunk queued
    graphs       replay captured graphs for the chunks (vofl_step_advance with
                 use_graph; vofl_step_graph for a solve issued in one call)
    precision    force every request to this precision (None: the request's)
    keep_results download (u, v) of every request
    """

    def __init__(self, slots=16, budget=None, chunk=None, graphs=True, precision=None,
                 keep_results=True, slice_s=2e-3, queue_s=8e-3):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the server needs a HIP device")
        V.load_library()
        self.torch = torch
        self.dev = torch.device("cuda", torch.cuda.current_device())
        if budget is None:
            free, _total = torch.cuda.mem_get_info()
            budget = int(0.9 * free)
        self.admission = Admission(budget, slots)
        self.chunk = None if chunk is None else int(chunk)
        self.slice_s = float(slice_s)
        self.queue_s = float(queue_s)
        self.graphs = bool(graphs)
        self.precision = precision
        self.keep_results = keep_results
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots)]
        self._retired = []          # (plan, nbytes) of finished requests, not yet destroyed

    def _start(self, job: _Job) -> None:
        """Build the plan and enqueue the upload of (u0, v0) on the job's stream."""
        torch = self.torch
        r = job.req
        st = self.streams[job.slot]
        job.plan = V.Plan(r.shape, r.lo, r.hi, **_plan_kwargs(r, job.precision))
        dt = torch.float32 if job.precision == "fp32" else torch.float64
        v0 = np.zeros(r.shape) if r.v0 is None else r.v0
        host = torch.empty((2,) + tuple(r.shape), dtype=dt, pin_memory=True)
        host[0].copy_(torch.from_numpy(np.ascontiguousarray(r.u0, dtype=np.float64)))
        host[1].copy_(torch.from_numpy(np.ascontiguousarray(v0, dtype=np.float64)))
        with torch.cuda.stream(st):
            dev = torch.empty_like(host, device=self.dev)
            dev.copy_(host, non_blocking=True)
        job.host, job.dev = host, dev
        job.u, job.v = dev[0], dev[1]
        if job.chunk < r.steps:
            # chunked: the spectral state stays in the plan between chunks
            V.vofl_step_begin(job.plan.handle, job.u.data_ptr(), job.v.data_ptr(), st.cuda_stream)
            job.resumable = True

    def _launch(self, job: _Job, k: int) -> None:
        st = self.streams[job.slot]
        h = job.plan.handle
        if job.resumable:
            V.vofl_step_advance(h, k, 1 if self.graphs else 0, st.cuda_stream)
        elif self.graphs:
            V.vofl_step_graph(h, job.u.data_ptr(), job.v.data_ptr(), k, st.cuda_stream)
        else:
            V.vofl_step(h, job.u.data_ptr(), job.v.data_ptr(), k, st.cuda_stream)
        ev = self.torch.cuda.Event()
        ev.record(st)
        job.events.append((ev, k * job.step_s))
        job.issued += k

    def _download(self, job: _Job) -> None:
        torch = self.torch
        st = self.streams[job.slot]
        if job.resumable:
            V.vofl_step_end(job.plan.handle, job.u.data_ptr(), job.v.data_ptr(), st.cuda_stream)
        if self.keep_results:
            with torch.cuda.stream(st):
                job.host.copy_(job.dev, non_blocking=True)
        job.done_ev = torch.cuda.Event()
        job.done_ev.record(st)

    def _flush_retired(self) -> None:
        for plan, nbytes in self._retired:
            plan.close()
            self.admission.release_memory(nbytes)
        self._retired = []

    def run(self, requests, realtime=True, poll=2e-4):
        """Serve a trace; returns ({index: Result}, stats). With realtime=False
        every request is taken as arrived at time 0 (arrivals kept for the record)."""
        adm = self.admission
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.index)))
        free_slots = list(range(adm.slots))[::-1]
        jobs = {}
        results = {}
        inflight = 0.0                # estimated device seconds queued
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
        try:
            while pending or jobs:
                progressed = False
                now = clock()
                while pending and free_slots and (not realtime or pending[0].arrival <= now):
                    r = pending[0]
                    prec = self.precision or r.precision
                    nbytes = footprint(r, prec)
                    if adm.never_fits(nbytes):
                        pending.popleft()
                        results[r.index] = Result(r.index, "rejected",
                                                  f"needs {nbytes} bytes, budget {adm.budget}", prec,
                                                  r.arrival, finished=now)
                        progressed = True
                        continue
                    if not adm.try_admit(nbytes):
                        if not self._retired:
                            break
                        self._flush_retired()
                        if not adm.try_admit(nbytes):
                            break
                    pending.popleft()
                    job = _Job(r, prec, nbytes, free_slots.pop(), now)
                    if self.chunk is None:
                        job.chunk = max(1, min(256, int(round(self.slice_s / job.step_s))))
                    else:
                        job.chunk = self.chunk if self.chunk > 0 else max(r.steps, 1)
                    jobs[r.index] = job
                    try:
                        self._start(job)
                    except Exception as exc:  # plan refused or device error
                        self._retire(job, results, "error", str(exc), clock(), free_slots, jobs)
                        continue
                    job.started = clock()
                    progressed = True
                # retire finished chunks
                for job in jobs.values():
                    while job.events and job.events[0][0].query():
                        inflight -= job.events.popleft()[1]
                        progressed = True
                # issue chunks, least remaining work first, within the queue bound
                for job in sorted((j for j in jobs.values() if j.state == "running"),
                                  key=lambda j: j.remaining_s()):
                    r = job.req
                    while job.issued < r.steps and len(job.events) < 2 and (
                            not job.events or inflight + job.chunk * job.step_s <= self.queue_s):
                        k = min(job.chunk, r.steps - job.issued)
                        self._launch(job, k)
                        inflight += k * job.step_s
                        progressed = True
                    if job.issued >= r.steps:
                        self._download(job)   # queued behind the last chunk
                        job.state = "finishing"
                        progressed = True
                for idx in list(jobs):
                    job = jobs[idx]
                    if job.state == "finishing" and job.done_ev.query():
                        while job.events:  # chunks that ended since the scan above
                            inflight -= job.events.popleft()[1]
                        rc = V.vofl_sync_status(job.plan.handle, self.streams[job.slot].cuda_stream)
                        status = ("ok" if rc == V.VOFL_OK else
                                  "unstable" if rc == V.VOFL_ERR_UNSTABLE else "error")
                        res = self._retire(job, results, status, "" if rc == 0 else "non-finite values",
                                           clock(), free_slots, jobs)
                        if self.keep_results:
                            res.u = job.host[0].double().numpy().copy()
                            res.v = job.host[1].double().numpy().copy()
                        job.host = None
                        progressed = True
                if not progressed:
                    if pending and not jobs and realtime and pending[0].arrival > clock():
                        time.sleep(min(pending[0].arrival - clock(), 0.01))
                    else:
                        time.sleep(poll)
        finally:
            self.torch.cuda.synchronize()
            for job in list(jobs.values()):
                if job.plan is not None:
                    self._retired.append((job.plan, job.nbytes))
                    job.plan = None
            self._flush_retired()
        stats = summarize(results.values(), requests)
        stats.update(peak_active=adm.peak_active, peak_bytes=adm.peak_used, budget=adm.budget,
                     slots=adm.slots, chunk=self.chunk, slice_s=self.slice_s, queue_s=self.queue_s,
                     graphs=self.graphs)
        return results, stats

    def _retire(self, job, results, status, msg, now, free_slots, jobs):
        """Record the result and free the slot; the plan's memory is released
        when the plan is destroyed (_flush_retired)."""
        r = job.req
        res = Result(r.index, status, msg, job.precision, r.arrival, admitted=job.admitted,
                     started=job.started, finished=now)
        results[r.index] = res
        if job.plan is not None:
            self._retired.append((job.plan, job.nbytes))
            job.plan = None
        else:
            self.admission.release_memory(job.nbytes)
        job.u = job.v = job.dev = None
        self.admission.release_slot()
        free_slots.append(job.slot)
        del jobs[r.index]
        return res


def summarize(results, requests) -> dict:
    """Latency percentiles, queue/service split and throughput of a served trace."""
    results = list(results)
    by_index = {r.index: r for r in requests}
    ok = [r for r in results if r.status == "ok"]
    out = dict(requests=len(results), completed=len(ok),
               rejected=sum(r.status == "rejected" for r in results),
               failed=sum(r.status in ("error", "unstable") for r in results))
    if not ok:
        return out
    lat = np.array([r.latency for r in ok])
    que = np.array([r.queue for r in ok])
    svc = np.array([r.service for r in ok])
    start = min(r.arrival for r in ok)
    end = max(r.finished for r in ok)
    span = max(end - start, 1e-9)
    work = sum(by_index[r.index].N * by_index[r.index].M * by_index[r.index].steps for r in ok)
    out.update(
        p50_latency_s=float(np.percentile(lat, 50)), p99_latency_s=float(np.percentile(lat, 99)),
        mean_queue_s=float(que.mean()), mean_service_s=float(svc.mean()),
        p50_service_s=float(np.percentile(svc, 50)), p99_service_s=float(np.percentile(svc, 99)),
        makespan_s=float(span), requests_per_s=len(ok) / span,
        gpts_M_steps_per_s=work / span / 1e9,
    )
    return out


def requests_from_stream(stream, step_scale: float = 1.0, progress=None) -> list:
    """Turn request records (index, arrival, shape, M, steps, precision, seed)
    into Requests with their seeded inputs (box, dt, Q field, pulse).
    progress: optional callable(done, total) called every 20 requests."""
    from workloads import c5_request_inputs
    out = []
    stream = list(stream)
    for i, rec in enumerate(stream):
        if progress and i % 20 == 0:
            progress(i, len(stream))
        x = c5_request_inputs(rec)
        steps = max(1, int(round(rec["steps"] * step_scale)))
        out.append(Request(index=rec["index"], arrival=rec["arrival"], shape=x["shape"], M=rec["M"],
                           steps=steps, precision=rec["precision"], lo=x["lo"], hi=x["hi"],
                           dt=x["dt"], Q=x["Q"], u0=x["u0"], v0=x["v0"], c0=x["c0"],
                           omega0=x["omega0"]))
    return out
