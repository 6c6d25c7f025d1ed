"""Continuous-batching server for wave solves of (1.1) on one GPU.

Requests (grid, Q field, initial data, M, step count, precision) arrive over
time. A request is admitted as soon as a slot is free and its device
footprint (the plan's workspace from vofl_plan_footprint plus the two
wavefields) fits the memory budget, in arrival order. Every admitted request
owns a HIP stream: its plan is built and its fields are uploaded by a host
worker thread, then the main loop advances it in chunks of TSFP2 steps (each
chunk a captured graph replay, vofl_step_graph) while other requests run on
their own streams, so that their kernels overlap on the device. Wavefields
stay resident in device memory for the whole solve. When the last chunk is
done a worker reads the stability flag, downloads (u, v), destroys the plan
and returns slot and memory to the admission queue.

Each solve runs the same kernels on its own buffers with no reduction across
solves, so a result does not depend on what else is in flight.

All computation runs in libvofl's HIP kernels; this module schedules.
"""

from __future__ import annotations

import collections
import concurrent.futures as cf
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
        self.used -= nbytes
        self.active -= 1
        assert self.used >= 0 and self.active >= 0


class _Job:
    def __init__(self, req, precision, nbytes, slot, admitted):
        self.req = req
        self.precision = precision
        self.nbytes = nbytes
        self.slot = slot
        self.admitted = admitted
        self.started = float("nan")
        self.state = "preparing"
        self.future = None
        self.plan = None
        self.u = None
        self.v = None
        self.issued = 0
        self.events = collections.deque()


class Server:
    """Request loop on one GPU (see the module docstring).

    slots        maximum number of requests admitted at once
    budget       device bytes for admitted requests (default: 90% of free memory)
    chunk        TSFP2 steps per launch; 0 issues the whole solve in one call
    graphs       replay captured graphs for the chunks (vofl_step_graph)
    precision    force every request to this precision (None: the request's)
    keep_results download (u, v) of every request
    """

    def __init__(self, slots=16, budget=None, chunk=64, graphs=True, precision=None,
                 keep_results=True, workers=4):
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
        self.chunk = int(chunk)
        self.graphs = bool(graphs)
        self.precision = precision
        self.keep_results = keep_results
        self.workers = int(workers)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots)]

    # -- worker-thread steps ------------------------------------------------
    def _prepare(self, job: _Job) -> None:
        torch = self.torch
        r = job.req
        torch.cuda.set_device(self.dev)
        st = self.streams[job.slot]
        with torch.cuda.stream(st):
            job.plan = V.Plan(r.shape, r.lo, r.hi, **_plan_kwargs(r, job.precision))
            dt = torch.float32 if job.precision == "fp32" else torch.float64
            job.u = torch.from_numpy(np.ascontiguousarray(r.u0, dtype=np.float64)).to(self.dev, dt)
            v0 = np.zeros(r.shape) if r.v0 is None else r.v0
            job.v = torch.from_numpy(np.ascontiguousarray(v0, dtype=np.float64)).to(self.dev, dt)
        st.synchronize()

    def _finish(self, job: _Job):
        torch = self.torch
        torch.cuda.set_device(self.dev)
        st = self.streams[job.slot]
        rc = V.vofl_sync_status(job.plan.handle, st.cuda_stream)
        u = v = None
        if self.keep_results:
            with torch.cuda.stream(st):
                u = job.u.double().cpu().numpy().reshape(job.req.shape)
                v = job.v.double().cpu().numpy().reshape(job.req.shape)
        done = time.perf_counter() - self._t0  # the result is with the client
        job.plan.close()
        job.plan = job.u = job.v = None
        st.synchronize()
        return rc, u, v, done

    # -- main loop ----------------------------------------------------------
    def _launch(self, job: _Job, k: int) -> None:
        st = self.streams[job.slot]
        h = job.plan.handle
        if self.graphs:
            V.vofl_step_graph(h, job.u.data_ptr(), job.v.data_ptr(), k, st.cuda_stream)
        else:
            V.vofl_step(h, job.u.data_ptr(), job.v.data_ptr(), k, st.cuda_stream)
        ev = self.torch.cuda.Event()
        ev.record(st)
        job.events.append(ev)
        job.issued += k

    def run(self, requests, realtime=True, poll=2e-4):
        """Serve a trace; returns ({index: Result}, stats). With realtime=False
        every request is taken as arrived at time 0 (arrivals kept for the record)."""
        adm = self.admission
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.index)))
        free_slots = list(range(adm.slots))[::-1]
        jobs = {}
        results = {}
        self._t0 = t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
        with cf.ThreadPoolExecutor(max_workers=self.workers) as pool:
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
                        break
                    pending.popleft()
                    job = _Job(r, prec, nbytes, free_slots.pop(), now)
                    job.future = pool.submit(self._prepare, job)
                    jobs[r.index] = job
                    progressed = True
                for idx in list(jobs):
                    job = jobs[idx]
                    r = job.req
                    if job.state == "preparing" and job.future.done():
                        progressed = True
                        try:
                            job.future.result()
                        except Exception as exc:  # plan refused or device error
                            self._retire(job, results, "error", str(exc), clock(), free_slots, jobs)
                            continue
                        job.state = "running"
                        job.started = clock()
                    if job.state == "running":
                        while job.events and job.events[0].query():
                            job.events.popleft()
                            progressed = True
                        step = self.chunk if self.chunk > 0 else r.steps
                        while job.issued < r.steps and len(job.events) < 2:
                            self._launch(job, min(step, r.steps - job.issued))
                            progressed = True
                        if job.issued >= r.steps and not job.events:
                            job.state = "finishing"
                            job.future = pool.submit(self._finish, job)
                            progressed = True
                    if job.state == "finishing" and job.future.done():
                        progressed = True
                        try:
                            rc, u, v, done = job.future.result()
                        except Exception as exc:
                            self._retire(job, results, "error", str(exc), clock(), free_slots, jobs)
                            continue
                        status = "ok" if rc == V.VOFL_OK else ("unstable" if rc == V.VOFL_ERR_UNSTABLE else "error")
                        res = self._retire(job, results, status, "" if rc == 0 else "non-finite values",
                                           done, free_slots, jobs)
                        res.u, res.v = u, v
                if not progressed:
                    if pending and not jobs and realtime and pending[0].arrival > clock():
                        time.sleep(min(pending[0].arrival - clock(), 0.01))
                    else:
                        time.sleep(poll)
        stats = summarize(results.values(), requests)
        stats.update(peak_active=adm.peak_active, peak_bytes=adm.peak_used, budget=adm.budget,
                     slots=adm.slots, chunk=self.chunk, graphs=self.graphs)
        return results, stats

    def _retire(self, job, results, status, msg, now, free_slots, jobs):
        r = job.req
        if job.plan is not None:
            job.plan.close()
            job.plan = job.u = job.v = None
        res = Result(r.index, status, msg, job.precision, r.arrival, admitted=job.admitted,
                     started=job.started, finished=now)
        results[r.index] = res
        self.admission.release(job.nbytes)
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


def requests_from_stream(stream, step_scale: float = 1.0) -> list:
    """Turn request records (index, arrival, shape, M, steps, precision, seed)
    into Requests with their seeded inputs (box, dt, Q field, pulse)."""
    from workloads import c5_request_inputs
    out = []
    for rec in stream:
        x = c5_request_inputs(rec)
        steps = max(1, int(round(rec["steps"] * step_scale)))
        out.append(Request(index=rec["index"], arrival=rec["arrival"], shape=x["shape"], M=rec["M"],
                           steps=steps, precision=rec["precision"], lo=x["lo"], hi=x["hi"],
                           dt=x["dt"], Q=x["Q"], u0=x["u0"], v0=x["v0"], c0=x["c0"],
                           omega0=x["omega0"]))
    return out
