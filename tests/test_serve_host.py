"""Host logic of the request server (no device): admission order, budget and
slot limits, and the latency summary."""

import types

import numpy as np

from paper_2311_13049_amd.serve import Admission, Result, summarize


def test_admission_budget_and_slots():
    a = Admission(budget=100, slots=2)
    assert a.try_admit(60)
    assert not a.try_admit(50)          # over budget
    assert a.try_admit(40)
    assert not a.try_admit(1)           # no slot left
    a.release(60)
    assert a.try_admit(10)
    assert a.peak_used == 100 and a.peak_active == 2
    assert a.never_fits(101) and not a.never_fits(100)


def test_admission_rejects_bad_slot_count():
    try:
        Admission(budget=1, slots=0)
    except ValueError:
        return
    raise AssertionError("slots=0 accepted")


def test_summary_percentiles_and_split():
    reqs = [types.SimpleNamespace(index=i, N=100, M=8, steps=10) for i in range(4)]
    res = [Result(i, "ok", "", "fp32", arrival=0.1 * i, admitted=0.1 * i + 0.05, started=0.1 * i + 0.06,
                  finished=1.0 + i) for i in range(4)]
    res.append(Result(9, "rejected", "too big", "fp64", arrival=0.0, finished=0.0))
    s = summarize(res, reqs + [types.SimpleNamespace(index=9, N=1, M=1, steps=1)])
    lat = np.array([1.0 + i - 0.1 * i for i in range(4)])
    assert s["completed"] == 4 and s["rejected"] == 1
    assert abs(s["p50_latency_s"] - np.percentile(lat, 50)) < 1e-12
    assert abs(s["mean_queue_s"] - 0.05) < 1e-12
    assert abs(s["makespan_s"] - 4.0) < 1e-12
    assert abs(s["gpts_M_steps_per_s"] - 4 * 100 * 8 * 10 / 4.0 / 1e9) < 1e-18
