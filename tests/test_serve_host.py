"""Scheduling core of the serving loop, on the CPU with a stand-in executor:
memory admission, first-fit order, slot concurrency, dependencies of
queries on builds, and failures that stay with their request."""
import threading
import time

import pytest

from paper_2503_18397_amd.serve import Request, Scheduler


class _Keys:
    def __init__(self, n):
        self.n = n

    def numel(self):
        return self.n


def _run(reqs, slots, budget, fail=(), resident=0.0):
    live = {"run": 0, "peak": 0, "mem": 0, "mem_peak": 0}
    lock = threading.Lock()
    order = []

    def footprint(r):
        return (r.keys.numel(), int(r.keys.numel() * resident)) if r.kind != "query" else (10, 0)

    def execute(slot, r, target):
        with lock:
            live["run"] += 1
            live["peak"] = max(live["peak"], live["run"])
            order.append(r.rid)
        time.sleep(0.002 + r.keys.numel() * 1e-6)
        with lock:
            live["run"] -= 1
        if r.rid in fail:
            raise RuntimeError("build failed")
        if r.kind == "query":
            assert target is not None and target.rid == r.target
        return r.rid

    s = Scheduler(slots, budget, execute, footprint)
    for r in reqs:
        s.submit(r)
    st = s.drain(timeout=30)
    s.close()
    return st, live, order


def test_admission_respects_the_budget_and_runs_everything():
    reqs = [Request(i, "vfunc", _Keys(1000 * (1 + i % 7))) for i in range(40)]
    st, live, _ = _run(reqs, slots=4, budget=12000)
    assert len(st.completed) == 40 and st.summary()["errors"] == 0
    assert st.peak_bytes <= 12000
    assert 1 < live["peak"] <= 4


def test_first_fit_lets_small_requests_pass_a_blocked_large_one():
    reqs = [Request(0, "vfunc", _Keys(6000)), Request(1, "vfunc", _Keys(6000)),
            Request(2, "vfunc", _Keys(500))]
    # budget for the first build and the small one, not for both large ones
    st, _, order = _run(reqs, slots=4, budget=7000)
    assert order.index(2) < order.index(1)
    assert st.summary()["errors"] == 0


def test_queries_wait_for_their_build_and_fail_with_it():
    reqs = [Request(0, "vfilter", _Keys(20000)), Request(1, "query", _Keys(5), target=0),
            Request(2, "vfunc", _Keys(100)), Request(3, "query", _Keys(5), target=2)]
    st, _, order = _run(reqs, slots=3, budget=10 ** 6, fail={2}, resident=0.5)
    assert order.index(0) < order.index(1)
    err = {r.rid: r.error for r in st.completed}
    assert err[0] is None and err[1] is None
    assert err[2] is not None and err[3] is not None


def test_a_request_larger_than_the_budget_is_rejected_not_hung():
    reqs = [Request(0, "vfunc", _Keys(10 ** 6)), Request(1, "vfunc", _Keys(100))]
    st, _, _ = _run(reqs, slots=2, budget=5000)
    err = {r.rid: r.error for r in st.completed}
    assert err[0] is not None and err[1] is None


def test_resident_structures_count_until_released():
    def footprint(r):
        return 100, 60
    done = []
    s = Scheduler(2, 200, lambda slot, r, t: done.append(r.rid), footprint)
    for i in range(3):
        s.submit(Request(i, "vfunc", _Keys(1)))
    with pytest.raises(TimeoutError):
        s.drain(timeout=0.5)  # 2 x 60 resident + 100 running > 200
    s.release(0)
    s.drain(timeout=5)
    s.close()
    assert sorted(done) == [0, 1, 2]


def _coalescing_run(nq, slots, budget, coalesce):
    calls = []
    lock = threading.Lock()
    live = {"mem": 0, "peak": 0}

    def footprint(r):
        return (100, 100) if r.kind != "query" else (10, 0)

    def execute(slot, r, target):
        if r.kind != "query":
            time.sleep(0.2)  # the queries arrive meanwhile and wait for it
            return r.rid
        with lock:
            calls.append([r.rid])
        return 2 * r.rid

    def execute_many(slot, rs, targets):
        assert all(t is not None and t.rid == r.target for r, t in zip(rs, targets))
        with lock:
            calls.append([r.rid for r in rs])
        return [2 * r.rid for r in rs]

    s = Scheduler(slots, budget, execute, footprint, execute_many=execute_many,
                  coalesce=coalesce)
    s.submit(Request(0, "vfilter", _Keys(100)))
    for i in range(1, nq + 1):
        s.submit(Request(i, "query", _Keys(5), target=0))
    st = s.drain(timeout=30)
    s.close()
    return st, calls, s.groups


def test_waiting_queries_share_one_launch():
    st, calls, groups = _coalescing_run(12, slots=2, budget=10 ** 6, coalesce=8)
    assert st.summary()["errors"] == 0
    res = {r.rid: r.result for r in st.completed}
    assert all(res[i] == 2 * i for i in range(1, 13))
    assert sorted(i for c in calls for i in c) == list(range(1, 13))
    assert max(len(c) for c in calls) == 8 and groups >= 1
    # arrival order is kept inside a group
    assert all(c == sorted(c) for c in calls)


def test_merged_queries_stay_within_the_budget():
    # the build's 100 resident bytes plus at most two 10-byte queries fit
    st, calls, _ = _coalescing_run(9, slots=3, budget=125, coalesce=8)
    assert st.summary()["errors"] == 0
    assert st.peak_bytes <= 125
    assert max(len(c) for c in calls) <= 2
    assert sorted(i for c in calls for i in c) == list(range(1, 10))


def test_without_execute_many_queries_run_one_by_one():
    done = []
    s = Scheduler(1, 10 ** 6, lambda slot, r, t: done.append(r.rid), lambda r: (1, 0),
                  coalesce=8)
    s.submit(Request(0, "vfunc", _Keys(1)))
    for i in range(1, 5):
        s.submit(Request(i, "query", _Keys(1), target=0))
    s.drain(timeout=5)
    s.close()
    assert sorted(done) == [0, 1, 2, 3, 4] and s.groups == 0


def test_queries_of_a_build_too_large_for_the_budget_fail_not_wait():
    s = Scheduler(2, 50, lambda slot, r, t: r.rid,
                  lambda r: (100, 100) if r.kind != "query" else (1, 0))
    s.submit(Request(0, "vfilter", _Keys(1)))
    s.submit(Request(1, "query", _Keys(1), target=0))
    st = s.drain(timeout=5)
    s.close()
    assert all(r.error is not None for r in st.completed) and len(st.completed) == 2
