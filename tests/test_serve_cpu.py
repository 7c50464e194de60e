"""Host-only tests of the serving scheduler: admission by memory budget,
waiting and rejection, continuous batching (late arrivals join the next
step while earlier ones run), slot reuse and termination.  A fake executor
runs steps on a simulated clock, so no GPU is involved."""
import collections

import pytest

from paper_2007_12065_amd.serve import (ADMITTED, REJECTED, FrameClass, Request, SlotPool,
                                        run_stream, slot_bytes, summarize)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    """Each step takes `step_s` plus `per_frame_s` per frame; steps run one
    after another on a simulated device."""

    def __init__(self, clock, step_s=1e-3, per_frame_s=1e-4):
        self.clock, self.step_s, self.per_frame_s = clock, step_s, per_frame_s
        self.n = 0
        self.busy_until = 0.0
        self.steps = []
        self.rebuilds = 0

    def rebuild(self):
        # like the GPU executor: the plan spans the slots that exist now
        self.rebuilds += 1
        self.n = len(self.pool.slots)

    def launch(self, members):
        start = max(self.clock(), self.busy_until)
        end = start + self.step_s + self.per_frame_s * len(members)
        self.busy_until = end
        self.steps.append((self.clock(), end, [r.rid for _, r in members]))
        return end

    def ready(self, end):
        return self.clock() >= end

    def wait(self, end):
        if self.clock() < end:
            self.clock.t = end
        return end


def make_pool(budget, per, exe, presize=None):
    pool = SlotPool(budget, per)
    exe.pool = pool
    for cls, k in (presize or {}).items():         # as Server.presize does
        got = [pool.acquire(cls)[1] for _ in range(k)]
        for sl in got:
            pool.release(sl)
    if presize:
        exe.rebuild()
    return pool


def test_pool_budget_wait_reject_release():
    pool = SlotPool(1000, {"a": 100, "b": 300, "huge": 2000})
    got = [pool.acquire("a") for _ in range(10)]
    assert all(st == ADMITTED for st, _ in got)
    assert pool.acquire("a")[0] == "waiting"
    assert pool.acquire("b")[0] == "waiting"
    assert pool.acquire("huge") == (REJECTED, None)
    pool.release(got[3][1])
    st, s = pool.acquire("a")
    assert st == ADMITTED and s is got[3][1]          # the resident slot is reused
    assert pool.used == 1000 and len(pool.slots) == 10
    with pytest.raises(AssertionError):
        pool.release(got[0][1]); pool.release(got[0][1])


def test_growth_closed_waits():
    pool = SlotPool(10_000, {"a": 100})
    st, s = pool.acquire("a")
    pool.release(s)
    pool.growth_open = False
    assert pool.acquire("a")[0] == ADMITTED
    assert pool.acquire("a")[0] == "waiting"


def test_continuous_batching_joins_next_step():
    clock = Clock()
    exe = FakeExecutor(clock, step_s=5e-3, per_frame_s=0.0)
    pool = make_pool(10_000, {"a": 100}, exe, presize={"a": 8})
    # 1 request at t=0, then 5 arriving while the first step (5 ms) runs
    times = [0.0, 1e-3, 1.5e-3, 2e-3, 3e-3, 4e-3]
    reqs = [Request(i, "a", t, 0) for i, t in enumerate(times)]
    stats = run_stream(reqs, pool, exe, clock, clock.sleep, max_inflight=2)
    assert all(r.status == ADMITTED and r.done > r.arrival for r in reqs)
    # the first step holds request 0 only; late arrivals are batched into the
    # next steps, which were enqueued while the first was still running
    assert exe.steps[0][2] == [0]
    later = [rid for _, _, ids in exe.steps[1:] for rid in ids]
    assert sorted(later) == [1, 2, 3, 4, 5]
    assert exe.steps[1][0] < exe.steps[0][1]          # enqueued before step 0 ended
    assert stats["steps"] < len(reqs)                 # batching happened


def test_budget_limits_concurrency_and_everything_completes():
    clock = Clock()
    exe = FakeExecutor(clock, step_s=2e-3, per_frame_s=1e-4)
    per = {"small": 100, "big": 400}
    pool = make_pool(1000, per, exe)
    kinds = ["big", "small"] * 20
    reqs = [Request(i, k, i * 1e-4, 0) for i, k in enumerate(kinds)]
    run_stream(reqs, pool, exe, clock, clock.sleep, max_inflight=2)
    assert all(r.status == ADMITTED for r in reqs)
    assert pool.used <= 1000
    # never more frames of a step than resident slots
    assert max(len(ids) for _, _, ids in exe.steps) <= len(pool.slots)
    # slots were reused: far fewer slots than requests
    assert len(pool.slots) < len(reqs)
    assert all(not s.busy for s in pool.slots)


def test_oversize_and_starved_requests_are_rejected():
    clock = Clock()
    exe = FakeExecutor(clock)
    pool = make_pool(1000, {"a": 600, "b": 500, "huge": 5000}, exe)
    reqs = [Request(0, "a", 0.0, 0), Request(1, "huge", 0.0, 0), Request(2, "b", 1.0, 0)]
    run_stream(reqs, pool, exe, clock, clock.sleep)
    assert reqs[0].status == ADMITTED
    assert reqs[1].status == REJECTED                 # could never fit
    assert reqs[2].status == REJECTED                 # budget held by class a forever
    s = summarize(reqs, 0.0, {"a": FrameClass("a", 10, 10, 3, 1.0, 1, 3, 0.1, 0.1, 1),
                              "b": FrameClass("b", 10, 10, 3, 1.0, 1, 3, 0.1, 0.1, 1),
                              "huge": FrameClass("huge", 10, 10, 3, 1.0, 1, 3, 0.1, 0.1, 1)})
    assert s["rejected"] == 2 and s["frames"] == 1


def test_plan_rebuilt_when_pool_grows():
    clock = Clock()
    exe = FakeExecutor(clock, step_s=1e-3)
    pool = make_pool(10_000, {"a": 100}, exe)
    reqs = [Request(i, "a", 0.0, 0) for i in range(4)]
    stats = run_stream(reqs, pool, exe, clock, clock.sleep)
    assert stats["plan_rebuilds"] >= 1 and exe.rebuilds == stats["plan_rebuilds"]
    assert all(r.status == ADMITTED for r in reqs)


def test_slot_bytes_accounts_for_every_buffer():
    c = FrameClass("rgbd", 480, 640, 3, 1.0, 4, 3, 0.1, 0.1, 2)
    b16 = slot_bytes(c, 2, 4, 1)
    b32 = slot_bytes(c, 4, 4, 1)
    P, T = 480 * 640, 2 * 479 * 639
    assert b32 - b16 >= 3 * T * 2 * 3               # three normal arrays shrink by 2 B/comp
    assert b16 >= 24 * P + 12 * T + T + 4 * T + 24 * T + 3 * T * 2 * 3
    assert b16 < 80e6


def test_arrival_wait_neither_oversleeps_nor_returns_late():
    # a short gap is spun out on the clock (returns once it has passed, not
    # much later); a long one is only half slept, leaving the rest to the
    # caller's next wait, so the OS sleep's overshoot cannot delay an arrival
    import time

    from paper_2007_12065_amd.serve import arrival_wait
    for dt in (0.0, 2e-5, 1.5e-4):
        t0 = time.perf_counter()
        arrival_wait(dt)
        took = time.perf_counter() - t0
        assert dt <= took < dt + 0.02
    t0 = time.perf_counter()
    arrival_wait(0.2)
    took = time.perf_counter() - t0
    assert 0.099 <= took < 0.19
