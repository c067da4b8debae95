"""Serving scheduler logic on the CPU: a simulated clock and a mock executor stand in
for the GPU, so admission, the HBM budget, slot limits and completion bookkeeping
are checked without a device."""
import concurrent.futures

import numpy as np
import pytest

from paper_1709_02733_amd import serving as SV


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class MockPlan:
    closed = 0

    def close(self):
        MockPlan.closed += 1


class MockWorkloads:
    keep_outputs = False

    def __init__(self, bytes_per_cell=50):
        self.bpc = bytes_per_cell

    def footprint(self, r):
        return r.n ** 3 * self.bpc

    def plan(self, r):
        return MockPlan()

    def io(self, r):
        return object(), object()

    def settle(self):
        pass


class MockExecutor:
    """Completes an operation after n^3 (M - 1) / rate seconds of simulated time."""

    def __init__(self, clock, max_slots=3, rate=5e9):
        self.clock, self.max_slots, self.rate = clock, max_slots, rate
        self.busy = {}
        self.started = []

    def start(self, plan, op, inp, out):
        free = [s for s in range(self.max_slots) if s not in self.busy]
        assert free, "scheduler started an operation without a free slot"
        s = free[0]
        self.busy[s] = self.clock() + self._dur
        self.started.append(s)
        return s

    def poll(self, slot):
        if self.clock() >= self.busy[slot]:
            del self.busy[slot]
            return True
        return False


def _run(reqs, budget, slots=3, bpc=50):
    clk = Clock()
    ex = MockExecutor(clk, max_slots=slots)
    wl = MockWorkloads(bpc)
    trace = []
    orig_start = ex.start
    # the scheduler admits in arrival order, so the k-th start is the k-th arrival
    order = iter(sorted(reqs, key=lambda q: q.arrival))

    def start_with_duration(plan, op, inp, out):
        r = next(order)
        ex._dur = r.cell_updates / ex.rate
        return orig_start(plan, op, inp, out)

    ex.start = start_with_duration
    SV.run_batched(reqs, wl, ex, budget_bytes=budget, clock=clk, sleep=clk.sleep, trace=trace)
    return reqs, trace, ex


def test_all_requests_complete_and_latency_is_causal():
    reqs = SV.request_mix(40, rate=10.0, seed=1, sizes=(32, 48, 64))
    out, trace, ex = _run(reqs, budget=1e12)
    assert all(r.done is not None and not r.rejected for r in out)
    for r in out:
        assert r.arrival <= r.admitted <= r.done
    assert max(a for _, _, a in trace) <= 3
    s = SV.summarize(out)
    assert s["n"] == 40 and s["p99_s"] >= s["p50_s"] > 0


def test_budget_is_never_exceeded_and_fifo_order_holds():
    reqs = SV.request_mix(30, rate=50.0, seed=2, sizes=(40, 64))
    budget = 64 ** 3 * 50 * 1.5          # at most one 64^3 request at a time next to smaller ones
    out, trace, ex = _run(reqs, budget=budget)
    assert all(used <= budget for _, used, _ in trace)
    adm = sorted(out, key=lambda r: r.arrival)
    assert all(adm[k].admitted <= adm[k + 1].admitted for k in range(len(adm) - 1))


def test_oversized_request_is_rejected_not_blocking():
    reqs = SV.request_mix(6, rate=5.0, seed=3, sizes=(32,))
    reqs[2].n = 200                     # footprint 200^3 * 50 B = 400 MB > budget
    out, trace, ex = _run(reqs, budget=1e8)
    assert out[2].rejected and out[2].done is None
    assert all(r.done is not None for k, r in enumerate(out) if k != 2)


def test_request_mix_statistics():
    reqs = SV.request_mix(2000, rate=4.0, seed=4)
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() - 0.25) < 0.02
    assert abs(np.mean([r.op == 0 for r in reqs]) - 0.6) < 0.05
    assert {r.n for r in reqs} == set(SV.SIZES)
    assert all(256 <= r.nrec <= 1024 for r in reqs)
    assert all(r.nsteps == 800 + (r.n - 96) * 1000 // 160 for r in reqs)


class TaggedWorkloads(MockWorkloads):
    """Plans that carry their request, so a mock start can look up its duration."""

    def plan(self, r):
        p = MockPlan()
        p.req = r
        return p


def _run_tagged(reqs, budget, slots=1):
    clk = Clock()
    ex = MockExecutor(clk, max_slots=slots)
    orig_start = ex.start
    started = []

    def start(plan, op, inp, out):
        ex._dur = plan.req.cell_updates / ex.rate
        started.append(plan.req.rid)
        return orig_start(plan, op, inp, out)

    ex.start = start
    trace = []
    SV.run_batched(reqs, TaggedWorkloads(), ex, budget_bytes=budget, clock=clk, sleep=clk.sleep, trace=trace)
    return reqs, started, trace


def test_cancelled_waiting_request_takes_no_slot():
    """With one slot, request 1 waits behind request 0 and is withdrawn while waiting: it is
    never started, takes no budget, and request 2 follows request 0 directly."""
    reqs = [SV.Request(rid=k, op=0, n=32, nsteps=200, nrec=8, seed=k, arrival=0.001 * k) for k in range(3)]
    dur = reqs[0].cell_updates / 5e9
    reqs[1].cancel_at = 0.5 * dur
    out, started, trace = _run_tagged(reqs, budget=1e12, slots=1)
    assert started == [0, 2]
    assert out[1].cancelled and out[1].admitted is None and out[1].done is None
    assert out[0].done is not None and out[2].done is not None
    assert out[2].admitted >= out[0].done
    assert SV.summarize(out)["n"] == 2


def test_cancelled_running_request_frees_its_slot_when_the_device_finishes():
    """Request 0 is withdrawn while it runs: its output is dropped, it gets no done time,
    and its slot and bytes return when its enqueued work ends, admitting request 1."""
    reqs = [SV.Request(rid=k, op=0, n=32, nsteps=200, nrec=8, seed=k, arrival=0.001 * k) for k in range(2)]
    dur = reqs[0].cell_updates / 5e9
    reqs[0].cancel_at = 0.3 * dur
    out, started, trace = _run_tagged(reqs, budget=1e12, slots=1)
    assert started == [0, 1]
    assert out[0].cancelled and out[0].output is None and out[0].done is None
    assert out[1].admitted >= dur and out[1].done is not None
    assert trace[-1][1] == 0 and trace[-1][2] == 0     # nothing held at the end


class MockGroup:
    """A simulated el_group: every tick advances each running member one step and takes
    (sum of the running members' cells) / rate seconds of device time; run() enqueues,
    sync(k) lets the simulated clock catch up with all but the last k runs."""

    def __init__(self, clock, max_members=4, rate=5e9):
        self.clock, self.max_members, self.rate = clock, max_members, rate
        self.m = {}          # slot -> dict(req, steps, end, done_at, withdrawn)
        self.dev_t = 0.0
        self.runs = []
        self.added = []
        self.max_running = 0

    def add(self, plan, op, inp, out):
        free = [s for s in range(self.max_members) if s not in self.m]
        assert free, "scheduler added a member without a free slot"
        s = free[0]
        r = plan.req
        self.m[s] = dict(req=r, steps=0, total=r.nsteps - 1, done_at=None)
        self.added.append(r.rid)
        return s

    def members(self):
        run = sum(1 for v in self.m.values() if v["done_at"] is None)
        return self.max_members, len(self.m), run

    def run(self, ticks):
        t = max(self.dev_t, self.clock())
        for _ in range(ticks):
            live = [v for v in self.m.values() if v["done_at"] is None]
            if not live:
                break
            self.max_running = max(self.max_running, len(live))
            t += sum(v["req"].n ** 3 for v in live) / self.rate
            for v in live:
                v["steps"] += 1
                if v["steps"] == v["total"]:
                    v["done_at"] = t
        self.dev_t = t
        self.runs.append(t)

    def sync(self, pending=0):
        while len(self.runs) > pending:
            self.clock.t = max(self.clock.t, self.runs.pop(0))

    def remove(self, slot):
        v = self.m[slot]
        if v["done_at"] is None:
            v["done_at"] = max(self.dev_t, self.clock())

    def poll(self, slot):
        v = self.m[slot]
        if v["done_at"] is not None and self.clock() >= v["done_at"]:
            del self.m[slot]
            return v["steps"], True
        return v["steps"], False


class SyncPool:
    """Builds a plan at submission (the simulated clock does not see a worker thread)."""

    def submit(self, fn, *args):
        f = concurrent.futures.Future()
        f.set_result(fn(*args))
        return f


def _run_grouped(reqs, budget, members=3, bpc=50):
    clk = Clock()
    g = MockGroup(clk, max_members=members)
    trace = []
    SV.run_grouped(reqs, TaggedWorkloads(bpc), g, budget_bytes=budget, clock=clk, sleep=clk.sleep, trace=trace,
                   rate_guess=5e9, pool=SyncPool())
    return reqs, trace, g


def test_grouped_all_requests_complete_within_slots_and_budget():
    reqs = SV.request_mix(40, rate=10.0, seed=1, sizes=(32, 48, 64))
    budget = 64 ** 3 * 50 * 2.5
    out, trace, g = _run_grouped(reqs, budget=budget, members=3)
    assert all(r.done is not None and not r.rejected for r in out)
    for r in out:
        assert r.arrival <= r.admitted <= r.done
    assert all(used <= budget for _, used, _ in trace)
    assert max(a for _, _, a in trace) <= 3 and g.max_running <= 3
    assert g.added == sorted(g.added)        # first come, first served
    assert trace[-1][1] == 0 and trace[-1][2] == 0
    s = SV.summarize(out)
    assert s["n"] == 40 and s["p99_s"] >= s["p50_s"] > 0


def test_grouped_requests_share_ticks():
    """Requests that overlap in time step together: three arrivals at once finish after
    about max(M) ticks of the three, not after the sum of their step counts."""
    reqs = [SV.Request(rid=k, op=k % 2, n=32, nsteps=100 + 50 * k, nrec=8, seed=k, arrival=0.0) for k in range(3)]
    out, trace, g = _run_grouped(reqs, budget=1e12, members=3)
    tick_all = 3 * 32 ** 3 / 5e9
    assert max(r.done for r in out) < 1.5 * 199 * tick_all
    assert g.max_running == 3


def test_grouped_withdrawal_while_waiting_and_running():
    reqs = [SV.Request(rid=k, op=0, n=32, nsteps=200, nrec=8, seed=k, arrival=0.001 * k) for k in range(3)]
    dur = reqs[0].cell_updates / 5e9
    reqs[0].cancel_at = 0.3 * dur          # while it runs
    reqs[2].cancel_at = 0.0005             # before it arrives: never admitted
    out, trace, g = _run_grouped(reqs, budget=1e12, members=1)
    assert out[0].cancelled and out[0].output is None and out[0].done is None
    assert out[2].cancelled and out[2].admitted is None
    assert out[1].done is not None and g.added == [0, 1]
    assert trace[-1][1] == 0 and trace[-1][2] == 0


def test_grouped_oversized_request_is_rejected():
    reqs = SV.request_mix(6, rate=5.0, seed=3, sizes=(32,))
    reqs[2].n = 200
    out, trace, g = _run_grouped(reqs, budget=1e8)
    assert out[2].rejected and out[2].done is None
    assert all(r.done is not None for k, r in enumerate(out) if k != 2)


def test_grouped_cap_on_large_requests_lets_small_ones_pass():
    """max_large = 1: never two large requests in the group at once; a small request that
    arrives behind a waiting large one joins before it."""
    reqs = [SV.Request(rid=0, op=0, n=64, nsteps=200, nrec=8, seed=0, arrival=0.0),
            SV.Request(rid=1, op=1, n=64, nsteps=200, nrec=8, seed=1, arrival=0.001),
            SV.Request(rid=2, op=0, n=24, nsteps=100, nrec=8, seed=2, arrival=0.002)]
    clk = Clock()
    g = MockGroup(clk, max_members=4)
    large = []
    orig_run = g.run

    def run(ticks):
        live = [v["req"].rid for v in g.m.values() if v["done_at"] is None and v["req"].n == 64]
        large.append(len(live))
        orig_run(ticks)

    g.run = run
    SV.run_grouped(reqs, TaggedWorkloads(), g, budget_bytes=1e12, clock=clk, sleep=clk.sleep, rate_guess=5e9,
                   pool=SyncPool(), max_large=1, large_cells=48 ** 3)
    assert max(large) == 1
    assert g.added == [0, 2, 1]
    assert all(r.done is not None for r in reqs)
    assert reqs[2].admitted < reqs[1].admitted


def test_hybrid_sends_large_requests_to_the_executor():
    """Hybrid mode: requests of >= large_cells cells start on executor slots (at most its
    slot count at once), the others join the group; all complete within the budget."""
    reqs = SV.request_mix(30, rate=20.0, seed=9, sizes=(24, 32, 64))
    clk = Clock()
    g = MockGroup(clk, max_members=4)
    ex = MockExecutor(clk, max_slots=2)
    started = []
    orig_start = ex.start

    def start(plan, op, inp, out):
        ex._dur = plan.req.cell_updates / ex.rate
        started.append(plan.req.rid)
        assert len(ex.busy) < ex.max_slots
        return orig_start(plan, op, inp, out)

    ex.start = start
    budget = 64 ** 3 * 50 * 3.5
    trace = []
    SV.run_grouped(reqs, TaggedWorkloads(), g, budget_bytes=budget, clock=clk, sleep=clk.sleep, trace=trace,
                   rate_guess=5e9, pool=SyncPool(), executor=ex, large_cells=48 ** 3)
    large = {r.rid for r in reqs if r.n == 64}
    assert set(started) == large and len(started) == len(large)
    assert set(g.added) == {r.rid for r in reqs} - large
    assert all(r.done is not None for r in reqs)
    assert all(used <= budget for _, used, _ in trace)
    assert trace[-1][1] == 0 and trace[-1][2] == 0
