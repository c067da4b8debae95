"""Serving scheduler logic on the CPU: a simulated clock and a mock executor stand in
for the GPU, so admission, the HBM budget, slot limits and completion bookkeeping
are checked without a device."""
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
