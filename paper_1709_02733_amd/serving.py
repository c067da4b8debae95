"""Serving forward and adjoint applications of many reconstructions at once.

Requests (a forward H p0 or an adjoint H^T y, each on its own grid, medium,
step count and receiver set) arrive as a Poisson stream.  Two ways to serve
them:

* plain: first come, first served, one request at a time, each through
  el_forward / el_adjoint with per-step kernel launches.
* batched (continuous batching): a request is admitted as soon as it has
  arrived, an executor slot is free and the HBM budget (sum of the plans'
  workspaces and buffers of the admitted requests) allows it.  Each admitted
  request runs on its own slot stream as replays of captured step graphs,
  concurrently with the others; the host builds the next plans while the
  device works and retires requests as their completion events fire.

Both paths run the same kernels in the same order per request, so each
result is bitwise the same alone and in the mix.  The report gives
throughput (requests/s and Gcell-updates/s) and p50/p99 latency (arrival to
result) per arrival rate.

    python -m paper_1709_02733_amd.serving --rates 2 5 10 20 --count 200
"""
from __future__ import annotations

import argparse
import collections
import dataclasses
import json
import math
import sys
import time

import numpy as np

from . import scenarios as S

SIZES = (96, 128, 192, 256)


@dataclasses.dataclass
class Request:
    rid: int
    op: int                 # 0 forward, 1 adjoint (el.OP_FORWARD / el.OP_ADJOINT)
    n: int                  # grid is n^3
    nsteps: int
    nrec: int
    seed: int
    arrival: float          # seconds after the start of the run
    bytes: int = 0          # device bytes while admitted (workspace + input + output)
    admitted: float | None = None
    done: float | None = None
    rejected: bool = False
    output: object = None
    cancel_at: float | None = None   # the client withdraws the request at this time (run_batched)
    cancelled: bool = False

    @property
    def cell_updates(self) -> int:
        return self.n ** 3 * (self.nsteps - 1)


def request_mix(count: int, rate: float, seed: int = 0, sizes=SIZES, fwd_fraction: float = 0.6,
                nrec_range=(256, 1024)) -> list[Request]:
    """Poisson arrivals at `rate` per second; sizes uniform over `sizes`, step counts scaled
    with the size (800 at 96^3 .. 1800 at 256^3), receivers uniform in nrec_range."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(rng.choice(sizes))
        op = 0 if rng.uniform() < fwd_fraction else 1
        out.append(Request(rid=k, op=op, n=n, nsteps=S.serving_steps(n), seed=int(rng.integers(1 << 30)),
                           nrec=int(rng.integers(nrec_range[0], nrec_range[1] + 1)), arrival=t))
    return out


def clone_requests(reqs):
    return [dataclasses.replace(r, admitted=None, done=None, rejected=False, output=None, cancelled=False) for r in reqs]


class Workloads:
    """Device-resident inputs per grid size: one skull-recipe medium per size, its vessel
    p0, and receivers on the upper hemisphere of radius 0.47 n (the recipe of the 384^3
    workload, scaled)."""

    def __init__(self, sizes=SIZES, device=None, seed=7, keep_outputs=False):
        import torch
        from . import el
        self.torch, self.el = torch, el
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.keep_outputs = keep_outputs
        self.media = {}
        for n in sizes:
            sc = S.skull_scenario(n=n, seed=seed + n, nsteps=S.serving_steps(n), npml=16, nrec=8)
            d = dict(sc=sc)
            for k in ("lam", "mu", "rho", "alpha", "p0"):
                d[k] = torch.from_numpy(getattr(sc, k)).to(self.device)
            self.media[n] = d

    def receivers(self, r: Request) -> np.ndarray:
        sc = self.media[r.n]["sc"]
        c = (r.n - 1) / 2.0
        return (c + 0.47 * r.n * S.fibonacci_sphere(r.nrec, hemisphere=True)) * sc.dx

    def grid(self, r: Request):
        sc = self.media[r.n]["sc"]
        return self.el.make_grid(r.n, r.n, r.n, sc.dx, sc.dt, r.nsteps, 16)

    def footprint(self, r: Request) -> int:
        ws = self.el.plan_bytes(self.grid(r), r.nrec)
        io = r.n ** 3 * 4 + r.nsteps * r.nrec * 8
        return int(ws + io)

    def plan(self, r: Request):
        m = self.media[r.n]
        sc = m["sc"]
        return self.el.Plan(r.n, r.n, r.n, sc.dx, sc.dt, r.nsteps, 16, m["lam"], m["mu"], m["rho"], m["alpha"],
                            self.receivers(r), device=self.device)

    def io(self, r: Request):
        torch = self.torch
        g = torch.Generator(device=self.device).manual_seed(r.seed)
        if r.op == 0:
            scale = 0.5 + (r.seed % 1000) / 1000.0
            inp = self.media[r.n]["p0"] * scale
            out = torch.empty((r.nsteps, r.nrec), dtype=torch.float64, device=self.device)
        else:
            inp = torch.randn((r.nsteps, r.nrec), generator=g, dtype=torch.float64, device=self.device)
            out = torch.empty((r.n, r.n, r.n), dtype=torch.float32, device=self.device)
        return inp, out


# ---------------------------------------------------------------------------------------
# the two serving loops
# ---------------------------------------------------------------------------------------

def run_plain(reqs, wl, clock=time.perf_counter, sleep=time.sleep, sync=None):
    """One request at a time in arrival order through el_forward / el_adjoint."""
    if sync is None:
        sync = wl.torch.cuda.synchronize
    t0 = clock()
    for r in sorted(reqs, key=lambda q: q.arrival):
        now = clock() - t0
        if now < r.arrival:
            sleep(r.arrival - now)
        r.admitted = clock() - t0
        plan = wl.plan(r)
        inp, out = wl.io(r)
        if r.op == 0:
            plan.forward(inp, out=out)
        else:
            plan.adjoint(inp, out=out)
        sync()
        r.done = clock() - t0
        if wl.keep_outputs:
            r.output = out
        plan.close()
    return reqs


def run_batched(reqs, wl, executor, budget_bytes: float = 200e9, clock=time.perf_counter, sleep=time.sleep,
                trace=None):
    """Continuous batching over the executor's slots under an HBM budget.

    Admission is first come, first served: the oldest arrived request is admitted
    once a slot is free and its footprint fits next to the admitted ones; a request
    whose footprint alone exceeds the budget is rejected.  A request withdrawn
    (cancel_at reached) while it waits leaves the queue without taking a slot or any
    budget; one withdrawn while it runs has its output dropped, and its slot and
    bytes return when the device finishes the work already enqueued on it (a stream
    cannot take back enqueued work).  Cancelled requests get no `done` time.
    `trace`, if given, receives (time, bytes in use, active count) after every change.
    """
    pending = collections.deque(sorted(reqs, key=lambda q: q.arrival))
    active = {}
    in_use = 0
    t0 = clock()
    while pending or active:
        now = clock() - t0
        changed = False
        if any(r.cancel_at is not None and r.cancel_at <= now for r in pending):
            keep = collections.deque()
            for r in pending:
                if r.cancel_at is not None and r.cancel_at <= now:
                    r.cancelled = True
                    changed = True
                else:
                    keep.append(r)
            pending = keep
        for slot in list(active):
            r = active[slot][0]
            if not r.cancelled and r.cancel_at is not None and r.cancel_at <= now:
                r.cancelled = True
                r.output = None
                changed = True
            if executor.poll(slot):
                r, plan = active.pop(slot)
                if not r.cancelled:
                    r.done = clock() - t0
                in_use -= r.bytes
                plan.close()
                changed = True
        while pending and pending[0].arrival <= now and len(active) < executor.max_slots:
            r = pending[0]
            if r.bytes == 0:
                r.bytes = wl.footprint(r)
            if r.bytes > budget_bytes:
                pending.popleft()
                r.rejected = True
                changed = True
                continue
            if in_use + r.bytes > budget_bytes:
                break
            pending.popleft()
            plan = wl.plan(r)
            inp, out = wl.io(r)
            slot = executor.start(plan, r.op, inp, out)
            r.admitted = clock() - t0
            if wl.keep_outputs:
                r.output = out
            active[slot] = (r, plan)
            in_use += r.bytes
            changed = True
        if trace is not None and changed:
            trace.append((clock() - t0, in_use, len(active)))
        if not changed:
            nxt = pending[0].arrival - (clock() - t0) if pending and not active else 0.0
            sleep(max(2e-4, min(nxt, 0.01)))
    return reqs


def summarize(reqs) -> dict:
    done = [r for r in reqs if r.done is not None]
    if not done:
        return dict(n=0)
    lat = np.array([r.done - r.arrival for r in done])
    span = max(r.done for r in done) - min(r.arrival for r in done)
    upd = sum(r.cell_updates for r in done)
    return dict(n=len(done), rejected=sum(r.rejected for r in reqs), span_s=span,
                throughput_rps=len(done) / span, gcells=upd / span / 1e9,
                p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()))


def serve_benchmark(rates=(2, 5, 10, 20), count=200, sizes=SIZES, max_slots=4, chunk=64, budget=200e9, seed=0,
                    log=lambda *a: print(*a, file=sys.stderr, flush=True)):
    """Plain versus batched serving of the same request streams; one entry per rate."""
    import torch
    from . import el
    wl = Workloads(sizes)
    ex = el.Executor(max_slots=max_slots, chunk=chunk)
    # warm both paths on one request per size (kernel loading, allocator growth)
    warm = [Request(rid=-1 - k, op=k % 2, n=n, nsteps=S.serving_steps(n), nrec=256, seed=k, arrival=0.0)
            for k, n in enumerate(sizes)]
    run_plain(clone_requests(warm), wl)
    run_batched(clone_requests(warm), wl, ex, budget)
    torch.cuda.synchronize()
    out = []
    for k, rate in enumerate(rates):
        reqs = request_mix(count, rate, seed=seed + k, sizes=sizes)
        a = run_plain(clone_requests(reqs), wl)
        b = run_batched(clone_requests(reqs), wl, ex, budget)
        sa, sb = summarize(a), summarize(b)
        ent = dict(rate=rate, count=count, plain=sa, batched=sb,
                   throughput_gain=sb["gcells"] / sa["gcells"] if sa.get("gcells") else None)
        log(f"[serve] rate {rate}/s: plain {sa['gcells']:.2f} Gcell/s p50 {sa['p50_s']:.2f}s p99 {sa['p99_s']:.2f}s | "
            f"batched {sb['gcells']:.2f} Gcell/s p50 {sb['p50_s']:.2f}s p99 {sb['p99_s']:.2f}s")
        out.append(ent)
    ex.close()
    return out


def main():
    ap = argparse.ArgumentParser(description="plain vs batched serving of H / H^T requests")
    ap.add_argument("--rates", type=float, nargs="+", default=[2, 5, 10, 20])
    ap.add_argument("--count", type=int, default=200)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    res = serve_benchmark(rates=args.rates, count=args.count, max_slots=args.slots, chunk=args.chunk,
                          budget=args.budget_gb * 1e9, seed=args.seed)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
