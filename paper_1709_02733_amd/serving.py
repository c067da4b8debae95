"""Serving forward and adjoint applications of many reconstructions at once.

Requests (a forward H p0 or an adjoint H^T y, each on its own grid, medium,
step count and receiver set) arrive as a Poisson stream.  Ways to serve them:

* plain: first come, first served, one request at a time, each through
  el_forward / el_adjoint with per-step kernel launches.
* grouped (continuous batching, el_group): a request is admitted as soon as
  it has arrived, a group slot is free and the HBM budget (sum of the plans'
  workspaces and buffers of the admitted requests) allows it.  A worker
  thread builds its plan while the device works; it then joins the group,
  which advances all running requests one time step per tick with one
  launch per sub-update for up to four requests at a time.  At most one
  large request runs at a time and small ones may pass a large one that
  waits (serve_benchmark's setting), so small requests do not queue behind
  large ones.  Requests leave the group after their last step.
* executor (run_batched): each admitted request runs on its own slot stream
  as replays of captured step graphs, concurrently with the others (the
  steadiest throughput gain over plain).
* hybrid (run_grouped with an executor): small requests join the group, large
  ones (which fill the device alone) run on executor slots, and the two
  overlap on the device.  The executor keeps two graph replays in flight per
  slot (el_exec_set_ahead), so the group's launches never wait behind a large
  request's whole time loop in a shared hardware queue.

All paths run the same per-cell arithmetic in the same order per request, so
each result is bitwise the same alone and in the mix.  The report gives
throughput (requests/s and Gcell-updates/s) and p50/p99 latency (arrival to
result) per arrival rate.

    python -m paper_1709_02733_amd.serving --rates 2 5 10 20 --count 100 --modes plain executor grouped hybrid
"""
from __future__ import annotations

import argparse
import collections
import concurrent.futures
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
    workload, scaled).

    per_request_media: each request gets its own medium, the size's skull medium shifted
    by up to 4 cells along each axis and its sound speeds and density scaled by up to
    +-3% (seeded by the request), so that every plan is built from different maps."""

    def __init__(self, sizes=SIZES, device=None, seed=7, keep_outputs=False, per_request_media=False):
        import torch
        from . import el
        self.torch, self.el = torch, el
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.keep_outputs = keep_outputs
        self.per_request_media = per_request_media
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

    def medium(self, r: Request):
        """lam, mu, rho, alpha of the request (device tensors)."""
        m = self.media[r.n]
        if not self.per_request_media:
            return m["lam"], m["mu"], m["rho"], m["alpha"]
        torch = self.torch
        rng = np.random.default_rng(r.seed)
        shift = tuple(int(v) for v in rng.integers(-4, 5, size=3))
        cs, rs = 1.0 + rng.uniform(-0.03, 0.03, size=2)
        roll = lambda a: torch.roll(a, shifts=shift, dims=(0, 1, 2))
        # lambda and mu scale with rho c^2: sound speeds by cs, density by rs
        k = float(rs * cs * cs)
        return roll(m["lam"]) * k, roll(m["mu"]) * k, roll(m["rho"]) * float(rs), roll(m["alpha"])

    def plan(self, r: Request):
        sc = self.media[r.n]["sc"]
        lam, mu, rho, alpha = self.medium(r)
        # a medium whose sound speeds grew by up to 3% needs a time step to match (CFL)
        dt = sc.dt / 1.03 if self.per_request_media else sc.dt
        return self.el.Plan(r.n, r.n, r.n, sc.dx, dt, r.nsteps, 16, lam, mu, rho, alpha, self.receivers(r),
                            device=self.device)

    def settle(self):
        """Wait for the work this thread enqueued (a plan's inputs built off the main thread)."""
        self.torch.cuda.current_stream(self.device).synchronize()

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


def _cells(r: Request) -> int:
    return r.n ** 3


def run_grouped(reqs, wl, group, budget_bytes: float = 200e9, clock=time.perf_counter, sleep=time.sleep,
                trace=None, run_ms: float = 2.0, rate_guess: float = 40e9, pool=None, ahead: int = 1,
                max_large: int | None = None, large_cells: int = 4_000_000, executor=None):
    """Continuous batching over an el_group under an HBM budget.

    Admission is first come, first served, as in run_batched; an admitted request's plan
    and buffers are built by a worker thread while the device steps the running members.
    Each round of the loop enqueues about `run_ms` of steps (estimated from the running
    members' cells at `rate_guess` cell-updates/s) and keeps at most `ahead` such runs queued
    behind the one the device is executing, so that joins and completions are seen within
    a few milliseconds.  Withdrawal (cancel_at) works as in run_batched.  `pool`: where
    plans are built (default: one worker thread).

    max_large: at most this many requests of >= large_cells cells run (or are being built)
    at once; an arrived large request that waits for this cap lets later small requests
    pass it, so small grids fill the launches of the large ones instead of several large
    requests sharing the device step by step.  None: no cap (strict arrival order).

    executor: large requests run on the executor's slots (a stream and captured step graphs
    each, at most max_large of them if set) instead of in the group, so that the group's
    small requests overlap with them on the device (hybrid mode).
    """
    pending = collections.deque(sorted(reqs, key=lambda q: q.arrival))
    building = {}      # future -> request
    ready = []         # (request, plan, input, output) built, waiting to join
    members = {}       # slot -> (request, plan)
    ex_active = {}     # executor slot -> (request, plan), hybrid mode
    in_use = 0
    own_pool = pool is None
    if own_pool:
        pool = concurrent.futures.ThreadPoolExecutor(max_workers=1)

    def build(r):
        plan = wl.plan(r)
        inp, out = wl.io(r)
        wl.settle()
        return plan, inp, out

    t0 = clock()
    try:
        while pending or building or ready or members or ex_active:
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
            for slot in list(members):
                r, plan = members[slot]
                if not r.cancelled and r.cancel_at is not None and r.cancel_at <= now:
                    r.cancelled = True
                    r.output = None
                    group.remove(slot)
                    changed = True
                _, done = group.poll(slot)
                if done:
                    members.pop(slot)
                    if not r.cancelled:
                        r.done = clock() - t0
                    in_use -= r.bytes
                    plan.close()
                    changed = True
            for slot in list(ex_active):
                r, plan = ex_active[slot]
                if not r.cancelled and r.cancel_at is not None and r.cancel_at <= now:
                    r.cancelled = True
                    r.output = None
                    changed = True
                if executor.poll(slot):
                    ex_active.pop(slot)
                    if not r.cancelled:
                        r.done = clock() - t0
                    in_use -= r.bytes
                    plan.close()
                    changed = True
            is_large = lambda q: _cells(q) >= large_cells
            # a request is built ahead of its turn (one beyond the free slots, and one large
            # request beyond the cap), so that its plan is ready when the device can take it
            ex_slots = executor.max_slots if executor is not None else 0
            large_cap = max_large if max_large is not None else (ex_slots if executor is not None else None)
            queued = len(members) + len(ex_active) + len(building) + len(ready)
            n_large = (sum(1 for q, _ in members.values() if is_large(q)) + len(ex_active)
                       + sum(1 for q in building.values() if is_large(q)) + sum(1 for q, *_ in ready if is_large(q)))
            idx = 0
            while idx < len(pending) and pending[idx].arrival <= now and queued < group.max_members + ex_slots + 1:
                r = pending[idx]
                if r.bytes == 0:
                    r.bytes = wl.footprint(r)
                if r.bytes > budget_bytes:
                    del pending[idx]
                    r.rejected = True
                    changed = True
                    continue
                if in_use + r.bytes > budget_bytes:
                    break
                if is_large(r) and large_cap is not None and n_large >= large_cap + 1:
                    idx += 1          # waits for the cap; later small requests may pass it
                    continue
                del pending[idx]
                in_use += r.bytes
                queued += 1
                n_large += 1 if is_large(r) else 0
                building[pool.submit(build, r)] = r
                changed = True
            # built plans in submission order, up to the first plan not built yet
            while building and next(iter(building)).done():
                fut = next(iter(building))
                r = building.pop(fut)
                ready.append((r,) + tuple(fut.result()))
                changed = True
            # join the group in admission order; a large request that waits for the cap lets
            # later small ones pass it
            large_running = sum(1 for q, _ in members.values() if is_large(q)) + len(ex_active)
            k = 0
            while k < len(ready):
                r, plan, inp, out = ready[k]
                if r.cancel_at is not None and r.cancel_at <= clock() - t0:
                    del ready[k]
                    r.cancelled = True
                    in_use -= r.bytes
                    plan.close()
                    changed = True
                    continue
                large = is_large(r)
                to_executor = large and executor is not None
                if ((large and large_cap is not None and large_running >= large_cap)
                        or (to_executor and len(ex_active) >= ex_slots)
                        or (not to_executor and len(members) >= group.max_members)):
                    k += 1
                    continue
                del ready[k]
                if to_executor:
                    slot = executor.start(plan, r.op, inp, out)
                    ex_active[slot] = (r, plan)
                else:
                    slot = group.add(plan, r.op, inp, out)
                    members[slot] = (r, plan)
                r.admitted = clock() - t0
                if wl.keep_outputs:
                    r.output = out
                large_running += 1 if large else 0
                changed = True
            if trace is not None and changed:
                trace.append((clock() - t0, in_use, len(members) + len(ex_active)))
            running = [r for r, _ in members.values() if not r.cancelled]
            if group.members()[2] > 0:
                per_tick = sum(_cells(r) for r in running) / rate_guess
                ticks = max(1, min(512, int(run_ms * 1e-3 / max(per_tick, 1e-7))))
                group.run(ticks)
                group.sync(ahead)
            elif not changed:
                if building or ready or ex_active:
                    sleep(2e-4)
                else:
                    nxt = pending[0].arrival - (clock() - t0) if pending and not members else 0.0
                    sleep(max(2e-4, min(nxt, 0.01)))
        group.sync(0)
    finally:
        if own_pool:
            pool.shutdown(wait=True)
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


def serve_benchmark(rates=(2, 5, 10, 20), count=200, sizes=SIZES, max_slots=8, chunk=64, budget=200e9, seed=0,
                    modes=("plain", "executor"), per_request_media=True, hybrid_ahead=2,
                    log=lambda *a: print(*a, file=sys.stderr, flush=True)):
    """Plain versus batched serving of the same request streams; one entry per rate, with a
    summary per mode ("plain"; "grouped": el_group; "executor": per-slot graph streams;
    "hybrid": large requests on the executor, small ones in the group)."""
    import torch
    from . import el
    wl = Workloads(sizes, per_request_media=per_request_media)
    group = el.Group(max_members=max_slots) if ("grouped" in modes or "hybrid" in modes) else None
    ex = el.Executor(max_slots=min(max_slots, 4), chunk=chunk) if "executor" in modes else None
    # hybrid: its own executor with two slots for the large requests, each holding at most
    # `hybrid_ahead` graph replays in flight.  The group's stream and the executor's share four
    # hardware queues per process; a large request enqueued whole can put the group's small
    # launches behind all of its steps, a bounded number of replays only behind those
    ex_h = el.Executor(max_slots=2, chunk=chunk, ahead=hybrid_ahead) if "hybrid" in modes else None
    runners = {"plain": lambda q: run_plain(q, wl),
               "grouped": lambda q: run_grouped(q, wl, group, budget, max_large=1),
               "executor": lambda q: run_batched(q, wl, ex, budget),
               "hybrid": lambda q: run_grouped(q, wl, group, budget, executor=ex_h)}
    # warm every path on one request per size (kernel loading, allocator growth)
    warm = [Request(rid=-1 - k, op=k % 2, n=n, nsteps=S.serving_steps(n), nrec=256, seed=k, arrival=0.0)
            for k, n in enumerate(sizes)]
    for m in modes:
        runners[m](clone_requests(warm))
    torch.cuda.synchronize()
    out = []
    for k, rate in enumerate(rates):
        reqs = request_mix(count, rate, seed=seed + k, sizes=sizes)
        ent = dict(rate=rate, count=count)
        for m in modes:
            ent[m] = summarize(runners[m](clone_requests(reqs)))
            e = ent[m]
            log(f"[serve] rate {rate}/s {m}: {e['gcells']:.2f} Gcell/s, {e['throughput_rps']:.2f} req/s, "
                f"p50 {e['p50_s']:.2f}s p99 {e['p99_s']:.2f}s")
        base = ent.get("plain", {}).get("gcells")
        ent["throughput_gain"] = {m: ent[m]["gcells"] / base for m in modes if m != "plain"} if base else None
        out.append(ent)
    for h in (group, ex, ex_h):
        if h is not None:
            h.close()
    return out


def main():
    ap = argparse.ArgumentParser(description="plain vs batched serving of H / H^T requests")
    ap.add_argument("--rates", type=float, nargs="+", default=[2, 5, 10, 20])
    ap.add_argument("--count", type=int, default=200)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--modes", nargs="+", default=["plain", "executor"], choices=["plain", "grouped", "executor", "hybrid"])
    ap.add_argument("--shared-media", action="store_true", help="one medium per size instead of one per request")
    ap.add_argument("--hybrid-ahead", type=int, default=2,
                    help="graph replays in flight per executor slot in hybrid mode (0: whole operations)")
    args = ap.parse_args()
    res = serve_benchmark(rates=args.rates, count=args.count, max_slots=args.slots, chunk=args.chunk,
                          budget=args.budget_gb * 1e9, seed=args.seed, modes=tuple(args.modes),
                          per_request_media=not args.shared_media, hybrid_ahead=args.hybrid_ahead)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
