"""Benchmark of the forward operator H and its adjoint H^T on one MI355X.

One step = one forward application H p0 followed by one adjoint application
H^T y (y = the forward traces) on the 384^3 skull workload: 2500 trace
samples, 16-cell C-PML, 1024 receivers, FP32 fields, FP64 traces.  Inputs are
resident in HBM before the timed region starts.  The JSON line reports
cell-updates per second over both operators (2 N (M - 1) per step), the
roofline of the dominant kernel (algorithmic bytes per launch over its mean
launch time, both measured inside the timed region) and the FP64 CPU oracle
timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gcell-updates/s (fwd+adj) & % HBM roofline, 384^3; serving p50/p99 vs plain"
HBM_PEAK_GBS = 8000.0
KERNEL_SRCS = [os.path.join(ROOT, "paper_1709_02733_amd", "csrc", f) for f in ("el_stencil.hip", "el_impl.h", "el_api.hip")]
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha1() -> str:
    """Hash of the stencil kernels' sources and of their tiling (el_api.hip), with comments
    and blank space removed: the counters are valid for this version of the code only."""
    h = hashlib.sha1()
    for fn in KERNEL_SRCS:
        with open(fn) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """Per-launch HBM bytes of a kernel from the committed counter summary, or None
    when the summary is missing or was taken on another version of the kernels."""
    try:
        with open(TRAFFIC_JSON) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    ent = t.get("kernels", {}).get(kernel)
    if not ent or t.get("workload") != workload or t.get("kernel_source_sha1") != kernel_source_sha1():
        return None
    return ent.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def lscpu_model() -> str:
    """The CPU model as lscpu names it (falls back to /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return cpu_model()


def _omp_set_threads(n: int) -> None:
    """Thread count of the oracle's later OpenMP parallel regions (libgomp's own setter)."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def _time_ops(m, p0, y, nsteps: int, repeats: int, warmup: bool):
    """Best wall time of the oracle's forward and adjoint (timed separately) over `repeats`
    runs, after one untimed run of each when warmup is set."""
    if warmup:
        m.forward(p0, nsteps=nsteps)
        m.adjoint(y, nsteps=nsteps)
    tf, ta = [], []
    for _ in range(repeats):
        t0 = time.perf_counter()
        m.forward(p0, nsteps=nsteps)
        t1 = time.perf_counter()
        m.adjoint(y, nsteps=nsteps)
        t2 = time.perf_counter()
        tf.append(t1 - t0)
        ta.append(t2 - t1)
    return min(tf), min(ta)


def cpu_baseline(sc, full: bool):
    """The FP64 stencil oracle (plain C, OpenMP over z) on the host cores.

    Main figure (`value`): the benchmark's own workload sc on every host core, a bounded
    sample of 2 forward and 2 adjoint updates (one run each).  Beside it, the 64^3 /
    400-sample parity workload (water with a solid spherical shell, 3 balls, 128
    receivers), forward and adjoint timed separately, best of 3 after one warm-up, on every
    host core, and a one-thread sample of that grid (29 updates each way, one run).  With
    `full`, the 96^3 / 600-sample skull cross-check as well, on every core and on one
    thread (best of 3 after a warm-up each)."""
    import numpy as np
    from oracle import oracle as O
    from paper_1709_02733_amd import scenarios as S

    ncores = os.cpu_count() or 1
    host = {"nproc": ncores, "lscpu_model": lscpu_model(), "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}

    def measure(sc, nsteps, threads, repeats, warmup):
        _omp_set_threads(threads)
        m = O.Model.from_scenario(sc)
        p0 = sc.p0.astype(np.float64)
        y = m.forward(p0, nsteps=nsteps)
        used = O.num_threads()
        tf, ta = _time_ops(m, p0, y, nsteps, repeats, warmup)
        upd = sc.ncells * (nsteps - 1)
        r = {"workload": f"{sc.name} {sc.nx}x{sc.ny}x{sc.nz}, M={nsteps}", "threads": used,
             "forward_s": tf, "adjoint_s": ta, "forward_gcells": upd / tf / 1e9, "adjoint_gcells": upd / ta / 1e9,
             "both_gcells": 2 * upd / (tf + ta) / 1e9,
             "timing": f"best of {repeats}" + (" after one warm-up" if warmup else ", no warm-up")}
        log(f"[cpu] {r['workload']} threads {used}: forward {tf:.2f}s ({r['forward_gcells']:.4f} Gcell/s), "
            f"adjoint {ta:.2f}s ({r['adjoint_gcells']:.4f} Gcell/s)")
        return r

    t0 = time.perf_counter()
    main_r = measure(sc, 3, ncores, 1, False)
    c1 = S.make("parity64")
    runs = [main_r, measure(c1, c1.nsteps, ncores, 3, True), measure(c1, 30, 1, 1, False)]
    if full:
        c3 = S.make("skull96")
        runs.append(measure(c3, c3.nsteps, ncores, 3, True))
        runs.append(measure(c3, c3.nsteps, 1, 3, True))
    _omp_set_threads(ncores)
    return {
        "value": main_r["both_gcells"],
        "unit": "Gcell-updates/s",
        "cores": main_r["threads"],
        "kind": "oracle",
        "sample": (f"{sc.nx}x{sc.ny}x{sc.nz} benchmark workload, 2 forward + 2 adjoint updates (one run each, "
                   f"{4 * sc.ncells:.3e} cell-updates) on {main_r['threads']} OpenMP threads; runs[1]: the 64^3 / "
                   f"400-sample parity workload, forward and adjoint timed separately, best of 3 after a warm-up, "
                   f"all threads; runs[2]: one thread on that grid (29 updates each way)"
                   + ("; runs[3:5]: the 96^3 / 600-sample skull cross-check on all threads and on one thread"
                      if full else "")),
        "cpu": host["lscpu_model"],
        "host": host,
        "runs": runs,
        "seconds": time.perf_counter() - t0,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="skull384")
    ap.add_argument("--nsteps", type=int, default=0, help="override the trace length M (diagnostics only)")
    ap.add_argument("--timing-every", type=int, default=10,
                    help="bracket the kernel launches of every n-th time step with HIP events (1: all)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle on the 96^3 / 600-sample cross-check (all cores and one thread; "
                         "several minutes)")
    ap.add_argument("--no-serving", action="store_true", help="skip the plain vs batched serving comparison")
    ap.add_argument("--no-general", action="store_true",
                    help="skip the general-update measurement (the workload with the fluid update off)")
    ap.add_argument("--no-fd", action="store_true",
                    help="skip the frequency-dependent absorption measurement (the workload with relaxation "
                         "mechanisms in the skull)")
    ap.add_argument("--serving-rates", type=float, nargs="+", default=[2.0, 10.0])
    ap.add_argument("--serving-count", type=int, default=40)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run an elementwise kernel three times over 256 MiB of floats (read and write of "
                         "known size: the reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only; the operator is not sharded across GPUs "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1709_02733_amd import bytemodel, el
    from paper_1709_02733_amd import scenarios as S

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.abs(src, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] counter calibration: 3 elementwise passes reading and writing {src.numel() * 4} bytes")
        del src, dst
    t0 = time.time()
    over = {"nsteps": args.nsteps} if args.nsteps else {}
    sc = S.make(args.workload, **over)
    log(f"[bench] workload {sc.name}: {sc.nx}x{sc.ny}x{sc.nz}, M={sc.nsteps}, L={sc.nrec}, npml={sc.npml}, "
        f"dt={sc.dt:.4e}s, generated in {time.time() - t0:.1f}s")
    plan = el.Plan.from_scenario(sc)
    fl = plan.fluid_stats()
    fluid_cells, fluid_layer = fl["cells"], fl["layer_cells"]
    skipped, uniform = fl["skipped_stores"], fl["uniform_cells"]
    log(f"[bench] fluid tiles: {fl['tiles']} ({fluid_cells / sc.ncells:.1%} of the cells take the fluid update; "
        f"{fluid_layer} fluid C-PML cell-axis pairs; {skipped} s22/s33 stores left out per stress pass; "
        f"{uniform / sc.ncells:.1%} of the cells take lambda, rho, alpha from the per-tile table)")
    dev = plan.device
    p0 = torch.from_numpy(sc.p0).to(dev)
    traces = torch.empty((sc.nsteps, sc.nrec), dtype=torch.float64, device=dev)
    padj = torch.empty(sc.shape, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    for w in range(args.warmup):
        plan.forward(p0, out=traces)
        plan.adjoint(traces, out=padj)
        torch.cuda.synchronize()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")

    plan.timing(True, every=args.timing_every)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record()
        plan.forward(p0, out=traces)
        ev[k][1].record()
        plan.adjoint(traces, out=padj)
        ev[k][2].record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_start
    plan.timing(False)
    kt = plan.kernel_times()
    fwd_ms = sum(e[0].elapsed_time(e[1]) for e in ev)
    adj_ms = sum(e[1].elapsed_time(e[2]) for e in ev)
    total_ms = fwd_ms + adj_ms
    upd = sc.ncells * (sc.nsteps - 1)
    value = 2 * upd * args.steps / (total_ms / 1e3) / 1e9
    log(f"[bench] timed {args.steps} step(s): forward {fwd_ms / args.steps:.1f} ms, adjoint "
        f"{adj_ms / args.steps:.1f} ms per step, wall {t_wall:.2f}s")
    assert torch.isfinite(traces).all() and torch.isfinite(padj).all()

    # dominant kernel and its roofline
    per = {}
    for name, (n, ms) in kt.items():
        if n == 0:
            continue
        b = bytemodel.kernel_bytes(name, sc.nx, sc.ny, sc.nz, sc.npml, sc.nrec, 4, fluid_cells, fluid_layer,
                                   skipped, uniform)
        avg = ms / n
        per[name] = dict(launches=n, total_ms=ms, avg_us=avg * 1e3, bytes_per_launch=b,
                         gbs=b / (avg / 1e3) / 1e9)
        log(f"[bench] {name:13s} {n:6d} launches  avg {avg * 1e3:9.2f} us  {per[name]['gbs']:8.1f} GB/s")
    dom = max(per, key=lambda k: per[k]["total_ms"])
    d = per[dom]
    traffic = measured_traffic(dom, sc.name)
    roofline = {"bound": "hbm", "achieved": d["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": d["gbs"] / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                "bytes_per_launch": d["bytes_per_launch"], "avg_launch_us": d["avg_us"],
                "timed_launches": d["launches"], "timing_every": args.timing_every}
    step_gb = sum(bytemodel.step_bytes(op, sc.nx, sc.ny, sc.nz, sc.npml, sc.nrec, 4, fluid_cells, fluid_layer,
                                       skipped, uniform) for op in ("fwd", "adj")) * (sc.nsteps - 1)
    whole_gbs = step_gb * args.steps / (total_ms / 1e3) / 1e9

    general = None
    if not args.no_general:
        # the same workload with the fluid update off: every cell takes the general (elastic)
        # update, whose algorithmic bytes are the dense model's (136 B forward, 142 B adjoint
        # per cell-update at this C-PML thickness)
        plan.fluid_path(False)
        plan.forward(p0, out=traces)          # one untimed operation in the new tile order
        torch.cuda.synchronize()
        plan.timing(True, every=args.timing_every)
        g0, g1, g2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        g0.record()
        plan.forward(p0, out=traces)
        g1.record()
        plan.adjoint(traces, out=padj)
        g2.record()
        torch.cuda.synchronize()
        plan.timing(False)
        gk = plan.kernel_times()
        plan.fluid_path(True)
        gf_ms, ga_ms = g0.elapsed_time(g1), g1.elapsed_time(g2)
        gper = {}
        for name, (n, ms) in gk.items():
            if n == 0:
                continue
            b = bytemodel.kernel_bytes(name, sc.nx, sc.ny, sc.nz, sc.npml, sc.nrec, 4, 0, 0, 0, 0)
            avg = ms / n
            gper[name] = {"avg_us": avg * 1e3, "gbs": b / (avg / 1e3) / 1e9, "launches": n,
                          "bytes_per_launch": b, "frac": b / (avg / 1e3) / 1e9 / HBM_PEAK_GBS}
            log(f"[bench] general {name:13s} {n:6d} launches  avg {avg * 1e3:9.2f} us  {gper[name]['gbs']:8.1f} GB/s")
        gdom = max(gper, key=lambda k: gper[k]["avg_us"] * gper[k]["launches"])
        general = {"value": 2 * upd / ((gf_ms + ga_ms) / 1e3) / 1e9, "unit": "Gcell-updates/s",
                   "fwd_gcells": upd / (gf_ms / 1e3) / 1e9, "adj_gcells": upd / (ga_ms / 1e3) / 1e9,
                   "ms_per_step": gf_ms + ga_ms, "steps": 1,
                   "byte_model": "dense: every cell at the general update's bytes",
                   "roofline": {"bound": "hbm", "kernel": gdom, "achieved": gper[gdom]["gbs"], "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": gper[gdom]["frac"]},
                   "kernels": gper}
        log(f"[bench] general update only: forward {gf_ms:.1f} ms, adjoint {ga_ms:.1f} ms, "
            f"{general['value']:.1f} Gcell-updates/s")

    freqdep = None
    if not args.no_fd:
        # the same workload with the skull's absorption given by two relaxation mechanisms
        # (frequency-dependent absorption): one forward + one adjoint, sampled kernel timing
        plan = None
        torch.cuda.empty_cache()
        t0 = time.time()
        scf = S.make(args.workload + "fd", **over)
        planf = el.Plan.from_scenario(scf)
        rtiles, rcells, rpoints = planf.relaxation_extent()
        log(f"[bench] {scf.name}: {len(scf.mechanisms)} mechanisms, relaxation on {rtiles} tiles, {rpoints} "
            f"velocity points (set up in {time.time() - t0:.1f}s)")
        p0f = torch.from_numpy(scf.p0).to(dev)
        planf.forward(p0f, out=traces)
        torch.cuda.synchronize()
        planf.timing(True, every=args.timing_every)
        f0, f1, f2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        f0.record()
        planf.forward(p0f, out=traces)
        f1.record()
        planf.adjoint(traces, out=padj)
        f2.record()
        torch.cuda.synchronize()
        planf.timing(False)
        fk = planf.kernel_times()
        ff_ms, fa_ms = f0.elapsed_time(f1), f1.elapsed_time(f2)
        n_r, ms_r = fk.get("relax", (0, 0.0))
        rb = bytemodel.relax_bytes(rpoints, len(scf.mechanisms), 4)
        r_us = ms_r / max(n_r, 1) * 1e3
        freqdep = {"workload": f"{scf.name}: the skull's absorption as relaxation mechanisms "
                               f"{[(round(o / 2 / 3.141592653589793 / 1e6, 3), w) for o, w in scf.mechanisms]} "
                               f"(MHz, weight), water diffusive",
                   "value": 2 * upd / ((ff_ms + fa_ms) / 1e3) / 1e9, "unit": "Gcell-updates/s",
                   "ms_per_step": ff_ms + fa_ms, "fwd_ms": ff_ms, "adj_ms": fa_ms,
                   "relax": {"tiles": rtiles, "cells": rcells, "points": rpoints, "launches": n_r, "avg_us": r_us,
                             "bytes_per_launch": rb, "gbs": rb / (r_us / 1e6) / 1e9 if n_r else None},
                   "kernels_us": {k: v[1] / v[0] * 1e3 for k, v in fk.items() if v[0]}}
        log(f"[bench] frequency-dependent: forward {ff_ms:.1f} ms, adjoint {fa_ms:.1f} ms, "
            f"{freqdep['value']:.1f} Gcell-updates/s; relaxation {r_us:.1f} us/launch")
        del planf, p0f
        torch.cuda.empty_cache()

    serving = None
    if not args.no_serving:
        from paper_1709_02733_amd import serving as SV
        del plan, p0, traces, padj
        torch.cuda.empty_cache()
        modes = ("plain", "executor", "grouped")
        res = SV.serve_benchmark(rates=args.serving_rates, count=args.serving_count, modes=modes, log=log)
        keys = ("gcells", "throughput_rps", "p50_s", "p99_s")
        serving = {"requests_per_rate": args.serving_count,
                   "mix": "96^3/128^3/192^3/256^3 skull media (one per request: shifted up to 4 cells, "
                          "speeds and density scaled up to 3%), 800-1800 samples, 256-1024 receivers, "
                          "60% forward / 40% adjoint, Poisson arrivals, 200 GB HBM budget; plain = one "
                          "request at a time through el_forward/el_adjoint; executor = el_exec with 4 slots "
                          "(a stream each, captured 64-step graphs); grouped = el_group with 8 slots (up to 4 "
                          "requests per launch, at most one request of >= 4M cells, plans built on a worker thread)",
                   "rates": [dict({m: {k: e[m][k] for k in keys} for m in modes}, rate=e["rate"],
                                  throughput_gain=e["throughput_gain"]) for e in res]}

    cpu = None
    if not args.no_cpu:
        torch.cuda.empty_cache()
        cpu = cpu_baseline(sc, args.cpu_full)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{sc.name}: {sc.nx}x{sc.ny}x{sc.nz} cells, dx {sc.dx * 1e3:.2f} mm, "
                               f"M={sc.nsteps} samples, npml={sc.npml}, L={sc.nrec} receivers, "
                               f"forward H + adjoint H^T per step",
                   "nx": sc.nx, "ny": sc.ny, "nz": sc.nz, "nsteps": sc.nsteps, "npml": sc.npml,
                   "nrec": sc.nrec, "seed": sc.seed, "fluid_tile_cells": fluid_cells,
                   "fluid_layer_cells": fluid_layer, "fluid_skipped_stores": skipped,
                   "fluid_uniform_cells": uniform},
        "fwd_gcells": upd * args.steps / (fwd_ms / 1e3) / 1e9,
        "adj_gcells": upd * args.steps / (adj_ms / 1e3) / 1e9,
        "whole_step_gbs": whole_gbs,
        "roofline": roofline,
        "kernels": {k: {"avg_us": v["avg_us"], "gbs": v["gbs"], "launches": v["launches"]} for k, v in per.items()},
        "general_path": general,
        "frequency_dependent": freqdep,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
