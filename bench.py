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


def cpu_baseline(sc, sample_steps: int):
    """FP64 oracle on the same grid and medium: (sample_steps - 1) forward and as many
    adjoint updates, reported in Gcell-updates/s."""
    import numpy as np
    from oracle import oracle as O
    t0 = time.time()
    m = O.Model.from_scenario(sc)
    log(f"[cpu] oracle model built in {time.time() - t0:.1f}s, threads {O.num_threads()}")
    p0 = sc.p0.astype(np.float64)
    t0 = time.perf_counter()
    tr = m.forward(p0, nsteps=sample_steps)
    t1 = time.perf_counter()
    m.adjoint(tr, nsteps=sample_steps)
    t2 = time.perf_counter()
    updates = 2 * sc.ncells * (sample_steps - 1)
    log(f"[cpu] forward {t1 - t0:.1f}s adjoint {t2 - t1:.1f}s")
    return {
        "value": updates / (t2 - t0) / 1e9,
        "unit": "Gcell-updates/s",
        "cores": O.num_threads(),
        "kind": "oracle",
        "sample": (f"{sc.nx}x{sc.ny}x{sc.nz} skull medium, {sample_steps - 1} forward + {sample_steps - 1} "
                   f"adjoint updates (FP64 stencil oracle, OpenMP), {updates:.3e} cell-updates"),
        "cpu": cpu_model(),
        "seconds": t2 - t0,
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
    ap.add_argument("--cpu-sample-steps", type=int, default=3)
    ap.add_argument("--no-serving", action="store_true", help="skip the plain vs batched serving comparison")
    ap.add_argument("--serving-rates", type=float, nargs="+", default=[2.0, 10.0])
    ap.add_argument("--serving-count", type=int, default=16)
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

    serving = None
    if not args.no_serving:
        from paper_1709_02733_amd import serving as SV
        del plan, p0, traces, padj
        torch.cuda.empty_cache()
        res = SV.serve_benchmark(rates=args.serving_rates, count=args.serving_count, log=log)
        serving = {"requests_per_rate": args.serving_count,
                   "mix": "96^3/128^3/192^3/256^3 skull media, 800-1800 samples, 256-1024 receivers, "
                          "60% forward / 40% adjoint, Poisson arrivals, 4 executor slots, 64-step graphs, "
                          "200 GB HBM budget",
                   "rates": [{"rate": e["rate"],
                              "plain": {k: e["plain"][k] for k in ("gcells", "throughput_rps", "p50_s", "p99_s")},
                              "batched": {k: e["batched"][k] for k in ("gcells", "throughput_rps", "p50_s", "p99_s")},
                              "throughput_gain": e["throughput_gain"]} for e in res]}

    cpu = None
    if not args.no_cpu:
        torch.cuda.empty_cache()
        cpu = cpu_baseline(sc, args.cpu_sample_steps)

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
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
