"""Penalised least-squares reconstruction on top of H and H^T.

When the pseudo-inverse image is not adequate, the principled alternative the
paper names (Sec. 8) is to minimise a penalised data-fidelity cost, which needs
only repeated actions of the operator pair.  Two standard first-order methods:

* `fista`: min 0.5 ||H p - y||^2 + 0.5 beta ||p||^2 subject to p >= 0
  (Tikhonov and nonnegativity) by FISTA, the accelerated proximal gradient
  method of Beck and Teboulle (2009), with step 1 / (||H||^2 + beta).
* `tv_pdhg`: min 0.5 ||H p - y||^2 + lam ||grad p||_{2,1} subject to p >= 0
  (isotropic total variation) by the primal-dual hybrid gradient method of
  Chambolle and Pock (2011) on K = [H; c grad], tau sigma ||K||^2 < 1.  The
  gradient is scaled by c = ||H|| / sqrt(12) so both blocks of K have the same
  norm bound (||grad||^2 <= 12 in 3-D with unit forward differences).

H and H^T run in the library's kernels (el_forward, el_adjoint); the vector
updates are elementwise torch operations on the operand's device.  `op` is
anything with forward(p) -> traces, adjoint(traces) -> p, and shape, dtype and
device attributes (an el.Plan, or a small dense operator in tests).

    python -m paper_1709_02733_amd.recon      # error and time per iteration at 128^3, 1000 samples
"""
from __future__ import annotations

import json
import math
import sys
import time

import torch


def power_norm2(op, iters: int = 20, seed: int = 0) -> float:
    """||H||_2^2 by power iteration on H^T H (float64 Rayleigh quotients)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.randn(op.shape, generator=g, dtype=torch.float64).to(op.device)
    v = v / torch.linalg.vector_norm(v)
    lam = 0.0
    for _ in range(iters):
        w = op.adjoint(op.forward(v.to(op.dtype))).to(torch.float64)
        lam = float(torch.sum(v * w))
        v = w / torch.linalg.vector_norm(w)
    return lam


def objective(op, p: torch.Tensor, y: torch.Tensor, beta: float = 0.0, lam: float = 0.0) -> float:
    """0.5 ||H p - y||^2 + 0.5 beta ||p||^2 + lam ||grad p||_{2,1} (float64)."""
    r = op.forward(p) - y
    val = 0.5 * float(torch.sum(r.double() * r.double()))
    if beta:
        val += 0.5 * beta * float(torch.sum(p.double() * p.double()))
    if lam:
        g = grad3(p.double())
        val += lam * float(torch.sum(torch.sqrt(torch.sum(g * g, dim=0))))
    return val


def fista(op, y: torch.Tensor, iters: int, beta: float = 0.0, norm2: float | None = None,
          p_init: torch.Tensor | None = None, callback=None, track: bool = True):
    """FISTA for 0.5 ||H p - y||^2 + 0.5 beta ||p||^2, p >= 0.  Returns (p, objectives).
    callback(it, p, objective) after every iteration; track=False skips the objective (one
    more H per iteration) except at the last iteration."""
    if norm2 is None:
        norm2 = power_norm2(op)
    step = 1.0 / (norm2 + beta)
    x = torch.zeros(op.shape, dtype=op.dtype, device=op.device) if p_init is None else p_init.clone()
    z = x.clone()
    t = 1.0
    hist = []
    for it in range(iters):
        r = op.forward(z) - y
        grad = op.adjoint(r).to(op.dtype)
        if beta:
            grad = grad + beta * z
        x_new = torch.clamp(z - step * grad, min=0.0)
        t_new = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
        z = x_new + ((t - 1.0) / t_new) * (x_new - x)
        x, t = x_new, t_new
        hist.append(objective(op, x, y, beta=beta) if (callback is not None and track) or it == iters - 1
                    else float("nan"))
        if callback is not None:
            callback(it, x, hist[-1])
    return x, hist


def grad3(p: torch.Tensor) -> torch.Tensor:
    """Forward differences along x, y, z of a [nz][ny][nx] field (zero across the last face):
    returns [3][nz][ny][nx] with components (d/dx, d/dy, d/dz)."""
    g = torch.zeros((3,) + tuple(p.shape), dtype=p.dtype, device=p.device)
    g[0, :, :, :-1] = p[:, :, 1:] - p[:, :, :-1]
    g[1, :, :-1, :] = p[:, 1:, :] - p[:, :-1, :]
    g[2, :-1, :, :] = p[1:, :, :] - p[:-1, :, :]
    return g


def div3(g: torch.Tensor) -> torch.Tensor:
    """Negative adjoint of grad3: <grad3 p, g> = -<p, div3 g>."""
    d = torch.zeros(g.shape[1:], dtype=g.dtype, device=g.device)
    for a, dim in ((0, 2), (1, 1), (2, 0)):
        n = g[a].shape[dim]
        if n < 2:
            continue
        head = g[a].narrow(dim, 0, n - 1)        # g_0 .. g_{n-2}; g_{n-1} meets no difference
        d.narrow(dim, 0, n - 1).add_(head)
        d.narrow(dim, 1, n - 1).sub_(head)
    return d


def tv_pdhg(op, y: torch.Tensor, iters: int, lam: float, norm2: float | None = None,
            p_init: torch.Tensor | None = None, callback=None, track: bool = True, ratio: float = 1.0):
    """Primal-dual hybrid gradient for 0.5 ||H p - y||^2 + lam TV(p), p >= 0.
    Returns (p, objectives); callback and track as for fista.  ratio = tau / sigma (the
    step sizes keep tau sigma ||K||^2 = 0.98, the convergence condition of the method)."""
    if norm2 is None:
        norm2 = power_norm2(op)
    c = math.sqrt(norm2 / 12.0)              # ||c grad||^2 <= norm2
    knorm = math.sqrt(2.0 * norm2)           # ||K||^2 <= ||H||^2 + ||c grad||^2
    tau = 0.99 * math.sqrt(ratio) / knorm
    sigma = 0.99 / (math.sqrt(ratio) * knorm)
    lam_c = lam / c                          # lam ||grad p|| = lam_c ||c grad p||
    p = torch.zeros(op.shape, dtype=op.dtype, device=op.device) if p_init is None else p_init.clone()
    pbar = p.clone()
    q = torch.zeros_like(y)                                            # dual of the data term
    r = torch.zeros((3,) + tuple(op.shape), dtype=op.dtype, device=op.device)   # dual of the TV term
    hist = []
    for it in range(iters):
        # dual steps: prox of sigma f* with f = 0.5 ||. - y||^2, and projection onto |r| <= lam_c
        q = (q + sigma * (op.forward(pbar) - y)) / (1.0 + sigma)
        if lam_c > 0:
            r = r + sigma * c * grad3(pbar)
            mag = torch.sqrt(torch.sum(r * r, dim=0, keepdim=True))
            r = r / torch.clamp(mag / lam_c, min=1.0)
        # primal step: p - tau K^T (q, r), projected onto p >= 0
        kt = op.adjoint(q).to(op.dtype) - c * div3(r)
        p_new = torch.clamp(p - tau * kt, min=0.0)
        pbar = 2.0 * p_new - p
        p = p_new
        hist.append(objective(op, p, y, lam=lam) if (callback is not None and track) or it == iters - 1
                    else float("nan"))
        if callback is not None:
            callback(it, p, hist[-1])
    return p, hist


def backprojection_error(op, y: torch.Tensor, p_true: torch.Tensor) -> float:
    """Relative error of the best multiple c H^T y of the adjoint image (the plain H^T
    reconstruction, whose scale is arbitrary): c = <H^T y, p> / ||H^T y||^2."""
    b = op.adjoint(y).double()
    p = p_true.double()
    c = float(torch.sum(b * p) / torch.sum(b * b))
    return float(torch.linalg.vector_norm(c * b - p) / torch.linalg.vector_norm(p))


def main():
    """Reconstruction study at 128^3 (1000 samples, 512 receivers on a hemisphere, skull
    medium): relative error of the adjoint image and of FISTA / TV-PDHG iterates against the
    true p0, from noiseless and 1%-noise data, and the time per iteration."""
    import argparse
    from . import el
    from . import scenarios as S
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--checkpoints", type=int, nargs="+", default=[10, 25, 50, 100, 200])
    ap.add_argument("--noise", type=float, default=0.01, help="Gaussian noise, relative to the traces' RMS")
    ap.add_argument("--tv", type=float, default=None, help="TV weight (default: 3e-4 of ||H^T y||_inf)")
    ap.add_argument("--tv-ratio", type=float, default=3000.0,
                    help="TV-PDHG step ratio tau / sigma (at 128^3: 0.885 / 0.755 / 0.623 / 0.588 / 0.565 / 0.547 "
                         "relative error after 100 iterations for 1 / 10 / 100 / 300 / 1000 / 3000)")
    ap.add_argument("--sweep", action="store_true", help="only TV-PDHG, 100 iterations for each --sweep-ratios")
    ap.add_argument("--sweep-ratios", type=float, nargs="+", default=[1.0, 10.0, 100.0])
    args = ap.parse_args()
    sc = S.make("skull128")
    plan = el.Plan.from_scenario(sc)
    p_true = torch.from_numpy(sc.p0).to(plan.device)
    y = plan.forward(p_true)
    g = torch.Generator(device="cpu").manual_seed(11)
    rms = float(torch.sqrt(torch.mean(y * y)))
    y = y + args.noise * rms * torch.randn(y.shape, generator=g, dtype=y.dtype).to(y.device)
    norm2 = power_norm2(plan, iters=10)
    pn = float(torch.linalg.vector_norm(p_true.double()))
    err = lambda p: float(torch.linalg.vector_norm(p.double() - p_true.double()) / pn)
    lam = args.tv if args.tv is not None else 3e-4 * float(plan.adjoint(y).abs().max())
    out = {"workload": f"{sc.nx}x{sc.ny}x{sc.nz}, M={sc.nsteps}, L={sc.nrec}, noise {args.noise:g} of RMS",
           "norm2": norm2, "backprojection_rel_err": backprojection_error(plan, y, p_true), "tv_lambda": lam}
    print(f"[recon] scaled H^T y: rel. error {out['backprojection_rel_err']:.3f}", file=sys.stderr, flush=True)
    if args.sweep:
        sweep = []
        for ratio in args.sweep_ratios:
            for scale in (1.0,):
                p, _ = tv_pdhg(plan, y, 100, lam * scale, norm2=norm2, ratio=ratio)
                sweep.append({"ratio": ratio, "lam": lam * scale, "rel_err_100": err(p)})
                print(f"[recon] tv_pdhg ratio {ratio:g} lam x{scale:g}: rel. error {err(p):.3f} after 100",
                      file=sys.stderr, flush=True)
        out["tv_sweep"] = sweep
        print(json.dumps(out))
        return
    for name, fn, kw in (("fista", fista, {"beta": 1e-4 * norm2}),
                         ("tv_pdhg", tv_pdhg, {"lam": lam, "ratio": args.tv_ratio})):
        errs = {}

        def cb(it, p, _obj):
            if it + 1 in args.checkpoints:
                errs[it + 1] = err(p)
                print(f"[recon] {name} iteration {it + 1}: rel. error {errs[it + 1]:.3f}", file=sys.stderr, flush=True)

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p, hist = fn(plan, y, args.iters, norm2=norm2, callback=cb, track=False, **kw)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.iters
        out[name] = {"s_per_iter": dt, "gcell_updates_per_s": 2 * sc.ncells * (sc.nsteps - 1) / dt / 1e9,
                     "objective_final": hist[-1], "rel_err": errs, **kw}
        print(f"[recon] {name}: {dt * 1e3:.1f} ms/iteration, final objective {hist[-1]:.4e}", file=sys.stderr,
              flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
