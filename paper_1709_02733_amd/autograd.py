"""Differentiation through the forward operator H with its hand-written adjoint.

The paper's reconstruction problem (Sec. 2.3) asks for p0 from p_hat = H p0;
iterative methods need repeated actions of H and of its adjoint (Sec. 2.3,
Sec. 8).  `ElasticH` wraps one plan as a torch.autograd.Function: forward is
H (el_forward), backward is H^T (el_adjoint).  H is linear in p0, so the
vector-Jacobian product of the traces with respect to p0 is exactly H^T g and
no forward wavefield needs to be kept.

`power_norm2` estimates ||H||^2 (largest eigenvalue of H^T H) by power
iteration, and `projected_gradient` runs projected gradient descent on
0.5 ||H p0 - y||^2 subject to p0 >= 0 with step 1 / ||H||^2.
"""
from __future__ import annotations

import torch

from . import el


class ElasticH(torch.autograd.Function):
    """traces = H p0 (float64 [M][L]); gradient w.r.t. p0 = H^T grad_traces."""

    @staticmethod
    def forward(ctx, p0: torch.Tensor, plan: "el.Plan"):
        ctx.plan = plan
        ctx.in_dtype = p0.dtype
        return plan.forward(p0.detach())

    @staticmethod
    def backward(ctx, grad_traces: torch.Tensor):
        g = ctx.plan.adjoint(grad_traces.detach().to(torch.float64).contiguous())
        return g.to(ctx.in_dtype), None


def apply_H(p0: torch.Tensor, plan: "el.Plan") -> torch.Tensor:
    return ElasticH.apply(p0, plan)


def loss_and_grad(plan: "el.Plan", p: torch.Tensor, y: torch.Tensor):
    """0.5 ||H p - y||^2 and its gradient H^T (H p - y), via autograd."""
    x = p.detach().clone().requires_grad_(True)
    r = apply_H(x, plan) - y
    loss = 0.5 * torch.sum(r * r)
    loss.backward()
    return loss.detach(), x.grad.detach()


def power_norm2(plan: "el.Plan", iters: int = 20, seed: int = 0) -> float:
    """||H||_2^2 by power iteration on H^T H (float64 Rayleigh quotients)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.randn(plan.shape, generator=g, dtype=torch.float64).to(plan.device)
    v = v / torch.linalg.vector_norm(v)
    lam = 0.0
    for _ in range(iters):
        w = plan.adjoint(plan.forward(v.to(plan.dtype))).to(torch.float64)
        lam = float(torch.sum(v * w))
        v = w / torch.linalg.vector_norm(w)
    return lam


def projected_gradient(plan: "el.Plan", y: torch.Tensor, iters: int = 50, step: float | None = None,
                       p_init: torch.Tensor | None = None, callback=None):
    """min 0.5 ||H p - y||^2 s.t. p >= 0 by projected gradient descent, step 1/||H||^2."""
    if step is None:
        step = 1.0 / power_norm2(plan)
    p = torch.zeros(plan.shape, dtype=plan.dtype, device=plan.device) if p_init is None else p_init.clone()
    history = []
    for it in range(iters):
        loss, grad = loss_and_grad(plan, p, y)
        history.append(float(loss))
        p = torch.clamp(p - step * grad, min=0.0)
        if callback is not None:
            callback(it, p, float(loss))
    return p, history, step
