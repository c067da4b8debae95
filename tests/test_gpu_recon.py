"""Penalised reconstruction on the GPU operators against the same iterations on the FP64
oracle.  The reference iterations below are written out separately in NumPy from the two
methods' definitions (FISTA: Beck and Teboulle 2009; PDHG: Chambolle and Pock 2011); only
the operators differ, so the iterates must agree to the operators' parity bound."""
import math

import numpy as np
import pytest
import torch

from oracle.oracle import Model
from paper_1709_02733_amd import el, recon
from paper_1709_02733_amd import scenarios as S
from tests.gpu_util import banner, need_gpu, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu(request):
    need_gpu()
    banner(request.node.nodeid)
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def problem():
    sc = S.skull_scenario(n=40, nsteps=150, nrec=64, seed=6)
    plan = el.Plan.from_scenario(sc)
    ref = Model.from_scenario(sc)
    y = ref.forward(sc.p0.astype(np.float64))
    y += 0.01 * np.abs(y).max() * np.random.default_rng(1).standard_normal(y.shape)
    norm2 = recon.power_norm2(plan, iters=15)
    return sc, plan, ref, y, norm2


def _grad3(p):
    g = np.zeros((3,) + p.shape)
    g[0, :, :, :-1] = np.diff(p, axis=2)
    g[1, :, :-1, :] = np.diff(p, axis=1)
    g[2, :-1, :, :] = np.diff(p, axis=0)
    return g


def _div3(g):
    d = np.zeros(g.shape[1:])
    for a, ax in ((0, 2), (1, 1), (2, 0)):
        n = g.shape[1 + ax]
        head = np.take(g[a], range(n - 1), axis=ax)
        idx0 = [slice(None)] * 3
        idx1 = [slice(None)] * 3
        idx0[ax] = slice(0, n - 1)
        idx1[ax] = slice(1, n)
        d[tuple(idx0)] += head
        d[tuple(idx1)] -= head
    return d


def test_fista_iterates_match_oracle_iterates(problem):
    sc, plan, ref, y, norm2 = problem
    beta, iters = 1e-3 * norm2, 5
    p_gpu, _ = recon.fista(plan, torch.from_numpy(y).to(plan.device), iters, beta=beta, norm2=norm2)
    step = 1.0 / (norm2 + beta)
    x = np.zeros(sc.shape)
    z = x.copy()
    t = 1.0
    for _ in range(iters):
        grad = ref.adjoint(ref.forward(z) - y) + beta * z
        x_new = np.maximum(z - step * grad, 0.0)
        t_new = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
        z = x_new + ((t - 1.0) / t_new) * (x_new - x)
        x, t = x_new, t_new
    e = rel_l2(p_gpu.cpu().numpy(), x)
    banner(f"FISTA 5 iterations, GPU vs oracle iterate: rel L2 {e:.2e}")
    assert e <= 1e-4


def test_tv_pdhg_iterates_match_oracle_iterates(problem):
    sc, plan, ref, y, norm2 = problem
    lam, iters = 1e-3 * math.sqrt(norm2), 5
    p_gpu, _ = recon.tv_pdhg(plan, torch.from_numpy(y).to(plan.device), iters, lam=lam, norm2=norm2)
    c = math.sqrt(norm2 / 12.0)
    tau = sigma = 0.99 / math.sqrt(2.0 * norm2)
    lam_c = lam / c
    p = np.zeros(sc.shape)
    pbar = p.copy()
    q = np.zeros_like(y)
    r = np.zeros((3,) + sc.shape)
    for _ in range(iters):
        q = (q + sigma * (ref.forward(pbar) - y)) / (1.0 + sigma)
        r = r + sigma * c * _grad3(pbar)
        mag = np.sqrt(np.sum(r * r, axis=0, keepdims=True))
        r = r / np.maximum(mag / lam_c, 1.0)
        p_new = np.maximum(p - tau * (ref.adjoint(q) - c * _div3(r)), 0.0)
        pbar = 2.0 * p_new - p
        p = p_new
    e = rel_l2(p_gpu.cpu().numpy(), p)
    banner(f"TV-PDHG 5 iterations, GPU vs oracle iterate: rel L2 {e:.2e}")
    assert e <= 1e-4


def test_reconstruction_reduces_the_objective(problem):
    sc, plan, ref, y, norm2 = problem
    yt = torch.from_numpy(y).to(plan.device)
    f0 = recon.objective(plan, torch.zeros(sc.shape, dtype=plan.dtype, device=plan.device), yt)
    p, hist = recon.fista(plan, yt, 20, norm2=norm2)
    assert hist[-1] < 0.95 * f0
    p, hist = recon.tv_pdhg(plan, yt, 20, lam=1e-3 * math.sqrt(norm2), norm2=norm2)
    assert hist[-1] < f0
