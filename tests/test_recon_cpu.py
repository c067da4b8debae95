"""Reconstruction solvers (paper_1709_02733_amd.recon) on small dense problems with known
minimisers; no GPU.  The solvers only need forward/adjoint actions, so a dense matrix
stands in for H."""
import numpy as np
import pytest
import torch
from scipy.optimize import nnls

from paper_1709_02733_amd import recon


class Dense:
    """p (shape `shape`) -> A p.ravel(); adjoint A^T y reshaped."""

    def __init__(self, A, shape):
        self.A = torch.as_tensor(A, dtype=torch.float64)
        self.shape, self.dtype, self.device = tuple(shape), torch.float64, torch.device("cpu")

    def forward(self, p):
        return self.A @ p.reshape(-1).to(torch.float64)

    def adjoint(self, y):
        return (self.A.T @ y).reshape(self.shape)


def test_grad_div_adjoint_identity():
    g = torch.Generator().manual_seed(0)
    for shape in ((5, 4, 3), (1, 6, 2), (3, 1, 1)):
        p = torch.randn(shape, generator=g, dtype=torch.float64)
        v = torch.randn((3,) + shape, generator=g, dtype=torch.float64)
        lhs = float(torch.sum(recon.grad3(p) * v))
        rhs = -float(torch.sum(p * recon.div3(v)))
        assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs))


def test_grad_of_linear_ramp():
    z, y, x = np.meshgrid(np.arange(3), np.arange(4), np.arange(5), indexing="ij")
    p = torch.as_tensor(2.0 * x - 3.0 * y + 0.5 * z, dtype=torch.float64)
    g = recon.grad3(p)
    assert torch.allclose(g[0, :, :, :-1], torch.tensor(2.0, dtype=torch.float64))
    assert torch.allclose(g[1, :, :-1, :], torch.tensor(-3.0, dtype=torch.float64))
    assert torch.allclose(g[2, :-1, :, :], torch.tensor(0.5, dtype=torch.float64))
    assert torch.all(g[0, :, :, -1] == 0) and torch.all(g[1, :, -1, :] == 0) and torch.all(g[2, -1] == 0)


@pytest.mark.parametrize("beta", [0.0, 0.3])
def test_fista_reaches_the_nonnegative_tikhonov_minimiser(beta):
    """min 0.5||Ap - y||^2 + 0.5 beta ||p||^2, p >= 0 equals NNLS on [A; sqrt(beta) I]."""
    rng = np.random.default_rng(1)
    A = rng.standard_normal((40, 25))
    y = A @ np.abs(rng.standard_normal(25)) * (rng.uniform(size=25) > 0.4).any() + 0.3 * rng.standard_normal(40)
    op = Dense(A, (25,))
    p, hist = recon.fista(op, torch.as_tensor(y), iters=4000, beta=beta, norm2=float(np.linalg.norm(A, 2) ** 2))
    Aa = np.vstack([A, np.sqrt(beta) * np.eye(25)]) if beta else A
    ya = np.concatenate([y, np.zeros(25)]) if beta else y
    ref, _ = nnls(Aa, ya)
    assert np.linalg.norm(p.numpy() - ref) <= 1e-6 * max(np.linalg.norm(ref), 1.0)
    assert (p.numpy() >= 0).all()


def test_fista_meets_its_convergence_bound():
    """Beck and Teboulle (2009, Thm. 4.4): F(x_k) - F* <= 2 L ||x_0 - x*||^2 / (k + 1)^2."""
    rng = np.random.default_rng(2)
    A = rng.standard_normal((30, 20))
    y = rng.standard_normal(30)
    L = float(np.linalg.norm(A, 2) ** 2)
    ref, _ = nnls(A, y)
    fstar = 0.5 * float(np.sum((A @ ref - y) ** 2))
    vals = []
    recon.fista(Dense(A, (20,)), torch.as_tensor(y), iters=200, norm2=L, callback=lambda it, p, f: vals.append(f))
    for k, f in enumerate(vals, start=1):
        assert f - fstar <= 2.0 * L * float(np.sum(ref ** 2)) / (k + 1) ** 2 + 1e-12
    assert vals[-1] - fstar <= 1e-6 * max(fstar, 1.0)


def test_tv_pdhg_closed_forms_for_identity():
    """H = I: with lam = 0 the minimiser is max(y, 0); with lam large it is the constant
    max(mean(y), 0) (total variation forces a constant, the data term picks the mean)."""
    rng = np.random.default_rng(3)
    y = rng.standard_normal((1, 1, 16)) + 0.4
    op = Dense(np.eye(16), (1, 1, 16))
    p0, _ = recon.tv_pdhg(op, torch.as_tensor(y.ravel()), iters=400, lam=0.0, norm2=1.0)
    assert np.allclose(p0.numpy(), np.maximum(y, 0), atol=1e-6)
    lam_big = 2.0 * np.max(np.abs(np.cumsum(y.ravel() - y.mean())))
    p1, hist = recon.tv_pdhg(op, torch.as_tensor(y.ravel()), iters=6000, lam=lam_big, norm2=1.0)
    assert np.allclose(p1.numpy(), max(y.mean(), 0.0), atol=2e-3)


def test_tv_pdhg_objective_decreases_on_a_dense_problem():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((60, 2 * 3 * 4))
    truth = np.zeros((2, 3, 4))
    truth[:, 1:, 2:] = 1.0
    y = A @ truth.ravel() + 0.05 * rng.standard_normal(60)
    op = Dense(A, (2, 3, 4))
    norm2 = float(np.linalg.norm(A, 2) ** 2)
    vals = []
    p, _ = recon.tv_pdhg(op, torch.as_tensor(y), iters=3000, lam=0.5, norm2=norm2,
                         callback=lambda it, p, f: vals.append(f))
    assert vals[-1] < 0.5 * vals[0]
    assert abs(vals[-1] - min(vals)) <= 1e-3 * abs(min(vals))
