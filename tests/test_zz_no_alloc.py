"""The allocation-free inner product el_dot_f64_noalloc, called through the C ABI, against
el_dot_f64 (the same kernels with the partial sums in the plan's workspace): equal results,
on two calls in a row, the second with a smaller input."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1709_02733_amd import el
from paper_1709_02733_amd import scenarios as S
from tests.gpu_util import banner, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu(request):
    need_gpu()
    banner(request.node.nodeid)
    yield
    torch.cuda.synchronize()


def _noalloc(prec, a, b):
    # straight through the C ABI (the binding el.dot_noalloc marshals the same call)
    out = torch.full((), float("nan"), dtype=torch.float64, device=a.device)
    st = el.lib().el_dot_f64_noalloc(prec, a.numel(), ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == el.EL_OK, el.lib().el_last_error().decode()
    return out


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_noalloc_dot_equals_workspace_dot(precision):
    prec = el.EL_F64 if precision == "f64" else el.EL_F32
    g = torch.Generator().manual_seed(11)
    for shape in ((41, 37, 29), (9, 8, 7)):          # the second call is smaller
        sc = S.random_scenario(shape[::-1], seed=2, nsteps=5, npml=0, nrec=3)
        plan = el.Plan.from_scenario(sc, precision=precision)
        a = torch.randn(sc.shape, generator=g, dtype=plan.dtype).to(plan.device)
        b = torch.randn(sc.shape, generator=g, dtype=plan.dtype).to(plan.device)
        ref = plan.dot(a, b, 0)
        got = _noalloc(prec, a, b)
        exact = float(np.dot(a.cpu().double().numpy().ravel(), b.cpu().double().numpy().ravel()))
        banner(f"{precision} {shape}: noalloc {float(got):.17g} workspace {float(ref):.17g}")
        assert torch.equal(got, ref)                 # same kernels, same reduction order
        assert torch.equal(el.dot_noalloc(a.reshape(-1), b.reshape(-1)), ref)
        assert abs(float(got) - exact) <= 1e-12 * float(torch.linalg.norm(a.double()) * torch.linalg.norm(b.double()))
    # traces (double) through the same call
    y = torch.randn(300, 7, generator=g, dtype=torch.float64).cuda()
    z = torch.randn(300, 7, generator=g, dtype=torch.float64).cuda()
    assert abs(float(_noalloc(el.EL_F64, y, z)) - float((y * z).sum())) <= 1e-12 * float(y.norm() * z.norm())
    # empty input, and the documented rejections
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    assert float(_noalloc(el.EL_F64, e, e)) == 0.0
    L = el.lib()
    vp = ctypes.c_void_p
    out = torch.empty((), dtype=torch.float64, device="cuda")
    assert L.el_dot_f64_noalloc(el.EL_F64, -1, vp(y.data_ptr()), vp(z.data_ptr()), vp(out.data_ptr()), None) == el.EL_EINVAL
    assert L.el_dot_f64_noalloc(el.EL_F64, (1 << 40) + 1, vp(y.data_ptr()), vp(z.data_ptr()), vp(out.data_ptr()),
                                None) == el.EL_EINVAL
    assert L.el_dot_f64_noalloc(5, 4, vp(y.data_ptr()), vp(z.data_ptr()), vp(out.data_ptr()), None) == el.EL_EINVAL
    assert L.el_dot_f64_noalloc(el.EL_F64, 4, None, vp(z.data_ptr()), vp(out.data_ptr()), None) == el.EL_EINVAL
