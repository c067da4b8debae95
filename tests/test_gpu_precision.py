"""Precision study: FP32 stencils against FP64 (on the GPU and in the CPU oracle).

Traces and inner products are accumulated in FP64 in both GPU paths.  The
FP32 path must stay within 1e-4 relative L2 of the FP64 reference on traces
and on H^T y, and its dot-product test within 1e-5; the FP64 GPU path must
match the FP64 oracle to 1e-11.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Model
from paper_1709_02733_amd import el
from paper_1709_02733_amd import scenarios as S
from tests.gpu_util import banner, need_gpu, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu(request):
    need_gpu()
    banner(request.node.nodeid)
    yield
    torch.cuda.synchronize()


def _dot_residual(plan, sc, seed):
    g = torch.Generator().manual_seed(seed)
    p = torch.randn(sc.shape, generator=g, dtype=torch.float64).to(plan.device, plan.dtype)
    q = torch.randn(sc.shape, generator=g, dtype=torch.float64).to(plan.device, plan.dtype)
    y = plan.forward(q)
    lhs = float(plan.dot(plan.forward(p), y, 1))
    rhs = float(plan.dot(p, plan.adjoint(y), 0))
    return abs(lhs - rhs) / abs(lhs)


def test_precision_96_against_oracle():
    """96^3, 600 samples: both GPU precisions against the FP64 CPU oracle."""
    sc = S.make("skull96")
    ref = Model.from_scenario(sc)
    tr_ref = ref.forward(sc.p0.astype(np.float64))
    y = tr_ref
    pa_ref = ref.adjoint(y)
    out = {}
    for prec in ("f32", "f64"):
        plan = el.Plan.from_scenario(sc, precision=prec)
        tr = plan.forward(torch.from_numpy(sc.p0)).cpu().numpy()
        pa = plan.adjoint(torch.from_numpy(y)).cpu().numpy().astype(np.float64)
        out[prec] = (rel_l2(tr, tr_ref), rel_l2(pa, pa_ref), _dot_residual(plan, sc, 1))
        banner(f"96^3/600 {prec}: traces {out[prec][0]:.2e}  H^T y {out[prec][1]:.2e}  dot {out[prec][2]:.2e}")
    assert out["f32"][0] <= 1e-4 and out["f32"][1] <= 1e-4 and out["f32"][2] <= 1e-5
    assert out["f64"][0] <= 1e-11 and out["f64"][1] <= 1e-11 and out["f64"][2] <= 1e-12


def test_precision_256_fp32_vs_fp64():
    """256^3, 1800 samples: the FP32 path against the FP64 GPU path."""
    sc = S.make("skull256")
    p32 = el.Plan.from_scenario(sc, precision="f32")
    tr32 = p32.forward(torch.from_numpy(sc.p0)).cpu().numpy()
    pa32 = p32.adjoint(torch.from_numpy(tr32)).cpu().numpy().astype(np.float64)
    d32 = _dot_residual(p32, sc, 2)
    del p32
    torch.cuda.empty_cache()
    p64 = el.Plan.from_scenario(sc, precision="f64")
    tr64 = p64.forward(torch.from_numpy(sc.p0)).cpu().numpy()
    pa64 = p64.adjoint(torch.from_numpy(tr32)).cpu().numpy()
    d64 = _dot_residual(p64, sc, 2)
    e_tr, e_pa = rel_l2(tr32, tr64), rel_l2(pa32, pa64)
    banner(f"256^3/1800 f32 vs f64: traces {e_tr:.2e}  H^T y {e_pa:.2e}  dot f32 {d32:.2e}  dot f64 {d64:.2e}")
    assert e_tr <= 1e-4 and e_pa <= 1e-4
    assert d32 <= 1e-5 and d64 <= 1e-12
