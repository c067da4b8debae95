"""GPU modified energy (el_forward_energy) against the FP64 oracle's energy.

The leapfrog scheme of Sec. 2.2 (eq. it) is skew with a symmetric stiffness,
so without absorption and C-PML its modified energy
E_m = 1/2 sum rho u_{m-1/2} u_{m+1/2} + 1/2 sigma_m^T C^+ sigma_m is invariant.
The oracle's E_m (oracle/energy.py, pinned on the CPU by conservation, decay
with absorption and the closed form E_0 = sum p0^2 / (18 K)) is the reference:
the GPU reduction must equal it at every sampled level (FP64 1e-12, FP32 1e-5
relative to E_0), and on the FP64 path E_m must stay within 1e-12 of E_0 over
400 steps.  The traces of el_forward_energy are bitwise those of el_forward.
"""
import numpy as np
import pytest
import torch

from oracle.energy import energy_series
from oracle.oracle import Model
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


@pytest.fixture(scope="module")
def shell40():
    # water (fluid tiles, uniform media) around a solid shell (general tiles with fluid
    # columns); absorption off, no C-PML: E_m is conserved
    sc = S.parity_scenario(seed=3, n=40, nsteps=401, npml=0, nrec=16)
    assert np.all(sc.alpha == 0) and np.any(sc.mu > 0) and np.any(sc.mu == 0)
    ref = energy_series(Model.from_scenario(sc), sc.p0.astype(np.float64), sc.nsteps, every=20)
    return sc, ref


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_energy_matches_oracle_and_is_conserved(shell40, precision, tol):
    sc, ref = shell40
    plan = el.Plan.from_scenario(sc, precision=precision)
    st = plan.fluid_stats()
    assert st["tiles"] > 0 and st["column_cells"] > 0   # every kind of tile takes part
    tr, en = plan.forward_energy(torch.from_numpy(sc.p0), every=20)
    e = en.cpu().numpy()
    assert e.shape == ref.shape == (20,)
    err = np.max(np.abs(e - ref)) / ref[0]
    drift = np.max(np.abs(e - e[0])) / e[0]
    banner(f"{precision}: E_0 {e[0]:.6e}, max |E - oracle| / E_0 {err:.2e}, drift {drift:.2e}")
    assert err <= tol
    assert drift <= tol
    # the traces are those of the plain forward, bit for bit
    tr2 = plan.forward(torch.from_numpy(sc.p0))
    assert torch.equal(tr, tr2)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_energy_every_step_with_pml_and_absorption(precision, tol):
    # ragged grid over two 64-wide tiles, C-PML and absorption: E_m is no longer invariant,
    # but the GPU must still form the oracle's value at every level
    sc = S.random_scenario((70, 11, 13), seed=5, nsteps=31, npml=3, nrec=7, fluid_fraction=0.5)
    assert np.any(sc.alpha > 0)
    ref = energy_series(Model.from_scenario(sc), sc.p0.astype(np.float64), sc.nsteps, every=1)
    plan = el.Plan.from_scenario(sc, precision=precision)
    _, en = plan.forward_energy(torch.from_numpy(sc.p0), every=1)
    e = en.cpu().numpy()
    assert e.shape == (30,)
    err = np.max(np.abs(e - ref)) / np.max(np.abs(ref))
    banner(f"{precision}: max |E - oracle| / max E {err:.2e}; E_29 / E_0 {e[-1] / e[0]:.3f}")
    assert err <= tol
    assert e[-1] < e[0]   # absorption and the layer take energy out


def test_energy_initial_closed_form_and_edge_cases():
    # E_0 = sum p0^2 / (18 K) with K = lambda + 2 mu / 3 (sigma_0 = -p0/3 I, u_{-1/2} = 0)
    sc = S.random_scenario((23, 19, 17), seed=9, nsteps=2, npml=2, nrec=3)
    plan = el.Plan.from_scenario(sc, precision="f64")
    _, en = plan.forward_energy(torch.from_numpy(sc.p0), every=1)
    K = sc.lam.astype(np.float64) + 2.0 * sc.mu.astype(np.float64) / 3.0
    ref = np.sum(sc.p0.astype(np.float64) ** 2 / (18.0 * K))
    assert en.numel() == 1
    assert abs(float(en[0]) - ref) <= 1e-13 * ref
    # count ceil((M - 1) / every); M = 1 has no update and no energy
    sc1 = S.random_scenario((9, 8, 7), seed=1, nsteps=1, npml=0, nrec=2)
    p1 = el.Plan.from_scenario(sc1)
    tr, en1 = p1.forward_energy(torch.from_numpy(sc1.p0), every=3)
    assert en1.numel() == 0 and tr.shape == (1, 2)
    sc2 = S.random_scenario((9, 8, 7), seed=1, nsteps=11, npml=0, nrec=2)
    p2 = el.Plan.from_scenario(sc2)
    assert p2.forward_energy(torch.from_numpy(sc2.p0), every=3)[1].numel() == 4   # m = 0, 3, 6, 9
    with pytest.raises(el.ElError) as ei:
        p2.forward_energy(torch.from_numpy(sc2.p0), every=0)
    assert ei.value.status == el.EL_EINVAL
