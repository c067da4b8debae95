"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP32 fields and stencils must match the FP64 oracle within
1e-4 relative L2 on traces and on H^T y, element-wise within 1e-4 of the
largest reference value; the dot-product test residual must be below 1e-5.
The FP64 GPU path must match to 1e-11.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Model
from paper_1709_02733_amd import el
from paper_1709_02733_amd import scenarios as S
from tests.gpu_util import banner, need_gpu, rel_l2, rel_max

pytestmark = pytest.mark.gpu

TOL32 = 1e-4
TOL64 = 1e-11


@pytest.fixture(autouse=True)
def _gpu(request):
    need_gpu()
    banner(request.node.nodeid)
    yield
    torch.cuda.synchronize()


def _run_pair(sc, precision, y=None):
    plan = el.Plan.from_scenario(sc, precision=precision)
    ref = Model.from_scenario(sc)
    p0 = sc.p0.astype(np.float64)
    tr = plan.forward(torch.from_numpy(sc.p0)).cpu().numpy()
    tr_ref = ref.forward(p0)
    if y is None:
        y = tr_ref
    pa = plan.adjoint(torch.from_numpy(y)).cpu().numpy().astype(np.float64)
    pa_ref = ref.adjoint(y)
    return plan, ref, tr, tr_ref, pa, pa_ref


CASES = [
    # shape (x, y, z), npml, nsteps, seed, fluid fraction
    ((23, 19, 17), 3, 40, 1, 0.5),
    ((70, 9, 12), 2, 25, 2, 0.3),      # more than one 64-wide tile along x, ragged tail
    ((17, 29, 8), 0, 30, 3, 0.6),      # no PML
    ((10, 10, 10), 4, 20, 4, 0.0),     # minimum size for npml = 4 (2P + 2), all solid
    ((12, 11, 13), 2, 1, 5, 0.5),      # one sample: no update at all
    ((4, 4, 4), 0, 15, 6, 1.0),        # smallest grid, all fluid: one fluid tile
    ((10, 10, 10), 4, 20, 7, 1.0),     # all fluid with npml = 4: the fluid loops write both slab copies
]


@pytest.mark.parametrize("shape,npml,nsteps,seed,ff", CASES)
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_small_ragged_parity(shape, npml, nsteps, seed, ff, precision):
    sc = S.random_scenario(shape, seed=seed, nsteps=nsteps, npml=npml, nrec=9, fluid_fraction=ff)
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((nsteps, sc.nrec))
    _, _, tr, tr_ref, pa, pa_ref = _run_pair(sc, precision, y)
    tol = TOL32 if precision == "f32" else TOL64
    assert rel_l2(tr, tr_ref) <= tol and rel_max(tr, tr_ref) <= tol, (rel_l2(tr, tr_ref), rel_max(tr, tr_ref))
    assert rel_l2(pa, pa_ref) <= tol and rel_max(pa, pa_ref) <= tol, (rel_l2(pa, pa_ref), rel_max(pa, pa_ref))


@pytest.fixture(scope="module")
def parity64():
    return S.parity_scenario(seed=1)


def test_parity64_forward_and_adjoint(parity64):
    """The 64^3 / 400-step shell case: traces and H^T y within 1e-4 relative L2."""
    sc = parity64
    _, _, tr, tr_ref, pa, pa_ref = _run_pair(sc, "f32")
    e_tr, e_pa = rel_l2(tr, tr_ref), rel_l2(pa, pa_ref)
    banner(f"parity64 rel L2 traces {e_tr:.3e} adjoint {e_pa:.3e}")
    assert e_tr <= TOL32 and e_pa <= TOL32
    assert rel_max(tr, tr_ref) <= TOL32
    assert rel_max(pa, pa_ref) <= TOL32


def _dot_residual(plan, sc, seed):
    g = torch.Generator().manual_seed(seed)
    p = torch.randn(sc.shape, generator=g, dtype=torch.float32)
    q = torch.randn(sc.shape, generator=g, dtype=torch.float32)
    y = plan.forward(q)
    hp = plan.forward(p)
    hty = plan.adjoint(y)
    lhs = float(plan.dot(hp, y, 1))
    rhs = float(plan.dot(p.to(plan.device, plan.dtype), hty, 0))
    return abs(lhs - rhs) / abs(lhs)


def test_dot_product_gpu_parity64(parity64):
    plan = el.Plan.from_scenario(parity64)
    r = _dot_residual(plan, parity64, 7)
    banner(f"dot residual parity64 {r:.3e}")
    assert r <= 1e-5


@pytest.mark.parametrize("precision,tol", [("f32", 1e-5), ("f64", 1e-12)])
def test_dot_product_gpu_ragged(precision, tol):
    sc = S.random_scenario((37, 29, 23), seed=8, nsteps=120, npml=4, nrec=17)
    plan = el.Plan.from_scenario(sc, precision=precision)
    assert _dot_residual(plan, sc, 3) <= tol


def test_dot_matches_numpy():
    sc = S.random_scenario((20, 18, 16), seed=9, nsteps=10, npml=2, nrec=5)
    plan = el.Plan.from_scenario(sc)
    rng = np.random.default_rng(0)
    a = rng.standard_normal(sc.shape).astype(np.float32)
    b = rng.standard_normal(sc.shape).astype(np.float32)
    got = float(plan.dot(torch.from_numpy(a), torch.from_numpy(b), 0))
    want = float(np.dot(a.astype(np.float64).ravel(), b.astype(np.float64).ravel()))
    assert abs(got - want) <= 1e-12 * np.sum(np.abs(a.astype(np.float64) * b))


def test_forward_is_deterministic():
    sc = S.random_scenario((40, 33, 21), seed=10, nsteps=60, npml=3, nrec=33)
    plan = el.Plan.from_scenario(sc)
    p = torch.from_numpy(sc.p0)
    a = plan.forward(p).clone()
    b = plan.forward(p).clone()
    assert torch.equal(a, b)
    y = torch.randn(sc.nsteps, sc.nrec, dtype=torch.float64)
    assert torch.equal(plan.adjoint(y).clone(), plan.adjoint(y).clone())


@pytest.mark.parametrize("every", [1, 3])
def test_kernel_timing_samples_steps(every):
    """el_plan_timing(every): event pairs bracket the launches of time steps m with
    m mod every = 0; results are those of an untimed run."""
    sc = S.random_scenario((23, 19, 17), seed=5, nsteps=11, npml=2, nrec=6)
    plan = el.Plan.from_scenario(sc)
    p = torch.from_numpy(sc.p0)
    y = torch.randn(sc.nsteps, sc.nrec, dtype=torch.float64, generator=torch.Generator().manual_seed(1))
    tr0 = plan.forward(p).cpu()
    pa0 = plan.adjoint(y).cpu()
    plan.timing(True, every=every)
    tr = plan.forward(p).cpu()
    pa = plan.adjoint(y).cpu()
    plan.timing(False)
    kt = plan.kernel_times()
    M = sc.nsteps
    steps = [m for m in range(1, M) if m % every == 0]        # stencil passes run for m = 1 .. M-1
    assert kt["velocity"][0] == kt["stress"][0] == len(steps)
    assert kt["adj_velocity"][0] == kt["adj_stress"][0] == len(steps)
    # adjoint stress pass m adds row m-1; only the last row has a scatter launch of its own
    assert kt["scatter"][0] == (1 if (M - 1) % every == 0 else 0)
    # velocity pass m gathers row m-1; only the last row has a gather launch of its own
    assert kt["gather"][0] == (1 if (M - 1) % every == 0 else 0)
    assert all(ms > 0 for n, ms in kt.values() if n)
    assert torch.equal(tr, tr0) and torch.equal(pa, pa0)
    assert all(n == 0 for n, _ in plan.kernel_times().values())   # the record was cleared


def test_negative_zero_shear_modulus():
    """A fluid cell given as mu = -0.0 behaves as mu = +0.0: the staggered harmonic means
    of the shear modulus are zero next to it (Sec. 2.2), results match the oracle and are
    bitwise those of the same medium with +0.0."""
    sc = S.random_scenario((23, 19, 17), seed=12, nsteps=40, npml=3, nrec=9, fluid_fraction=0.5)
    assert (sc.mu == 0).any() and (sc.mu > 0).any()
    neg = S.random_scenario((23, 19, 17), seed=12, nsteps=40, npml=3, nrec=9, fluid_fraction=0.5)
    neg.mu = np.where(neg.mu == 0, np.float32(-0.0), neg.mu).astype(np.float32)
    assert np.signbit(neg.mu[neg.mu == 0]).all()
    p = torch.from_numpy(sc.p0)
    a = el.Plan.from_scenario(sc).forward(p).cpu()
    b = el.Plan.from_scenario(neg).forward(p).cpu()
    assert torch.isfinite(b).all()
    assert torch.equal(a, b)
    ref = Model.from_scenario(sc).forward(sc.p0.astype(np.float64))
    assert rel_l2(b.numpy(), ref) <= TOL32


def _fluid_ball_scenario(seed=13, nsteps=60):
    """192 x 40 x 40 absorbing fluid (mu = 0) holding a solid ball of radius 6 cells: the
    interior tiles away from the ball take the fluid update, the others the general one.
    The fluid is homogeneous water for x < 96 cells (uniform fluid tiles) and has random
    lambda, rho, alpha per cell elsewhere."""
    sc = S.random_scenario((192, 40, 40), seed=seed, nsteps=nsteps, npml=4, nrec=24, fluid_fraction=1.0)
    z, y, x = np.meshgrid(np.arange(40), np.arange(40), np.arange(192), indexing="ij")
    water = x < 96
    sc.lam = np.where(water, np.float32(1000.0 * 1500.0 ** 2), sc.lam).astype(np.float32)
    sc.rho = np.where(water, np.float32(1000.0), sc.rho).astype(np.float32)
    sc.alpha = np.where(water, np.float32(1.0e5), sc.alpha).astype(np.float32)
    ball = (x - 100) ** 2 + (y - 20) ** 2 + (z - 20) ** 2 <= 36
    cp, cs, rho = 2800.0, 1500.0, 1850.0
    sc.lam = np.where(ball, rho * (cp * cp - 2 * cs * cs), sc.lam).astype(np.float32)
    sc.mu = np.where(ball, rho * cs * cs, sc.mu).astype(np.float32)
    sc.rho = np.where(ball, rho, sc.rho).astype(np.float32)
    sc.dt = 0.3 * sc.dx / cp
    return sc


@pytest.mark.parametrize("precision,tol_same,tol_ref", [("f32", 1e-6, TOL32), ("f64", 1e-13, TOL64)])
def test_fluid_tiles_match_general_update_and_oracle(precision, tol_same, tol_ref):
    """Tiles that are fluid with a two-cell margin are updated from s11 alone (the fluid limit,
    Sec. 2.1): H and H^T equal the general update and the oracle."""
    sc = _fluid_ball_scenario()
    plan = el.Plan.from_scenario(sc, precision=precision)
    st = plan.fluid_stats()
    tiles, cells, skipped = st["tiles"], st["cells"], st["skipped_stores"]
    banner(f"fluid tiles {tiles}, cells {cells} of {sc.ncells}, s22/s33 stores left out {skipped}, "
           f"uniform-media cells {st['uniform_cells']}, fluid-column cells {st['column_cells']}")
    assert tiles > 0 and 0 < cells < sc.ncells
    assert 0 < st["uniform_cells"] < cells
    # the tiles around the ball hold fluid columns: those lanes take the fluid update too
    assert 0 < st["column_cells"] < cells
    # the ball's neighbourhood leaves y and z faces next to general tiles: both bands occur
    assert 0 < skipped < 2 * cells
    p = torch.from_numpy(sc.p0)
    y = np.random.default_rng(3).standard_normal((sc.nsteps, sc.nrec))

    def run():
        tr = plan.forward(p).cpu().numpy()
        fwd_state = {f: plan.field(f).cpu().numpy().astype(np.float64) for f in el.FIELDS}
        pa = plan.adjoint(torch.from_numpy(y)).cpu().numpy().astype(np.float64)
        adj_state = {f: plan.field(f).cpu().numpy().astype(np.float64) for f in el.FIELDS}
        return tr, pa, fwd_state, adj_state

    tr_fast, pa_fast, fs_fast, as_fast = run()
    assert set(plan.fluid_stats(False).values()) == {0}
    tr_gen, pa_gen, fs_gen, as_gen = run()
    assert plan.fluid_stats(True) == st
    banner(f"fluid vs general: traces bitwise {np.array_equal(tr_fast, tr_gen)}, "
           f"max {rel_max(tr_fast, tr_gen):.2e}; adjoint bitwise {np.array_equal(pa_fast, pa_gen)}, "
           f"max {rel_max(pa_fast, pa_gen):.2e}")
    assert rel_max(tr_fast, tr_gen) <= tol_same and rel_max(pa_fast, pa_gen) <= tol_same
    # the whole state after each operation (s22 = s33 = s11 restored on fluid tiles)
    for name in el.FIELDS:
        for a, b, op in ((fs_fast, fs_gen, "forward"), (as_fast, as_gen, "adjoint")):
            scale = max(np.abs(b[name]).max(), np.abs(b["s11"]).max())
            err = np.abs(a[name] - b[name]).max() / scale
            assert err <= tol_same, (op, name, err)
    ref = Model.from_scenario(sc)
    assert rel_l2(tr_fast, ref.forward(sc.p0.astype(np.float64))) <= tol_ref
    assert rel_l2(pa_fast, ref.adjoint(y)) <= tol_ref


@pytest.mark.parametrize("npml,precision,tol_same,tol_ref", [(0, "f32", 1e-6, TOL32), (3, "f32", 1e-6, TOL32),
                                                         (3, "f64", 1e-13, TOL64)])
def test_fluid_path_ragged_grid(npml, precision, tol_same, tol_ref):
    """A 150 x 37 x 29 grid (partial last tiles in x, y and z) of homogeneous water holding a
    solid ball near the +x face: fluid tiles, fluid rows and mixed rows of partial tiles all
    occur; the fluid path equals the general update and the oracle, with and without C-PML."""
    nx, ny, nz = 150, 37, 29
    sc = S.random_scenario((nx, ny, nz), seed=21, nsteps=50, npml=npml, nrec=12, fluid_fraction=1.0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ball = (x - 138) ** 2 + (y - 18) ** 2 + (z - 14) ** 2 <= 25
    cp, cs, rho = 2800.0, 1500.0, 1850.0
    sc.lam = np.where(ball, rho * (cp * cp - 2 * cs * cs), 1000.0 * 1500.0 ** 2).astype(np.float32)
    sc.mu = np.where(ball, rho * cs * cs, 0.0).astype(np.float32)
    sc.rho = np.where(ball, rho, 1000.0).astype(np.float32)
    sc.alpha = np.where(ball, 2.0e5, 1.0e5).astype(np.float32)
    sc.dt = 0.3 * sc.dx / cp
    plan = el.Plan.from_scenario(sc, precision=precision)
    st = plan.fluid_stats()
    banner(f"ragged fluid path ({precision}): {st}")
    assert 0 < st["column_cells"] and 0 < st["uniform_cells"] and st["cells"] < sc.ncells
    p = torch.from_numpy(sc.p0)
    y = np.random.default_rng(4).standard_normal((sc.nsteps, sc.nrec))
    tr_f = plan.forward(p).cpu().numpy()
    s_f = {f: plan.field(f).cpu().numpy().astype(np.float64) for f in el.FIELDS}
    pa_f = plan.adjoint(torch.from_numpy(y)).cpu().numpy().astype(np.float64)
    plan.fluid_path(False)
    tr_g = plan.forward(p).cpu().numpy()
    s_g = {f: plan.field(f).cpu().numpy().astype(np.float64) for f in el.FIELDS}
    pa_g = plan.adjoint(torch.from_numpy(y)).cpu().numpy().astype(np.float64)
    assert rel_max(tr_f, tr_g) <= tol_same and rel_max(pa_f, pa_g) <= tol_same
    for name in el.FIELDS:
        scale = max(np.abs(s_g[name]).max(), np.abs(s_g["s11"]).max())
        assert np.abs(s_f[name] - s_g[name]).max() / scale <= tol_same, name
    ref = Model.from_scenario(sc)
    assert rel_l2(tr_f, ref.forward(sc.p0.astype(np.float64))) <= tol_ref
    assert rel_l2(pa_f, ref.adjoint(y)) <= tol_ref


def test_fluid_tiles_dot_product():
    sc = _fluid_ball_scenario(seed=14, nsteps=80)
    plan = el.Plan.from_scenario(sc)
    assert plan.fluid_path()[0] > 0
    r = _dot_residual(plan, sc, 5)
    banner(f"dot residual with fluid tiles {r:.3e}")
    assert r <= 1e-5


def test_zero_receivers():
    """L = 0: the forward returns an (M, 0) trace array and leaves the wavefield state
    bitwise as with receivers; the adjoint of no data is zero."""
    sc = S.random_scenario((70, 18, 16), seed=3, nsteps=12, npml=2, nrec=4, fluid_fraction=0.8)
    p = torch.from_numpy(sc.p0)
    with_rec = el.Plan.from_scenario(sc)
    with_rec.forward(p)
    ref = {f: with_rec.field(f).cpu().clone() for f in el.FIELDS}
    sc.rec = np.zeros((0, 3))
    plan = el.Plan.from_scenario(sc)
    tr = plan.forward(p)
    assert tuple(tr.shape) == (sc.nsteps, 0)
    for f in el.FIELDS:
        assert torch.equal(plan.field(f).cpu(), ref[f]), f
    pa = plan.adjoint(torch.zeros((sc.nsteps, 0), dtype=torch.float64))
    assert pa.abs().max().item() == 0.0


def test_receivers_on_faces_and_corners():
    sc = S.random_scenario((14, 12, 10), seed=11, nsteps=15, npml=2, nrec=1)
    rec = np.array([[0, 0, 0], [13, 11, 9], [13, 0, 4.5], [6.5, 11, 0], [0.25, 5.75, 9]]) * sc.dx
    sc.rec = rec
    y = np.random.default_rng(1).standard_normal((sc.nsteps, rec.shape[0]))
    _, _, tr, tr_ref, pa, pa_ref = _run_pair(sc, "f32", y)
    assert rel_max(tr, tr_ref) <= TOL32
    assert rel_max(pa, pa_ref) <= TOL32


def test_many_receivers_share_cells():
    """Receivers on top of each other exercise the grid-point-major scatter."""
    sc = S.random_scenario((16, 15, 14), seed=12, nsteps=12, npml=2, nrec=1)
    base = np.array([[5.5, 6.25, 7.0], [5.5, 6.25, 7.0], [5.0, 6.0, 7.0], [5.9, 6.1, 7.3]])
    sc.rec = np.vstack([base] * 20) * sc.dx
    y = np.random.default_rng(2).standard_normal((sc.nsteps, sc.rec.shape[0]))
    _, _, tr, tr_ref, pa, pa_ref = _run_pair(sc, "f32", y)
    assert rel_max(tr, tr_ref) <= TOL32
    assert rel_max(pa, pa_ref) <= TOL32


# --------------------------------------------------------------- error paths

def _maps(sc):
    return dict(lam=sc.lam.copy(), mu=sc.mu.copy(), rho=sc.rho.copy(), alpha=sc.alpha.copy())


def _plan(sc, **over):
    kw = dict(nx=sc.nx, ny=sc.ny, nz=sc.nz, dx=sc.dx, dt=sc.dt, nsteps=sc.nsteps, npml=sc.npml, rec=sc.rec)
    kw.update(_maps(sc))
    kw.update(over)
    return el.Plan(**kw)


def test_plan_rejects_unstable_and_invalid_media():
    sc = S.random_scenario((12, 12, 12), seed=13, nsteps=5, npml=2, nrec=3)
    with pytest.raises(el.ElError) as ei:
        _plan(sc, dt=sc.dt * 2.0)                   # CFL 0.6 > 0.4949
    assert ei.value.status == el.EL_EUNSTABLE
    rho = sc.rho.copy()
    rho[3, 4, 5] = 0.0
    with pytest.raises(el.ElError) as ei:
        _plan(sc, rho=rho)
    assert ei.value.status == el.EL_EINVAL
    mu = sc.mu.copy()
    mu[1, 1, 1] = -1.0
    with pytest.raises(el.ElError) as ei:
        _plan(sc, mu=mu)
    assert ei.value.status == el.EL_EINVAL
    alpha = sc.alpha.copy()
    alpha[2, 2, 2] = 2.0 / sc.dt
    with pytest.raises(el.ElError) as ei:
        _plan(sc, alpha=alpha)
    assert ei.value.status == el.EL_EUNSTABLE
    lam = sc.lam.copy()
    lam[0, 0, 0] = np.nan
    with pytest.raises(el.ElError) as ei:
        _plan(sc, lam=lam)
    assert ei.value.status == el.EL_EINVAL
    # a zero or negative bulk modulus (3 lambda + 2 mu <= 0) with lambda + 2 mu > 0
    for lam_v, mu_v in ((-2.0e9, 3.0e9), (-0.8e9, 1.0e9)):
        lam, mu = sc.lam.copy(), sc.mu.copy()
        lam[4, 5, 6], mu[4, 5, 6] = lam_v, mu_v
        assert lam_v + 2 * mu_v > 0 and 3 * lam_v + 2 * mu_v <= 0
        with pytest.raises(el.ElError) as ei:
            _plan(sc, lam=lam, mu=mu)
        assert ei.value.status == el.EL_EINVAL and "3 lambda + 2 mu" in str(ei.value)
    # the plan still works after rejected attempts
    plan = _plan(sc)
    assert torch.isfinite(plan.forward(torch.from_numpy(sc.p0))).all()


# ------------------------------------------------------- full-size (384^3)

@pytest.fixture(scope="module")
def skull384():
    return S.make("skull384", nsteps=4)


def test_full_size_state_and_traces(skull384):
    """384^3 skull medium in the benchmark's launch configuration: after 3 updates every
    wavefield array and the 4 trace samples match the FP64 oracle."""
    sc = skull384
    plan = el.Plan.from_scenario(sc)
    tr = plan.forward(torch.from_numpy(sc.p0)).cpu().numpy()
    fields = {n: plan.field(n).cpu().numpy() for n in el.FIELDS}
    del plan
    torch.cuda.empty_cache()
    ref = Model.from_scenario(sc)
    v = ref.inject(sc.p0.astype(np.float64))
    tr_ref = [ref.measure(v)]
    for _ in range(sc.nsteps - 1):
        ref.step(v)
        tr_ref.append(ref.measure(v))
    tr_ref = np.array(tr_ref)
    sv = ref.state_views(v)
    refs = dict(zip(el.FIELDS, list(sv["u"]) + list(sv["sig"])))
    for n in el.FIELDS:
        e = rel_max(fields[n], refs[n])
        banner(f"384^3 field {n}: rel max err {e:.2e}")
        assert e <= 1e-5, (n, e)
    assert rel_max(tr, tr_ref) <= 1e-5


def test_full_size_full_length_dot_product():
    """The benchmark's workload itself (384^3 skull medium, M = 2500, L = 1024, C-PML, fluid
    path as launched by bench.py): <H p, y> = <p, H^T y> for random p and y = H q, within
    the FP32 bound of the dot test."""
    sc = S.make("skull384")
    plan = el.Plan.from_scenario(sc)
    st = plan.fluid_stats()
    assert st["cells"] > 0.9 * sc.ncells and st["uniform_cells"] > 0.9 * sc.ncells
    r = _dot_residual(plan, sc, 11)
    banner(f"384^3, M={sc.nsteps}: dot residual {r:.3e}")
    del plan
    torch.cuda.empty_cache()
    assert r <= 1e-5


def test_full_size_adjoint(skull384):
    sc = skull384
    plan = el.Plan.from_scenario(sc)
    y = np.random.default_rng(4).standard_normal((sc.nsteps, sc.nrec))
    pa = plan.adjoint(torch.from_numpy(y)).cpu().numpy().astype(np.float64)
    del plan
    torch.cuda.empty_cache()
    pa_ref = Model.from_scenario(sc).adjoint(y)
    e = rel_max(pa, pa_ref)
    banner(f"384^3 adjoint rel max err {e:.2e}, rel L2 {rel_l2(pa, pa_ref):.2e}")
    assert e <= 1e-5
