"""Grouped time stepping (el_group) on the GPU.

Members of uneven grids, step counts, receiver sets and directions step together, up to
four per launch, joining and leaving between ticks; every member's result is bitwise that
of el_forward / el_adjoint on its plan.  The serving loop over a group (plans built on a
worker thread, a medium per request) gives bitwise the plain path's results at 96^3 and
128^3 and matches the FP64 oracle; a request withdrawn while it runs leaves the others
unchanged.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Model
from paper_1709_02733_amd import el
from paper_1709_02733_amd import scenarios as S
from paper_1709_02733_amd import serving as SV
from tests.gpu_util import banner, need_gpu, rel_l2, rel_max

pytestmark = pytest.mark.gpu

MECH = [(2 * np.pi * 0.3e6, 0.5), (2 * np.pi * 1.5e6, 0.5)]


@pytest.fixture(autouse=True)
def _gpu(request):
    need_gpu()
    banner(request.node.nodeid)
    yield
    torch.cuda.synchronize()


def _relaxed(sc, seed):
    rng = np.random.default_rng(seed)
    m = sc.npml + 2
    ar = np.zeros(sc.shape, np.float32)
    nz, ny, nx = sc.shape
    ar[m:nz - m, m:ny - m, m:nx - m] = rng.uniform(0.0, 3e6, (nz - 2 * m, ny - 2 * m, nx - 2 * m))
    sc.alpha_r, sc.mechanisms = ar, list(MECH)
    return sc


# shape (x, y, z), npml, nsteps, nrec, seed, fluid fraction, relaxation, op
MEMBERS = [
    ((40, 33, 29), 4, 37, 11, 1, 0.5, False, el.OP_FORWARD),
    ((70, 26, 22), 3, 51, 9, 2, 0.8, False, el.OP_ADJOINT),
    ((23, 19, 17), 2, 23, 0, 3, 0.5, False, el.OP_FORWARD),      # no receivers
    ((48, 20, 36), 5, 44, 13, 4, 1.0, False, el.OP_ADJOINT),     # all fluid
    ((31, 27, 25), 3, 1, 5, 5, 0.5, False, el.OP_ADJOINT),       # a single sample: no steps
    ((36, 30, 28), 3, 33, 7, 6, 0.4, True, el.OP_FORWARD),       # relaxation mechanisms
    ((29, 41, 19), 2, 29, 6, 7, 0.6, True, el.OP_ADJOINT),
]


def _member(k, precision):
    shape, npml, nsteps, nrec, seed, ff, relax, op = MEMBERS[k]
    sc = S.random_scenario(shape, seed=seed, nsteps=nsteps, npml=npml, nrec=max(nrec, 1), fluid_fraction=ff)
    if nrec == 0:
        sc.rec = sc.rec[:0]
    if relax:
        sc = _relaxed(sc, seed)
    plan = el.Plan.from_scenario(sc, precision=precision)
    if op == el.OP_FORWARD:
        inp = torch.from_numpy(sc.p0).to(plan.device, plan.dtype)
        ref = plan.forward(inp).clone()
    else:
        g = torch.Generator().manual_seed(100 + k)
        inp = torch.randn((nsteps, sc.nrec), dtype=torch.float64, generator=g).to(plan.device)
        ref = plan.adjoint(inp).clone()
    torch.cuda.synchronize()
    return plan, op, inp, ref


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_members_equal_direct_calls(precision):
    """Seven members (forward and adjoint, uneven grids and step counts, no receivers, a
    single sample, relaxation) in a group of seven: two launches of up to four members per
    sub-update.  Four join at once, three more after 10 ticks; every result is bitwise the
    direct call's."""
    ms = [_member(k, precision) for k in range(len(MEMBERS))]
    grp = el.Group(max_members=len(MEMBERS), precision=el.EL_F64 if precision == "f64" else el.EL_F32)
    outs = [torch.full_like(ref, float("nan")) for _, _, _, ref in ms]
    slots = {}
    for k in range(4):
        plan, op, inp, _ = ms[k]
        slots[k] = grp.add(plan, op, inp, outs[k])
    grp.run(10)
    for k in range(4, len(ms)):
        plan, op, inp, _ = ms[k]
        slots[k] = grp.add(plan, op, inp, outs[k])
    for _ in range(100):
        grp.run(7)
        grp.sync(1)
        if grp.members()[2] == 0:
            break
    grp.sync(0)
    for k, s in slots.items():
        steps, done = grp.poll(s)
        assert done, k
    for k, (plan, op, inp, ref) in enumerate(ms):
        assert torch.equal(outs[k], ref), (k, MEMBERS[k])
    assert grp.members() == (len(MEMBERS), 0, 0)
    grp.close()


def test_large_and_small_members_share_launches():
    """A 160^3 forward and a 162 x 160 x 158 adjoint (several thousand tiles each) in the
    same grouped launches as two small members: all bitwise equal to direct calls."""
    shapes = [((160, 160, 160), el.OP_FORWARD), ((162, 160, 158), el.OP_ADJOINT),
              ((40, 33, 29), el.OP_FORWARD), ((29, 41, 19), el.OP_ADJOINT)]
    ms = []
    for k, (shape, op) in enumerate(shapes):
        sc = S.random_scenario(shape, seed=20 + k, nsteps=17 + 3 * k, npml=4, nrec=25, fluid_fraction=0.7)
        plan = el.Plan.from_scenario(sc)
        if op == el.OP_FORWARD:
            inp = torch.from_numpy(sc.p0).to(plan.device)
            ref = plan.forward(inp).clone()
        else:
            inp = torch.randn((sc.nsteps, sc.nrec), dtype=torch.float64, generator=torch.Generator().manual_seed(k)).cuda()
            ref = plan.adjoint(inp).clone()
        ms.append((plan, op, inp, ref))
    assert ms[0][0].grid.nx * ms[0][0].grid.ny * ms[0][0].grid.nz >= 4000000
    grp = el.Group(max_members=4)
    outs = [torch.full_like(ref, float("nan")) for *_, ref in ms]
    slots = [grp.add(plan, op, inp, outs[k]) for k, (plan, op, inp, _) in enumerate(ms)]
    while grp.members()[2]:
        grp.run(5)
        grp.sync(1)
    grp.sync(0)
    for k, s in enumerate(slots):
        assert grp.poll(s)[1]
        assert torch.equal(outs[k], ms[k][3]), k
    grp.close()


def test_withdrawn_member_leaves_the_others_unchanged():
    ms = [_member(k, "f32") for k in (0, 1, 3)]
    grp = el.Group(max_members=3)
    outs = [torch.empty_like(ref) for _, _, _, ref in ms]
    slots = [grp.add(plan, op, inp, outs[k]) for k, (plan, op, inp, _) in enumerate(ms)]
    grp.run(12)
    grp.remove(slots[1])
    assert grp.members()[2] == 2
    while grp.members()[2] > 0:
        grp.run(8)
        grp.sync(1)
    grp.sync(0)
    assert grp.poll(slots[1]) == (12, True)
    for k in (0, 2):
        assert torch.equal(outs[k], ms[k][3])
        assert grp.poll(slots[k])[1]
    # the withdrawn member's plan is usable again
    plan, op, inp, ref = ms[1]
    assert torch.equal(plan.adjoint(inp), ref)
    grp.close()


def test_group_rejects_bad_members():
    plan, op, inp, ref = _member(0, "f32")
    plan64, _, _, _ = _member(2, "f64")
    grp = el.Group(max_members=1)
    out = torch.empty_like(ref)
    with pytest.raises(el.ElError) as ei:
        grp.add(plan64, el.OP_FORWARD, inp.double(), torch.empty(0, device=inp.device))
    assert ei.value.status == el.EL_EINVAL
    with pytest.raises(el.ElError) as ei:
        grp.add(plan, 7, inp, out)
    assert ei.value.status == el.EL_EINVAL
    s = grp.add(plan, op, inp, out)
    plan2, op2, inp2, ref2 = _member(2, "f32")
    with pytest.raises(el.ElError) as ei:
        grp.add(plan2, op2, inp2, torch.empty_like(ref2))
    assert ei.value.status == el.EL_EBUSY
    grp2 = el.Group(max_members=2)
    with pytest.raises(el.ElError) as ei:      # a plan may be a member once at a time
        grp2.add(plan2, op2, inp2, torch.empty_like(ref2))
        grp2.add(plan2, op2, inp2, torch.empty_like(ref2))
    assert ei.value.status == el.EL_EINVAL
    grp2.close()
    while grp.members()[2]:
        grp.run(16)
    grp.sync(0)
    assert grp.poll(s)[1] and torch.equal(out, ref)
    grp.close()


def test_group_call_edges():
    """run / sync / poll / remove on an empty group, a free slot, a member that has taken
    some steps, and out-of-range arguments."""
    plan, op, inp, ref = _member(0, "f32")
    grp = el.Group(max_members=2)
    grp.run(0)
    grp.run(5)                                   # nothing to step
    grp.sync(0)
    assert grp.poll(1) == (0, True)              # a free slot is done
    grp.remove(1)                                # withdrawing a free slot does nothing
    out = torch.empty_like(ref)
    s = grp.add(plan, op, inp, out)
    assert grp.poll(s) == (0, False)
    grp.run(3)
    grp.sync(0)
    assert grp.poll(s) == (3, False)
    assert grp.members() == (2, 1, 1)
    for bad in (lambda: grp.run(-1), lambda: grp.sync(-1), lambda: grp.poll(2), lambda: grp.remove(-1)):
        with pytest.raises(el.ElError) as ei:
            bad()
        assert ei.value.status == el.EL_EINVAL
    grp.remove(s)
    grp.sync(0)
    assert grp.poll(s) == (3, True)
    assert grp.members() == (2, 0, 0)
    # the plan runs again, in the group, to the direct call's result
    s = grp.add(plan, op, inp, out)
    while grp.members()[2]:
        grp.run(16)
    grp.sync(0)
    assert grp.poll(s)[1] and torch.equal(out, ref)
    grp.close()


@pytest.fixture(scope="module")
def serving_96_128():
    wl = SV.Workloads(sizes=(96, 128), keep_outputs=True, per_request_media=True)
    rng = np.random.default_rng(3)
    reqs = []
    for k in range(6):
        n = (96, 128)[k % 2]
        reqs.append(SV.Request(rid=k, op=(k // 2) % 2, n=n, nsteps=int(rng.integers(150, 260)),
                               nrec=int(rng.integers(200, 600)), seed=500 + k, arrival=0.003 * k))
    return wl, reqs


def test_grouped_serving_equals_plain_at_96_and_128(serving_96_128):
    """Six requests at 96^3 and 128^3 (a medium each, forward and adjoint) through the grouped
    serving loop: bitwise the results of the plain path (each request alone through
    el_forward / el_adjoint)."""
    wl, reqs = serving_96_128
    grp = el.Group(max_members=4)
    a = SV.run_plain(SV.clone_requests(reqs), wl)
    b = SV.run_grouped(SV.clone_requests(reqs), wl, grp, budget_bytes=1e12)
    for ra, rb in zip(a, b):
        assert rb.done is not None
        assert torch.equal(ra.output, rb.output), (ra.rid, ra.n, ra.op)
    grp.close()


def test_hybrid_serving_equals_plain(serving_96_128):
    """Hybrid mode (128^3 requests on executor slots, 96^3 ones in the group, overlapping on
    the device): bitwise the plain path's results."""
    wl, reqs = serving_96_128
    grp = el.Group(max_members=4)
    ex = el.Executor(max_slots=2, chunk=16)
    a = SV.run_plain(SV.clone_requests(reqs), wl)
    b = SV.run_grouped(SV.clone_requests(reqs), wl, grp, budget_bytes=1e12, executor=ex, large_cells=128 ** 3)
    for ra, rb in zip(a, b):
        assert rb.done is not None
        assert torch.equal(ra.output, rb.output), (ra.rid, ra.n, ra.op)
    assert grp.members()[1] == 0 and ex.slots()[1] == 0
    grp.close()
    ex.close()


def test_grouped_serving_matches_the_oracle_at_96(serving_96_128):
    """One forward and one adjoint 96^3 request of the grouped loop against the FP64 oracle on
    the same medium (within 1e-4 relative L2 and element-wise of the largest value)."""
    wl, reqs = serving_96_128
    reqs = [SV.clone_requests(reqs)[k] for k in (0, 2)]      # 96^3 forward, 96^3 adjoint
    for r in reqs:
        r.nsteps = 200
    assert [(r.n, r.op) for r in reqs] == [(96, 0), (96, 1)]
    grp = el.Group(max_members=2)
    out = SV.run_grouped(reqs, wl, grp, budget_bytes=1e12)
    grp.close()
    for r in out:
        sc = wl.media[r.n]["sc"]
        lam, mu, rho, alpha = (t.cpu().numpy() for t in wl.medium(r))
        m = Model(r.n, r.n, r.n, sc.dx, sc.dt / 1.03, r.nsteps, 16, lam, mu, rho, alpha, wl.receivers(r))
        inp, _ = wl.io(r)
        ref = m.forward(inp.double().cpu().numpy()) if r.op == 0 else m.adjoint(inp.cpu().numpy())
        got = r.output.cpu().numpy()
        e2, em = rel_l2(got, ref), rel_max(got, ref)
        banner(f"request {r.rid} op {r.op} n {r.n}: rel L2 {e2:.2e}, rel max {em:.2e}")
        assert e2 <= 1e-4 and em <= 1e-4


def test_request_withdrawn_while_running_on_the_gpu(serving_96_128):
    """A request withdrawn while it runs in the group: its output is dropped and its slot
    and bytes return; the other requests stay bitwise equal to running alone."""
    wl, reqs = serving_96_128
    reqs = SV.clone_requests(reqs)[:4]
    reqs[1].nsteps = 3000                    # arrives at 3 ms and would run for over 100 ms
    reqs[1].cancel_at = 0.06
    grp = el.Group(max_members=4)
    trace = []
    out = SV.run_grouped(reqs, wl, grp, budget_bytes=1e12, trace=trace)
    assert out[1].cancelled and out[1].output is None and out[1].done is None
    assert out[1].admitted is not None       # it did start
    plain = SV.run_plain(SV.clone_requests([reqs[k] for k in (0, 2, 3)]), wl)
    for ra, rb in zip(plain, [out[k] for k in (0, 2, 3)]):
        assert rb.done is not None and torch.equal(ra.output, rb.output), ra.rid
    assert trace[-1][1] == 0 and trace[-1][2] == 0
    assert grp.members()[1] == 0
    grp.close()
