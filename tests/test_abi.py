"""The C ABI library loads, exports every symbol include/el.h declares, and its
host-only logic (grid checks, workspace sizing) behaves as documented.  No
GPU is touched."""
import os
import re

import numpy as np
import pytest

from paper_1709_02733_amd import el

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "el.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(el_[a-z0-9_]+)\s*\(", src)))


def test_header_symbols_exported():
    L = el.lib()
    names = _declared()
    assert "el_forward" in names and "el_adjoint" in names and "el_plan_create" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(el.EXPORTS)


def test_version_and_status_strings():
    assert "gfx950" in el.version()
    assert el.status_name(el.EL_ERANGE) == "EL_ERANGE"
    assert el.status_name(-77) == "EL_UNKNOWN"


def _g(**kw):
    base = dict(nx=16, ny=12, nz=10, dx=1e-4, dt=1e-8, nsteps=10, npml=3)
    base.update(kw)
    prec = base.pop("precision", "f32")
    return el.make_grid(precision=prec, **base)


@pytest.mark.parametrize("bad,code", [
    (dict(nx=3), el.EL_EINVAL), (dict(dx=0.0), el.EL_EINVAL), (dict(dt=-1.0), el.EL_EINVAL),
    (dict(nsteps=0), el.EL_EINVAL), (dict(npml=-1), el.EL_EINVAL), (dict(npml=5), el.EL_EINVAL),
    (dict(precision=7), el.EL_EINVAL), (dict(dx=float("nan")), el.EL_EINVAL),
])
def test_grid_check_rejects(bad, code):
    with pytest.raises(el.ElError) as ei:
        el.grid_check(_g(**bad))
    assert ei.value.status == code


def test_grid_check_receivers():
    g = _g()
    dx = g.dx
    el.grid_check(g, np.array([[0, 0, 0], [15, 11, 9], [7.5, 3.25, 0.0]]) * dx)
    for bad in ([[15.0001, 1, 1]], [[1, -0.01, 1]], [[1, 1, 9.5]]):
        with pytest.raises(el.ElError) as ei:
            el.grid_check(g, np.array(bad) * dx)
        assert ei.value.status == el.EL_ERANGE
    # npml = 2*P+2 boundary is accepted, one less is not
    el.grid_check(_g(nx=8, ny=8, nz=8, npml=3))
    with pytest.raises(el.ElError):
        el.grid_check(_g(nx=7, ny=8, nz=8, npml=3))


def test_plan_bytes_scales_with_precision_and_grid():
    b32 = el.plan_bytes(_g(), 5)
    b64 = el.plan_bytes(_g(precision="f64"), 5)
    N = 16 * 12 * 10
    # 9 fields + 4 maps dominate; doubles take twice the bytes
    assert b32 >= 13 * N * 4
    assert b64 >= 13 * N * 8
    assert b64 > b32
    assert el.plan_bytes(_g(npml=0), 5) < b32
    big = el.make_grid(384, 384, 384, 1e-4, 1e-8, 2500, 16)
    nb = el.plan_bytes(big, 1024)
    # 13 padded volumes (rows of 416 >= 384 + 2 elements, 386 rows, 388 planes) plus boundary slabs
    padded = 416 * 386 * 388
    assert 13 * padded * 4 < nb < 1.2 * 13 * padded * 4


def test_grid_check_rejects_arrays_beyond_32bit_offsets():
    el.grid_check(el.make_grid(1000, 1000, 900, 1e-4, 1e-8, 10, 16))            # ~3.7 GiB per array: accepted
    with pytest.raises(el.ElError) as ei:
        el.grid_check(el.make_grid(1100, 1100, 1000, 1e-4, 1e-8, 10, 16))       # > 4 GiB per array
    assert ei.value.status == el.EL_EINVAL
    with pytest.raises(el.ElError):
        el.grid_check(el.make_grid(820, 820, 820, 1e-4, 1e-8, 10, 16, precision="f64"))   # 4.5 GiB in double


def test_grid_check_rejects_slabs_beyond_32bit_offsets():
    # thin grids: a C-PML memory-variable slab (2 (P + 7) planes of nx * ny cells along z) can
    # outgrow the volume arrays; its 32-bit byte offsets must not wrap
    with pytest.raises(el.ElError) as ei:
        el.grid_check(el.make_grid(8000, 8000, 10, 1e-4, 1e-8, 10, 4))        # 22 * 8000^2 * 4 B = 5.6 GB
    assert ei.value.status == el.EL_EINVAL and "C-PML" in str(ei.value)
    with pytest.raises(el.ElError) as ei:
        el.grid_check(el.make_grid(11000, 11000, 4, 1e-4, 1e-8, 10, 1))       # 16 * 11000^2 * 4 B = 7.7 GB
    assert ei.value.status == el.EL_EINVAL
    # just inside: 22 * 6900^2 * 4 B = 4.19e9 < 2^32, volumes 2.7 GB
    el.grid_check(el.make_grid(6900, 6900, 10, 1e-4, 1e-8, 10, 4))
    assert el.plan_bytes(el.make_grid(6900, 6900, 10, 1e-4, 1e-8, 10, 4), 1) > 0
    # the same thin grid without a C-PML has no slabs and is accepted
    el.grid_check(el.make_grid(8000, 8000, 10, 1e-4, 1e-8, 10, 0))
    # in double the limit halves
    with pytest.raises(el.ElError):
        el.grid_check(el.make_grid(6900, 6900, 10, 1e-4, 1e-8, 10, 4, precision="f64"))


def test_grid_check_relaxation_mechanisms():
    ok = [(2e6, 0.5), (1e7, 0.5)]
    el.grid_check(el.make_grid(16, 12, 10, 1e-4, 1e-8, 10, 3, mechanisms=ok))
    for bad in ([(0.0, 1.0)], [(-1e6, 1.0)], [(1e6, -0.1)], [(float("nan"), 1.0)], [(1e6, float("inf"))],
                [(1e6, 0.2)] * 5):
        with pytest.raises(el.ElError) as ei:
            el.grid_check(el.make_grid(16, 12, 10, 1e-4, 1e-8, 10, 3, mechanisms=bad))
        assert ei.value.status == el.EL_EINVAL
    # the memory variables take 3 arrays per mechanism over every tile, plus the strength map
    b0 = el.plan_bytes(el.make_grid(64, 40, 30, 1e-4, 1e-8, 10, 3), 4)
    b1 = el.plan_bytes(el.make_grid(64, 40, 30, 1e-4, 1e-8, 10, 3, mechanisms=ok[:1]), 4)
    b2 = el.plan_bytes(el.make_grid(64, 40, 30, 1e-4, 1e-8, 10, 3, mechanisms=ok), 4)
    assert b2 - b1 >= 3 * 64 * 40 * 30 * 4 and b1 - b0 >= 4 * 64 * 40 * 30 * 4
