"""Algorithmic byte model (bytemodel.py) on the CPU: the C-PML layer count against brute
force, the per-cell figures against the arrays each kernel reads and writes, and the fluid
reductions against the arrays the fluid loops touch."""
import itertools

import numpy as np
import pytest

from paper_1709_02733_amd import bytemodel as B

# arrays per cell of each kernel kind (reads, writes), general update
ARRAYS = {
    "velocity": (["s11", "s22", "s33", "s23", "s13", "s12", "u1", "u2", "u3", "rho", "alpha"], ["u1", "u2", "u3"]),
    "stress": (["u1", "u2", "u3", "s11", "s22", "s33", "s23", "s13", "s12", "lam", "mu"],
               ["s11", "s22", "s33", "s23", "s13", "s12"]),
}
ARRAYS["adj_velocity"] = ARRAYS["velocity"]    # r = Q^-1 q and w = C s have the forward shapes
ARRAYS["adj_stress"] = ARRAYS["stress"]
# fluid loops: s11 alone stands for the normal stresses; no shear stress, no mu
FLUID = {
    "velocity": (["s11", "u1", "u2", "u3", "rho", "alpha"], ["u1", "u2", "u3"]),
    "stress": (["u1", "u2", "u3", "s11", "lam"], ["s11", "s22", "s33"]),
}
FLUID["adj_velocity"] = FLUID["velocity"]
FLUID["adj_stress"] = FLUID["stress"]


def test_pml_cells_brute_force():
    for n, P in ((10, 2), (13, 3), (9, 4)):
        nx, ny, nz = n, n + 1, n + 2
        count = 0
        for i, j, k in itertools.product(range(nx), range(ny), range(nz)):
            for c, m in ((i, nx), (j, ny), (k, nz)):
                count += c < P or c > m - 1 - P
        assert B.pml_cells(nx, ny, nz, P) == count
    assert B.pml_cells(10, 10, 10, 0) == 0


@pytest.mark.parametrize("kind", ["velocity", "stress", "adj_velocity", "adj_stress"])
def test_general_update_bytes_are_the_arrays_touched(kind):
    reads, writes = ARRAYS[kind]
    n = 12
    for es in (4, 8):
        assert B.kernel_bytes(kind, n, n, n, 0, 0, es) == (len(reads) + len(writes)) * es * n ** 3


@pytest.mark.parametrize("kind", ["velocity", "stress", "adj_velocity", "adj_stress"])
def test_fluid_update_bytes(kind):
    reads, writes = FLUID[kind]
    n = 12
    N = n ** 3
    es = 4
    fluid = B.kernel_bytes(kind, n, n, n, 0, 0, es, fluid_cells=N)
    assert fluid == (len(reads) + len(writes)) * es * N
    # uniform media: rho and alpha (velocity) or lambda (stress) come from a per-tile table
    maps = {"rho", "alpha", "lam"} & set(reads)
    uni = B.kernel_bytes(kind, n, n, n, 0, 0, es, fluid_cells=N, uniform_cells=N)
    assert uni == fluid - len(maps) * es * N
    # every s22 and s33 store left out (stress passes only)
    skip = B.kernel_bytes(kind, n, n, n, 0, 0, es, fluid_cells=N, skipped_stores=2 * N)
    assert skip == fluid - (2 * es * N if "s22" in writes else 0)


def test_pml_bytes_and_step_sum():
    n, P, L = 20, 3, 7
    layer = B.pml_cells(n, n, n, P)
    base = {k: B.kernel_bytes(k, n, n, n, 0, L) for k in B.PER_CELL}
    for k in B.PER_CELL:
        assert B.kernel_bytes(k, n, n, n, P, L) - base[k] == layer * B.PER_PML_CELL[k] * 4
    for op, kinds in (("fwd", ("velocity", "stress", "gather")), ("adj", ("adj_velocity", "adj_stress", "scatter"))):
        assert B.step_bytes(op, n, n, n, P, L) == sum(B.kernel_bytes(k, n, n, n, P, L) for k in kinds)
    # receivers: 8 corners of (three FP32 stresses, a 64-bit offset, an FP64 weight) plus one FP64 sample
    assert B.kernel_bytes("gather", n, n, n, P, L) == L * 8 * (3 * 4 + 8 + 8) + L * 8
