"""Algorithmic HBM bytes of each kernel of the time loops.

Every input array a kernel needs is counted as read once and every array it
produces as written once (the minimum traffic of the algorithm, with the
staggered-grid averages of rho, alpha and mu formed on chip from the four
cell maps).  Memory variables of the C-PML live only on the 2*npml planes of
each axis where the layer coefficient a is non-zero.

Per cell of the volume (es = bytes per element, 4 for float):
  velocity      reads s x6, u x3, rho, alpha;   writes u x3     -> 14 es
  stress        reads u x3, s x6, lambda, mu;   writes s x6     -> 17 es
  adj_velocity  reads w x6, r x3, rho, alpha;   writes r x3     -> 14 es
  adj_stress    reads r x3, w x6, lambda, mu;   writes w x6     -> 17 es
(the adjoint state is r = Q^-1 q and w = C s, so its passes have the forward shapes).
Per C-PML cell of each axis:
  velocity / stress          phi (psi) x3 read + x3 written        ->  6 es
  adj_velocity / adj_stress  a psi~ (a phi~) x3 read, a phi~ (a psi~) x3 read + written -> 9 es
Per cell of a fluid tile (mu = 0 on the tile and two cells around it), where
s22 = s33 = s11 and the shear stresses are zero:
  velocity / adj_velocity  reads s11, u x3, rho, alpha; writes u x3              ->  9 es
  stress / adj_stress      reads u x3, s11, lambda;     writes s11, s22, s33      ->  8 es
less one element for every s22 or s33 store the stress passes leave out (those
stresses are stored only where a general-update tile reads them, el_plan_fluid_path),
less rho and alpha (velocity) or lambda (stress) on a fluid cell of uniform media, whose
values come from a per-tile table (the algorithm's bytes: where a kernel still reads a map
it does not need, that read counts as traffic above the model),
and per fluid cell of each axis's C-PML layers only the diagonal memory variable:
  velocity / stress        phi^aa (psi^aa) read + written                        ->  2 es
  adj_velocity / adj_stress a psi~^aa (a phi~^aa) read, a phi~^aa (a psi~^aa) read + written -> 3 es
Receivers: gather 24 + 8 + 8 bytes per (receiver, corner) plus 8 per trace
sample; scatter the same per entry.
"""
from __future__ import annotations

PER_CELL = {"velocity": 14, "stress": 17, "adj_velocity": 14, "adj_stress": 17}
PER_PML_CELL = {"velocity": 6, "stress": 6, "adj_velocity": 9, "adj_stress": 9}
PER_FLUID_CELL = {"velocity": 9, "stress": 8, "adj_velocity": 9, "adj_stress": 8}
PER_FLUID_PML_CELL = {"velocity": 2, "stress": 2, "adj_velocity": 3, "adj_stress": 3}
UNIFORM_MAPS_VELOCITY = 2   # rho, alpha
UNIFORM_MAPS_STRESS = 1     # lambda


def pml_cells(nx: int, ny: int, nz: int, npml: int) -> int:
    """Cells of the C-PML summed over the three axes (2*npml planes each)."""
    if npml <= 0:
        return 0
    return 2 * npml * (ny * nz + nx * nz + nx * ny)


def kernel_bytes(kind: str, nx: int, ny: int, nz: int, npml: int, nrec: int, es: int = 4,
                 fluid_cells: int = 0, fluid_layer_cells: int = 0, skipped_stores: int = 0,
                 uniform_cells: int = 0) -> float:
    """Algorithmic bytes of one launch of a kernel kind; fluid_cells of the volume take the
    fluid-tile update, fluid_layer_cells of the C-PML (cell, axis) pairs lie in fluid tiles,
    the stress passes leave out skipped_stores s22 / s33 stores, and uniform_cells of the
    fluid cells read no material map (el_plan_fluid_path)."""
    N = nx * ny * nz
    if kind in PER_CELL:
        layer = pml_cells(nx, ny, nz, npml)
        stress = kind in ("stress", "adj_stress")
        skipped = skipped_stores if stress else 0
        maps = uniform_cells * (UNIFORM_MAPS_STRESS if stress else UNIFORM_MAPS_VELOCITY)
        return float((N - fluid_cells) * PER_CELL[kind] * es + fluid_cells * PER_FLUID_CELL[kind] * es
                     - skipped * es - maps * es
                     + (layer - fluid_layer_cells) * PER_PML_CELL[kind] * es
                     + fluid_layer_cells * PER_FLUID_PML_CELL[kind] * es)
    if kind in ("gather", "scatter"):
        return float(nrec * 8 * (3 * es + 16) + nrec * 8)
    raise KeyError(kind)


def step_bytes(op: str, nx, ny, nz, npml, nrec, es=4, fluid_cells: int = 0, fluid_layer_cells: int = 0,
               skipped_stores: int = 0, uniform_cells: int = 0) -> float:
    """Bytes of one time step of the forward ('fwd') or adjoint ('adj') operator."""
    if op == "fwd":
        ks = ("velocity", "stress", "gather")
    else:
        ks = ("adj_velocity", "adj_stress", "scatter")
    return sum(kernel_bytes(k, nx, ny, nz, npml, nrec, es, fluid_cells, fluid_layer_cells, skipped_stores,
                            uniform_cells) for k in ks)


def relax_bytes(points: int, nmech: int, es: int = 4) -> float:
    """Algorithmic bytes of one relaxation launch (frequency-dependent absorption): per velocity
    point with beta > 0 (el_plan_relaxation) its strength beta read, and the velocity and the
    nmech memory variables read and written.  Elsewhere the sub-update is the identity."""
    return float(points * (3 + 2 * nmech) * es)
