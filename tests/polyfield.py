"""Tiny multivariate polynomial helper used by the closed-form difference pins."""
from __future__ import annotations

import numpy as np


class Poly:
    """sum_c coef * x^a y^b z^c, exponents as (a, b, c)."""

    def __init__(self, terms=None):
        self.t = {k: float(v) for k, v in (terms or {}).items() if v != 0.0}

    @staticmethod
    def random(rng, degree=3, scale=1.0):
        terms = {}
        for a in range(degree + 1):
            for b in range(degree + 1 - a):
                for c in range(degree + 1 - a - b):
                    terms[(a, b, c)] = rng.uniform(-1, 1) * scale
        return Poly(terms)

    def __call__(self, x, y, z):
        out = 0.0
        for (a, b, c), v in self.t.items():
            out = out + v * x ** a * y ** b * z ** c
        return out

    def d(self, axis):
        terms = {}
        for e, v in self.t.items():
            if e[axis] == 0:
                continue
            ne = list(e)
            ne[axis] -= 1
            terms[tuple(ne)] = terms.get(tuple(ne), 0.0) + v * e[axis]
        return Poly(terms)

    def __add__(self, o):
        terms = dict(self.t)
        for k, v in o.t.items():
            terms[k] = terms.get(k, 0.0) + v
        return Poly(terms)

    def scale(self, s):
        return Poly({k: v * s for k, v in self.t.items()})


def staggered_coords(shape_zyx, dx, offset_xyz):
    """Broadcastable metre coordinates of a staggered sample set (offsets in cells)."""
    nz, ny, nx = shape_zyx
    x = (np.arange(nx) + offset_xyz[0])[None, None, :] * dx
    y = (np.arange(ny) + offset_xyz[1])[None, :, None] * dx
    z = (np.arange(nz) + offset_xyz[2])[:, None, None] * dx
    return x, y, z


# staggered offsets (cells) of every field, x-y-z order
U_OFF = [(0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5)]
SIG_OFF = [(0, 0, 0), (0, 0, 0), (0, 0, 0), (0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0)]
VOIGT = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (1, 2): 3, (2, 1): 3, (0, 2): 4, (2, 0): 4, (0, 1): 5, (1, 0): 5}
