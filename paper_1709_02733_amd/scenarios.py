"""Seeded synthetic inputs for the forward operator H and its adjoint.

This module only draws inputs: Lame maps, density, absorption, initial
pressure, receiver positions, grid spacing and time step.  It holds none of
the operator's arithmetic (no staggering, no averaging, no stencils), so that
the FP64 CPU oracle and the GPU path can both be fed from it without sharing
any code of the method itself.

Units are SI throughout: Pa for lambda and mu, kg/m^3 for rho, 1/s for the
velocity damping alpha of the paper's diffusive absorption model (Sec. 2.1,
eq. subeq1), metres for dx and for receiver coordinates (measured from the
centre of cell (0,0,0)), seconds for dt.  Arrays are float32 in C order
[nz][ny][nx], i.e. x is the fastest axis.

Workload shapes follow the paper's studies where it gives them (Sec. 6 and
Sec. 7: water background rho 1000, c_l 1.5 mm/us; skull rho 1850, c_l 3.0,
c_s 1.5 mm/us, alpha ~0.1/us; vessel-like initial pressure under the inner
skull surface; transducers on rings / a hemisphere around the head).  The CT
skull, the vessel phantom and the ring radii of the paper are not available,
so the recipes below stand in for them.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

WATER_CP = 1500.0      # m/s
WATER_RHO = 1000.0     # kg/m^3
SKULL_CP = 2800.0
SKULL_CS = 1500.0
SKULL_RHO = 1850.0
CFL = 0.3              # c_max * dt / dx used by every recipe


@dataclasses.dataclass
class Scenario:
    name: str
    seed: int
    nx: int
    ny: int
    nz: int
    dx: float
    dt: float
    nsteps: int
    npml: int
    lam: np.ndarray      # float32 [nz][ny][nx], Pa
    mu: np.ndarray       # float32, Pa
    rho: np.ndarray      # float32, kg/m^3
    alpha: np.ndarray    # float32, 1/s
    p0: np.ndarray       # float32, Pa
    rec: np.ndarray      # float64 [L][3], metres from the centre of cell (0,0,0); columns x, y, z
    # frequency-dependent absorption (optional): strength map alpha_r (float32, 1/s) and the
    # relaxation mechanisms as (omega_l in rad/s, weight w_l) pairs
    alpha_r: np.ndarray | None = None
    mechanisms: list | None = None

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nrec(self) -> int:
        return int(self.rec.shape[0])

    def cell_updates(self) -> int:
        """Cell-updates of one operator application: N (M - 1)."""
        return self.ncells * (self.nsteps - 1)

    def grid_kwargs(self) -> dict:
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, dx=self.dx, dt=self.dt,
                    nsteps=self.nsteps, npml=self.npml)


# ----------------------------------------------------------------------------
# small helpers (geometry and unit conversions only)
# ----------------------------------------------------------------------------

def lame_from_speeds(cp, cs, rho):
    """lambda, mu from c_l, c_s and rho (Sec. 2.1: c_l^2 = (lambda+2mu)/rho, c_s^2 = mu/rho)."""
    cp = np.asarray(cp, dtype=np.float64)
    cs = np.asarray(cs, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    mu = rho * cs * cs
    lam = rho * cp * cp - 2.0 * mu
    return lam, mu


def neper_per_m_to_rate(alpha_np_per_m, cp):
    """Velocity-damping rate (1/s) whose plane-wave amplitude decay is alpha Np/m.

    The damping acts on the particle velocity only, which in the low-loss
    limit carries half of the wave energy, so the amplitude decays at rate
    alpha_t / 2 in time, i.e. alpha_t / (2 c) per metre.
    """
    return 2.0 * np.asarray(cp, dtype=np.float64) * np.asarray(alpha_np_per_m, dtype=np.float64)


def fibonacci_sphere(n: int, hemisphere: bool = False) -> np.ndarray:
    """n unit vectors on the (upper hemi)sphere, golden-angle spiral."""
    k = np.arange(n, dtype=np.float64) + 0.5
    if hemisphere:
        z = 1.0 - k / n
    else:
        z = 1.0 - 2.0 * k / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    th = k * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(th), r * np.sin(th), z], axis=1)


def _grid_coords(n: int):
    """Cell-index coordinates of a cubic n^3 grid as broadcastable z, y, x arrays."""
    ax = np.arange(n, dtype=np.float64)
    return ax[:, None, None], ax[None, :, None], ax[None, None, :]


def _dt_for(cp_max: float, dx: float) -> float:
    return CFL * dx / cp_max


def _finish(name, seed, n_xyz, dx, nsteps, npml, cp, cs, rho, alpha_t, p0, rec_cells):
    nx, ny, nz = n_xyz
    lam, mu = lame_from_speeds(cp, cs, rho)
    dt = _dt_for(float(np.max(cp)), dx)
    return Scenario(
        name=name, seed=seed, nx=nx, ny=ny, nz=nz, dx=dx, dt=dt, nsteps=nsteps, npml=npml,
        lam=np.ascontiguousarray(lam, dtype=np.float32),
        mu=np.ascontiguousarray(mu, dtype=np.float32),
        rho=np.ascontiguousarray(rho, dtype=np.float32),
        alpha=np.ascontiguousarray(alpha_t, dtype=np.float32),
        p0=np.ascontiguousarray(p0, dtype=np.float32),
        rec=np.ascontiguousarray(np.asarray(rec_cells, dtype=np.float64) * dx),
    )


# ----------------------------------------------------------------------------
# recipe 1: 64^3 parity case (spherical shell in water, three balls)
# ----------------------------------------------------------------------------

def parity_scenario(seed: int = 1, n: int = 64, nsteps: int = 400, npml: int = 8,
                    dx: float = 0.2e-3, nrec: int = 128) -> Scenario:
    """Water with a 4-cell spherical shell (22 <= r < 26 cells), three uniform balls.

    Absorption off.  Receivers: Fibonacci sphere of radius 28 cells.  The
    radii scale with n/64 so that smaller variants keep the same geometry.
    """
    rng = np.random.default_rng(seed)
    s = n / 64.0
    c = (n - 1) / 2.0
    z, y, x = _grid_coords(n)
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    shell = (r >= 22.0 * s) & (r < 26.0 * s)
    cp = np.where(shell, SKULL_CP, WATER_CP)
    cs = np.where(shell, SKULL_CS, 0.0)
    rho = np.where(shell, SKULL_RHO, WATER_RHO)
    alpha = np.zeros_like(cp)
    p0 = np.zeros((n, n, n))
    for _ in range(3):
        R = rng.uniform(2.0, 5.0) * s
        A = rng.uniform(0.5, 1.0)
        # centre uniform in the ball of radius 20 s - R
        while True:
            v = rng.uniform(-1.0, 1.0, size=3)
            if np.dot(v, v) <= 1.0:
                break
        cen = c + v * (20.0 * s - R)
        d = np.sqrt((x - cen[0]) ** 2 + (y - cen[1]) ** 2 + (z - cen[2]) ** 2)
        p0 = p0 + A * (d <= R)
    rec = c + 28.0 * s * fibonacci_sphere(nrec)
    return _finish(f"parity{n}", seed, (n, n, n), dx, nsteps, npml, cp, cs, rho, alpha, p0, rec)


# ----------------------------------------------------------------------------
# recipe 2: ellipsoidal skull shell, smooth +-5% heterogeneity, vessel tubes
# ----------------------------------------------------------------------------

def _smooth_noise(rng, shape, sigma):
    from scipy.ndimage import gaussian_filter
    g = rng.standard_normal(shape, dtype=np.float32)
    g = gaussian_filter(g, sigma, output=np.float32, truncate=3.0)
    m = float(np.max(np.abs(g)))
    return g / m if m > 0 else g


def _angular_field(rng, dirs, nterms=6):
    """Smooth function on the unit sphere with max |h| = 1 over the given directions."""
    h = np.zeros(dirs.shape[:-1])
    for _ in range(nterms):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        f = rng.uniform(1.0, 3.0)
        ph = rng.uniform(0.0, 2 * math.pi)
        h = h + rng.uniform(0.5, 1.0) * np.cos(f * (dirs @ v) + ph)
    m = float(np.max(np.abs(h)))
    return h / m if m > 0 else h


def _tubes(rng, n, semi_in, ntubes, margin_extra=2.0):
    """Max-combined vessel-like tubes inside the inner skull surface."""
    c = (n - 1) / 2.0
    p0 = np.zeros(n * n * n, dtype=np.float32)
    a = np.asarray(semi_in, dtype=np.float64)
    for _ in range(ntubes):
        rad = rng.uniform(1.0, 3.0)
        amp = rng.uniform(0.0, 1.0)
        length = rng.uniform(20.0, 80.0)
        shrink = 1.0 - (margin_extra + rad + 1.0) / a      # keep the tube >= 2 cells inside
        lim = a * shrink

        def inside(p):
            q = (p - c) / lim
            return float(np.dot(q, q)) <= 1.0

        # start: uniform in the allowed ellipsoid, biased towards the outer part
        while True:
            v = rng.uniform(-1.0, 1.0, size=3)
            if np.dot(v, v) <= 1.0 and np.dot(v, v) >= 0.25:
                break
        p = c + v * lim
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        pts = [p.copy()]
        step = 0.5
        for _ in range(int(length / step)):
            d = d + 0.08 * rng.standard_normal(3)
            d /= np.linalg.norm(d)
            q = p + step * d
            if not inside(q):
                d = -d
                q = p + step * d
                if not inside(q):
                    break
            p = q
            pts.append(p.copy())
        pts = np.asarray(pts)
        r_i = int(math.ceil(rad))
        off = np.arange(-r_i, r_i + 1)
        oz, oy, ox = np.meshgrid(off, off, off, indexing="ij")
        off3 = np.stack([ox.ravel(), oy.ravel(), oz.ravel()], axis=1)       # x, y, z
        base = np.rint(pts).astype(np.int64)                               # nearest cell
        cells = (base[:, None, :] + off3[None, :, :]).reshape(-1, 3)
        ctr = np.repeat(pts, off3.shape[0], axis=0)
        dist2 = np.sum((cells - ctr) ** 2, axis=1)
        keep = dist2 <= rad * rad
        cells = cells[keep]
        if cells.size == 0:
            continue
        idx = np.unique(cells[:, 0] + n * (cells[:, 1] + n * cells[:, 2]))
        p0[idx] = np.maximum(p0[idx], np.float32(amp))
    return p0.reshape(n, n, n)


def skull_scenario(n: int = 384, seed: int = 2, nsteps: int = 2500, npml: int = 16,
                   dx: float = 0.1e-3, nrec: int = 1024, ntubes: int | None = None,
                   absorption: bool = True, frequency_dependent: bool = False) -> Scenario:
    """Ellipsoidal skull shell in water with smooth heterogeneity and vessel tubes.

    Inner semi-axes (0.39, 0.36, 0.33) n; radial thickness 8 +- 2 cells from a
    smooth angular field; c_p, c_s, rho of the skull each scaled by
    (1 + 0.05 g) with g a Gaussian-filtered (sigma = 4 cells) noise field with
    max |g| = 1.  Absorption: water one scalar U(0, 2) Np/m, skull 20 Np/m,
    converted to a velocity-damping rate.  p0: max-combined tubes (radius
    1-3 cells, length 20-80 cells, amplitude U(0, 1)) kept >= 2 cells inside
    the inner surface.  Receivers: Fibonacci points on the upper hemisphere of
    radius 0.47 n (180 cells at n = 384).
    """
    rng = np.random.default_rng(seed)
    if ntubes is None:
        ntubes = max(10, int(round(200 * (n / 384.0) ** 2)))
    c = (n - 1) / 2.0
    semi = np.array([0.39, 0.36, 0.33]) * n                 # x, y, z
    z, y, x = _grid_coords(n)
    X, Y, Z = x - c, y - c, z - c
    r = np.sqrt(X * X + Y * Y + Z * Z)
    with np.errstate(invalid="ignore", divide="ignore"):
        inv = np.sqrt((X / semi[0]) ** 2 + (Y / semi[1]) ** 2 + (Z / semi[2]) ** 2)
        r_in = np.where(inv > 0, r / np.where(inv > 0, inv, 1.0), 0.0)   # inner radius along the ray
    # radial thickness 8 +- 2 cells from a smooth angular field
    cand = (r >= r_in) & (r < r_in + 10.5) & (r > 0)
    ci = np.nonzero(cand)
    rc = r[ci]
    dirs = np.stack([X[0, 0, ci[2]] / rc, Y[0, ci[1], 0] / rc, Z[ci[0], 0, 0] / rc], axis=1)
    h = _angular_field(np.random.default_rng(rng.integers(1 << 31)), dirs)
    thick = 8.0 + 2.0 * h
    shell = np.zeros((n, n, n), dtype=bool)
    shell[ci] = (rc - r_in[ci]) < thick
    del dirs, h, cand, ci, rc
    g_cp = _smooth_noise(rng, (n, n, n), 4.0)
    g_cs = _smooth_noise(rng, (n, n, n), 4.0)
    g_rho = _smooth_noise(rng, (n, n, n), 4.0)
    cp = np.where(shell, SKULL_CP * (1.0 + 0.05 * g_cp), WATER_CP)
    cs = np.where(shell, SKULL_CS * (1.0 + 0.05 * g_cs), 0.0)
    rho = np.where(shell, SKULL_RHO * (1.0 + 0.05 * g_rho), WATER_RHO)
    del g_cp, g_cs, g_rho
    if absorption:
        a_water = rng.uniform(0.0, 2.0)
        alpha_x = np.where(shell, 20.0, a_water)
        alpha_t = neper_per_m_to_rate(alpha_x, cp)
    else:
        alpha_t = np.zeros_like(cp)
    p0 = _tubes(rng, n, semi, ntubes)
    p0 = np.where(shell, 0.0, p0)                         # p0 lives in the fluid only
    rec = c + 0.47 * n * fibonacci_sphere(nrec, hemisphere=True)
    sc = _finish(f"skull{n}", seed, (n, n, n), dx, nsteps, npml, cp, cs, rho, alpha_t, p0, rec)
    if frequency_dependent:
        # the skull's attenuation grows with frequency (Sec. 8): its diffusive rate is replaced
        # by two relaxation mechanisms at 0.5 and 2 MHz of equal weight, whose damping rate
        # alpha_r sum_l w_l f^2 / (f_l^2 + f^2) equals the diffusive rate at 1 MHz
        # (0.4 + 0.1 = 0.5 of alpha_r) and rises from 0.25 of it at 0.5 MHz to 0.73 at 2 MHz;
        # the water keeps its diffusive rate, and so do skull cells within npml + 2 cells of a
        # face (on small grids the shell reaches the C-PML, where the plans take no relaxation)
        m = npml + 2 if npml > 0 else 0
        inner = np.zeros((n, n, n), dtype=bool)
        inner[m:n - m, m:n - m, m:n - m] = True
        relax = shell & inner
        sc.mechanisms = [(2.0 * np.pi * 0.5e6, 0.5), (2.0 * np.pi * 2.0e6, 0.5)]
        sc.alpha_r = np.ascontiguousarray(np.where(relax, 2.0 * sc.alpha, 0.0), dtype=np.float32)
        sc.alpha = np.ascontiguousarray(np.where(relax, 0.0, sc.alpha), dtype=np.float32)
        sc.name += "fd"
    return sc


def serving_steps(n: int) -> int:
    """Step count of the serving mix: 800 at 96^3 rising linearly to 1800 at 256^3."""
    return int(round(800 + (n - 96) * 1000.0 / 160.0))


# ----------------------------------------------------------------------------
# recipe 3: small random heterogeneous media for the oracle and parity tests
# ----------------------------------------------------------------------------

def random_scenario(shape_xyz=(12, 10, 9), seed: int = 0, nsteps: int = 20, npml: int = 2,
                    nrec: int = 5, dx: float = 1e-4, fluid_fraction: float = 0.5,
                    absorption: bool = True, cfl: float = CFL) -> Scenario:
    """Blocky random medium mixing fluid (mu = 0) and solid cells, random p0.

    p0 is random over the interior (the operator is linear, so no support
    constraint is needed for operator tests); receivers are uniform inside
    the grid's [0, n-1] box.
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape_xyz
    shp = (nz, ny, nx)
    solid = rng.uniform(size=shp) >= fluid_fraction
    cp = np.where(solid, rng.uniform(2400, 3200, shp), rng.uniform(1400, 1600, shp))
    cs = np.where(solid, rng.uniform(1000, 1600, shp), 0.0)
    rho = np.where(solid, rng.uniform(1500, 2000, shp), rng.uniform(950, 1100, shp))
    if absorption:
        alpha = rng.uniform(0.0, 2.0e5, shp)
    else:
        alpha = np.zeros(shp)
    p0 = rng.standard_normal(shp)
    lo = np.zeros(3)
    hi = np.array([nx - 1, ny - 1, nz - 1], dtype=np.float64)
    rec = lo + rng.uniform(size=(nrec, 3)) * hi
    lam, mu = lame_from_speeds(cp, cs, rho)
    dt = cfl * dx / float(np.max(cp))
    return Scenario(
        name=f"random{nx}x{ny}x{nz}", seed=seed, nx=nx, ny=ny, nz=nz, dx=dx, dt=dt,
        nsteps=nsteps, npml=npml,
        lam=np.ascontiguousarray(lam, dtype=np.float32), mu=np.ascontiguousarray(mu, dtype=np.float32),
        rho=np.ascontiguousarray(rho, dtype=np.float32), alpha=np.ascontiguousarray(alpha, dtype=np.float32),
        p0=np.ascontiguousarray(p0, dtype=np.float32), rec=np.ascontiguousarray(rec * dx))


def transducer_response(dt: float, f0: float = 2.25e6, cycles: float = 2.0) -> np.ndarray:
    """Synthetic electrical impulse response of a transducer, sampled at dt: a sine at the
    centre frequency f0 under a Gaussian window whose half-width is `cycles` periods,
    causal (starting at t = 0), normalised to unit peak.  Stands in for a measured EIR."""
    period = 1.0 / f0
    t = np.arange(int(np.ceil(2 * cycles * period / dt)) + 1) * dt
    tc = cycles * period
    h = np.sin(2 * np.pi * f0 * (t - tc)) * np.exp(-0.5 * ((t - tc) / (0.5 * cycles * period)) ** 2)
    return h / np.max(np.abs(h))


def homogeneous_fluid_scenario(n: int, dx: float, nsteps: int, npml: int, p0: np.ndarray,
                               rec_cells: np.ndarray, cp: float = WATER_CP,
                               rho: float = WATER_RHO) -> Scenario:
    """Homogeneous lossless fluid (mu = 0) with a caller-given p0 and receivers."""
    shp = (n, n, n)
    cpa = np.full(shp, cp)
    return _finish(f"fluid{n}", 0, (n, n, n), dx, nsteps, npml, cpa, np.zeros(shp),
                   np.full(shp, rho), np.zeros(shp), p0, rec_cells)


def gaussian_ball(n: int, centre, width: float, amp: float = 1.0) -> np.ndarray:
    """p0(r) = amp exp(-r^2 / (2 width^2)) in cell units."""
    z, y, x = _grid_coords(n)
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    return amp * np.exp(-r2 / (2.0 * width * width))


CONFIGS = {
    "parity64": dict(recipe="parity", n=64, nsteps=400, npml=8, dx=0.2e-3, nrec=128),
    "skull384": dict(recipe="skull", n=384, nsteps=2500, npml=16, dx=0.1e-3, nrec=1024),
    "skull384fd": dict(recipe="skull", n=384, nsteps=2500, npml=16, dx=0.1e-3, nrec=1024, frequency_dependent=True),
    "skull256": dict(recipe="skull", n=256, nsteps=1800, npml=16, dx=0.1e-3, nrec=1024),
    "skull96": dict(recipe="skull", n=96, nsteps=600, npml=16, dx=0.1e-3, nrec=1024),
    "skull128": dict(recipe="skull", n=128, nsteps=1000, npml=16, dx=0.1e-3, nrec=512),
}


def make(name: str, seed: int | None = None, **over) -> Scenario:
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    recipe = cfg.pop("recipe")
    if seed is not None:
        cfg["seed"] = seed
    if recipe == "parity":
        return parity_scenario(**cfg)
    return skull_scenario(**cfg)
