"""Pins of the oracle's frequency-dependent absorption (relaxation mechanisms).

The paper's absorption is diffusive: a velocity damping alpha u whose rate does
not depend on frequency (Sec. 2.1, eq. subeq1); its conclusion (Sec. 8) names a
frequency-dependent attenuation model as the next step.  The reading built here
adds relaxation mechanisms to the same damping term:

    d/dt u + alpha u + sum_l beta_l (u - zeta_l) = div(sigma) / rho,
    d/dt zeta_l = omega_l (u - zeta_l),        beta_l = w_l alpha_r,

so that the damping rate is a(omega) = alpha + sum_l beta_l i omega / (omega_l + i omega),
growing with frequency.  These tests pin the oracle's implementation against
things other than itself:
  - alpha_r = 0 reduces it bit for bit to the diffusive operator;
  - the adjoint is the transpose: explicit H and H^T columns on a tiny grid,
    and the dot-product test;
  - the attenuation and phase velocity of a spherical wave in a homogeneous
    fluid, measured between two radii, follow the closed-form dispersion
    relation of the scheme, K(k)^2 c^2 = Omega^2 - i Omega a_d(omega), at three
    frequencies, and differ from the frequency-independent model as the
    closed form says they should.
"""
import numpy as np
import pytest

from oracle.oracle import Model
from paper_1709_02733_amd import scenarios as S

TWO_MECH = [(2 * np.pi * 0.3e6, 0.5), (2 * np.pi * 1.5e6, 0.5)]


def _relax_model(sc, alpha_r, mech=TWO_MECH, **over):
    return Model.from_scenario(sc, alpha_r=alpha_r, mechanisms=mech, **over)


def test_zero_strength_is_the_diffusive_operator():
    sc = S.random_scenario((11, 9, 8), seed=21, nsteps=25, npml=2, nrec=6)
    plain = Model.from_scenario(sc)
    relax = _relax_model(sc, np.zeros(sc.shape, np.float32))
    assert relax.state_len == (27 + 6) * relax.N
    p0 = sc.p0.astype(np.float64)
    tr = plain.forward(p0)
    assert np.array_equal(relax.forward(p0), tr)
    assert np.array_equal(relax.adjoint(tr), plain.adjoint(tr))


def test_relaxation_changes_the_operator_and_is_linear():
    sc = S.random_scenario((11, 9, 8), seed=22, nsteps=25, npml=2, nrec=6)
    rng = np.random.default_rng(0)
    ar = rng.uniform(0.0, 3e6, sc.shape).astype(np.float32)
    plain, relax = Model.from_scenario(sc), _relax_model(sc, ar)
    a, b = rng.standard_normal(sc.shape), rng.standard_normal(sc.shape)
    ha, hb, hab = relax.forward(a), relax.forward(b), relax.forward(2.0 * a - 3.0 * b)
    assert np.max(np.abs(hab - (2.0 * ha - 3.0 * hb))) <= 1e-12 * np.max(np.abs(hab))
    # the extra damping takes energy out: the traces differ from the diffusive ones
    assert np.linalg.norm(ha - plain.forward(a)) > 1e-3 * np.linalg.norm(ha)


def test_transposed_columns_on_a_tiny_grid():
    """H assembled column by column (forward of unit p0) equals the transpose of H^T
    assembled column by column (adjoint of unit traces): C-PML, absorption, solid and
    fluid cells, two relaxation mechanisms."""
    sc = S.random_scenario((7, 6, 5), seed=23, nsteps=6, npml=1, nrec=3)
    rng = np.random.default_rng(1)
    ar = rng.uniform(0.5e6, 3e6, sc.shape).astype(np.float32)
    m = _relax_model(sc, ar)
    N, LM = m.N, sc.nsteps * sc.nrec
    H = np.zeros((LM, N))
    for q in range(N):
        e = np.zeros(N)
        e[q] = 1.0
        H[:, q] = m.forward(e.reshape(sc.shape)).ravel()
    HT = np.zeros((N, LM))
    for r in range(LM):
        e = np.zeros(LM)
        e[r] = 1.0
        HT[:, r] = m.adjoint(e.reshape(sc.nsteps, sc.nrec)).ravel()
    assert np.max(np.abs(H)) > 0
    assert np.max(np.abs(HT.T - H)) <= 1e-13 * np.max(np.abs(H))


def test_dot_product_with_relaxation():
    sc = S.random_scenario((17, 13, 11), seed=24, nsteps=40, npml=2, nrec=9)
    rng = np.random.default_rng(2)
    ar = rng.uniform(0.0, 3e6, sc.shape).astype(np.float32)
    m = _relax_model(sc, ar)
    p, q = rng.standard_normal(sc.shape), rng.standard_normal(sc.shape)
    y = m.forward(q)
    lhs = float(np.sum(m.forward(p) * y))
    rhs = float(np.sum(p * m.adjoint(y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# --------------------------------------------------------------------------------------
# Attenuation and dispersion against the closed form
# --------------------------------------------------------------------------------------

def _discrete_wavenumber(om, dt, dx, c, alpha, mechs, alpha_r):
    """Complex wavenumber k (e^{i(omega t - k x)}) of a plane wave along a grid axis under
    the leapfrog scheme with the 4th-order staggered difference:
      K(k)^2 c^2 = Omega^2 - i Omega a_d,
      Omega = 2 sin(omega dt / 2) / dt,   K(k) = (2/dx)(9/8 sin(k dx/2) - 1/24 sin(3 k dx/2)),
      a_d = z^{-1/2} [alpha + sum_l beta_l z (z - 1) / (z - c_l)],  z = e^{i omega dt},
    the last from u^{n+1/2} = (J u^{n-1/2} + dt F + dt sum beta_l zeta_l^{n-1/2}) / (1 + dt B),
    zeta_l^{n+1/2} = c_l zeta_l^{n-1/2} + (1 - c_l) u^{n+1/2} in the frequency domain."""
    z = np.exp(1j * om * dt)
    Om = 2.0 * np.sin(om * dt / 2.0) / dt
    ad = alpha + 0j
    for wl, wt in mechs:
        cl = np.exp(-wl * dt)
        ad = ad + wt * alpha_r * z * (z - 1.0) / (z - cl)
    ad = ad / np.sqrt(z)
    Kt = np.sqrt(Om * Om - 1j * Om * ad) / c
    if Kt.real < 0:
        Kt = -Kt
    k = Kt
    for _ in range(60):                       # Newton on K(k) = Kt
        f = (2.0 / dx) * (9.0 / 8.0 * np.sin(k * dx / 2.0) - np.sin(1.5 * k * dx) / 24.0) - Kt
        fp = 9.0 / 8.0 * np.cos(k * dx / 2.0) - np.cos(1.5 * k * dx) / 8.0
        k = k - f / fp
    return k


def _spherical_ratio(alpha, alpha_r, mechs):
    """Spherical wave from a Gaussian p0 in homogeneous water (96^3, dx 0.1 mm, C-PML 10):
    spectra at 8 and 22 cells on the six axis directions; returns (omega grid, measured
    attenuation, measured wavenumber, dt) from P(r2) r2 / (P(r1) r1) = e^{-i k (r2 - r1)}."""
    n, dx, c, P, ctr, M = 96, 1e-4, 1500.0, 10, 48, 170
    dt = S.CFL * dx / c
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    p0 = np.exp(-((x - ctr) ** 2 + (y - ctr) ** 2 + (z - ctr) ** 2) / 8.0)
    radii = (8, 22)
    rec = []
    for r in radii:
        for s in (1, -1):
            for ax in range(3):
                v = [ctr, ctr, ctr]
                v[ax] += s * r
                rec.append(v)
    shp = (n, n, n)
    kw = dict(alpha_r=np.full(shp, alpha_r, np.float32), mechanisms=mechs) if mechs else {}
    m = Model(n, n, n, dx, dt, M, P, np.full(shp, 1000.0 * c * c, np.float32), np.zeros(shp, np.float32),
              np.full(shp, 1000.0, np.float32), np.full(shp, alpha, np.float32), np.array(rec, float) * dx, **kw)
    tr = m.forward(p0)
    # the window ends before the first reflection from the layer reaches the outer receivers
    w = np.ones(M)
    w[-15:] = 0.5 * (1.0 + np.cos(np.pi * np.arange(15) / 15))
    nfft = 4096
    P1 = np.fft.rfft(tr[:, :6] * w[:, None], nfft, axis=0).mean(axis=1)
    P2 = np.fft.rfft(tr[:, 6:] * w[:, None], nfft, axis=0).mean(axis=1)
    om = 2.0 * np.pi * np.fft.rfftfreq(nfft, dt)
    ratio = P2 * radii[1] / (P1 * radii[0])
    d = (radii[1] - radii[0]) * dx
    return om, -np.log(np.abs(ratio)) / d, -np.unwrap(np.angle(ratio)) / d, dt


@pytest.mark.parametrize("alpha,alpha_r,mechs", [(2.0e5, 0.0, None), (1.0e5, 1.0e6, TWO_MECH)])
def test_attenuation_and_dispersion_follow_the_closed_form(alpha, alpha_r, mechs):
    om, att, kr, dt = _spherical_ratio(alpha, alpha_r, mechs)
    got = []
    for f in (0.6e6, 0.9e6, 1.2e6):
        i = int(np.argmin(np.abs(om - 2.0 * np.pi * f)))
        k = _discrete_wavenumber(om[i], dt, 1e-4, 1500.0, alpha, mechs or [], alpha_r)
        assert abs(att[i] - (-k.imag)) <= 0.05 * (-k.imag), (f, att[i], -k.imag)
        assert abs(kr[i] - k.real) <= 0.005 * k.real, (f, kr[i], k.real)
        got.append(att[i])
    if mechs:
        # the relaxation mechanisms make the attenuation grow with frequency (closed form:
        # 1.38x from 0.6 to 1.2 MHz for these mechanisms) ...
        assert got[2] / got[0] > 1.25
    else:
        # ... while the diffusive model's is flat: alpha / (2 c)
        assert abs(got[2] / got[0] - 1.0) < 0.01
        assert abs(got[1] - alpha / (2 * 1500.0)) <= 0.01 * alpha / (2 * 1500.0)
