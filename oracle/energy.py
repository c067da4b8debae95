"""Modified energy of the forward recursion, in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the operator library
or its Python binding.  It shares no code with the GPU path.

The leapfrog scheme of Sec. 2.2 (eq. it) advances the velocity at half steps
and the stress at integer steps.  Its spatial operators are skew (the
zero-extended 4th-order differences satisfy Dp^T = -Dm) and the stiffness C
is symmetric, so without absorption and without the C-PML the quantity

  E_m = 1/2 sum_c sum_cells rho_c u^c_{m-1/2} u^c_{m+1/2}
      + 1/2 sigma_m^T C^+ sigma_m

is exactly invariant.  At a normal-stress point with moduli lambda, mu,

  sigma^T C^+ sigma = (tr sigma)^2 / (9 K) + |dev sigma|^2 / (2 mu),
  K = lambda + 2 mu / 3,

where the second term is dropped at fluid points (mu = 0; their deviatoric
stress stays zero, Sec. 2.1), and at a shear point sigma_ij^2 / mu_ij, dropped
where the edge modulus mu_ij vanishes (sigma_ij stays zero there).  rho_c and
mu_ij are the staggered material values of the update itself
(Model.coefficients()).
"""
from __future__ import annotations

import numpy as np


def modified_energy(cf: dict, u_prev, u_next, sig) -> float:
    """E_m from the staggered coefficients cf (Model.coefficients()), the velocities
    u_{m-1/2} (u_prev) and u_{m+1/2} (u_next), three arrays each, and the six Voigt
    stresses sigma_m (11, 22, 33, 23, 13, 12)."""
    rho_u = cf["rho_u"]
    kin = sum(float(np.sum(rho_u[c] * u_prev[c] * u_next[c])) for c in range(3))
    lam, mu = cf["lam"], cf["mu"]
    K = lam + 2.0 * mu / 3.0
    tr = sig[0] + sig[1] + sig[2]
    pot = float(np.sum(tr * tr / (9.0 * K)))
    solid = mu > 0
    dev2 = sum((sig[c] - tr / 3.0) ** 2 for c in range(3))
    pot += float(np.sum(dev2[solid] / (2.0 * mu[solid])))
    for a, sid in ((3, 0), (4, 1), (5, 2)):
        ms = cf["mu_s"][sid]
        nz = ms > 0
        pot += float(np.sum(sig[a][nz] ** 2 / ms[nz]))
    return 0.5 * (kin + pot)


def energy_series(model, p0, nsteps: int, every: int = 1) -> np.ndarray:
    """E_m of the forward recursion started from p0 (tau' injection, u_{-1/2} = 0) for
    m = 0, every, 2 every, ... <= nsteps - 2 (E_m needs u_{m+1/2}, which the update m+1
    produces; a run of nsteps samples has nsteps - 1 updates)."""
    cf = model.coefficients()
    v = model.inject(p0)
    sv = model.state_views(v)
    out = []
    for m in range(max(nsteps - 1, 0)):
        take = m % every == 0
        if take:
            u_prev = [a.copy() for a in sv["u"]]
            sig = [a.copy() for a in sv["sig"]]
        model.step(v)
        if take:
            out.append(modified_energy(cf, u_prev, sv["u"], sig))
    return np.array(out, dtype=np.float64)
