"""Explicit sparse assembly of the paper's matrices on tiny grids.

TEST INFRASTRUCTURE ONLY (imported by tests/).  It builds, from their block
definitions, the matrices of Mitsuhashi et al.:

  Sec. 2.2 (eq. Operatordef and the stacked J, Phi, Psi), Sec. 3 (eq. W,
  eq. initialp0, eq. interpgrid, eq. H), and the Appendix "Discrete
  formulation" (eq. constPML, eq. opPML, the stacked B, B~, E, E~, Gamma,
  Delta, F = Phi + Gamma E, G = Psi + Delta E~, the 27N x 27N propagator
  W', tau', Theta', and H = M' T'_{M-1} ... T'_1 T'_0).

The diagonal entries (staggered material values, PML a/b/chi tables and the
trilinear receiver weights) are taken from the stencil oracle's model, so a
comparison of this assembly with the stencil oracle checks the update
algebra (which blocks exist, where each derivative and coefficient sits);
the coefficient values have pins of their own.

Readings (same as the stencil oracle): D+ / D- difference types per
component, tau' = -1/3 on the normal stresses, measurement row
-R_l (sigma11 + sigma22 + sigma33).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

C1 = 9.0 / 8.0
C2 = -1.0 / 24.0


def d1(n: int, dx: float, kind: str) -> sp.csr_matrix:
    """1-D 4th-order staggered difference (Sec. 2.2, eq. derivative) with zero extension.

    kind 'p': value at i+1/2 from integer samples; 'm': value at i from the
    half samples stored at index i (position i+1/2).
    """
    rows, cols, vals = [], [], []
    if kind == "p":
        taps = [(1, C1), (0, -C1), (2, C2), (-1, -C2)]
    else:
        taps = [(0, C1), (-1, -C1), (1, C2), (-2, -C2)]
    for i in range(n):
        for o, w in taps:
            q = i + o
            if 0 <= q < n:
                rows.append(i)
                cols.append(q)
                vals.append(w / dx)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


class Assembly:
    """Paper matrices for one oracle model (oracle.oracle.Model)."""

    def __init__(self, model):
        self.m = model
        g = model.g
        self.nx, self.ny, self.nz = g.nx, g.ny, g.nz
        self.N = N = g.nx * g.ny * g.nz
        self.dt = dt = g.dt
        dx = g.dx
        n = (g.nx, g.ny, g.nz)
        I = [sp.identity(k, format="csr") for k in n]

        def along(axis, A):
            mats = [I[2], I[1], I[0]]          # kron order z, y, x (x fastest)
            mats[2 - axis] = A
            return sp.kron(mats[0], sp.kron(mats[1], mats[2], format="csr"), format="csr")

        self.Dp = [along(a, d1(n[a], dx, "p")) for a in range(3)]
        self.Dm = [along(a, d1(n[a], dx, "m")) for a in range(3)]
        cf = model.coefficients()
        diag = lambda v: sp.diags(np.asarray(v).reshape(-1), format="csr")
        Q = [diag(cf["rho_u"][i]) for i in range(3)]
        Qinv = [diag(1.0 / cf["rho_u"][i].reshape(-1)) for i in range(3)]
        A = [diag(cf["alpha_u"][i]) for i in range(3)]
        Lam = diag(cf["lam"])
        Mu = diag(cf["mu"])
        shear_ids = {(1, 2): 0, (0, 2): 1, (0, 1): 2}
        MuS = {k: diag(cf["mu_s"][v]) for k, v in shear_ids.items()}
        self.Q = Q

        def voigt(i, j):
            if i == j:
                return i
            return {(1, 2): 3, (0, 2): 4, (0, 1): 5}[tuple(sorted((i, j)))]

        def Mu_ij(i, j):
            return Mu if i == j else MuS[tuple(sorted((i, j)))]

        # derivative acting on sigma^{ij} along j (velocity update), on u^i along j (stress update)
        def dsig(i, j):
            return self.Dp[j] if i == j else self.Dm[j]

        def du(i, j):
            return self.Dm[j] if i == j else self.Dp[j]

        # PML tables broadcast to N along their axis
        def table(axis, half, which):
            a, b, chi = model.pml_table(axis, half)
            v = {"a": a, "b": b, "chi": chi}[which]
            shp = [1, 1, 1]
            shp[2 - axis] = n[axis]
            return np.broadcast_to(v.reshape(shp), (g.nz, g.ny, g.nx)).reshape(-1)

        # phi^{ij} at the u^i point: half along j iff i == j; psi^{ij} at sigma^{ij}: half iff i != j
        phi_h = lambda i, j: 1 if i == j else 0
        psi_h = lambda i, j: 0 if i == j else 1
        Z = lambda r, c: sp.csr_matrix((r, c))
        Id = sp.identity(N, format="csr")

        # ---- Sec. 2.2: J, Phi, Psi
        self.J = sp.block_diag([Id - dt * A[i] for i in range(3)], format="csr")
        blk = [[None] * 6 for _ in range(3)]
        for i in range(3):
            for j in range(3):
                t = dt * Qinv[i] @ dsig(i, j)
                c = voigt(i, j)
                blk[i][c] = t if blk[i][c] is None else blk[i][c] + t
        self.Phi = sp.bmat([[b if b is not None else Z(N, N) for b in row] for row in blk], format="csr")
        order = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]      # Voigt rows
        blk = [[Z(N, N) for _ in range(3)] for _ in range(6)]
        for r, (i, j) in enumerate(order):
            if i == j:
                for k in range(3):
                    blk[r][k] = blk[r][k] + dt * Lam @ du(k, k)
            # M_ij (d_i u^j + d_j u^i)
            blk[r][j] = blk[r][j] + dt * Mu_ij(i, j) @ du(j, i)
            blk[r][i] = blk[r][i] + dt * Mu_ij(i, j) @ du(i, j)
        self.Psi = sp.bmat(blk, format="csr")

        # ---- Appendix: B, B~, E, E~, Gamma, Delta (eq. constPML, eq. opPML)
        pairs = [(i, j) for i in range(3) for j in range(3)]            # 11,12,13,21,...,33
        self.B = sp.block_diag([diag(table(j, phi_h(i, j), "b")) for i, j in pairs], format="csr")
        self.Bt = sp.block_diag([diag(table(j, psi_h(i, j), "b")) for i, j in pairs], format="csr")
        blk = [[Z(N, N) for _ in range(6)] for _ in range(9)]
        for r, (i, j) in enumerate(pairs):
            blk[r][voigt(i, j)] = diag(table(j, phi_h(i, j), "a")) @ dsig(i, j)
        self.E = sp.bmat(blk, format="csr")
        blk = [[Z(N, N) for _ in range(3)] for _ in range(9)]
        for r, (i, j) in enumerate(pairs):
            blk[r][i] = diag(table(j, psi_h(i, j), "a")) @ du(i, j)
        self.Et = sp.bmat(blk, format="csr")
        blk = [[Z(N, N) for _ in range(9)] for _ in range(3)]
        for c, (i, j) in enumerate(pairs):
            blk[i][c] = dt * Qinv[i] @ diag(table(j, phi_h(i, j), "chi"))
        self.Gamma = sp.bmat(blk, format="csr")
        blk = [[Z(N, N) for _ in range(9)] for _ in range(6)]
        for r, (i, j) in enumerate(order):
            if i == j:
                for k in range(3):
                    blk[r][pairs.index((k, k))] = blk[r][pairs.index((k, k))] + dt * Lam
            Xij = diag(table(j, psi_h(i, j), "chi"))
            Xji = diag(table(i, psi_h(j, i), "chi"))
            blk[r][pairs.index((i, j))] = blk[r][pairs.index((i, j))] + dt * Mu_ij(i, j) @ Xij
            blk[r][pairs.index((j, i))] = blk[r][pairs.index((j, i))] + dt * Mu_ij(i, j) @ Xji
        self.Delta = sp.bmat(blk, format="csr")
        self.F = (self.Phi + self.Gamma @ self.E).tocsr()
        self.G = (self.Psi + self.Delta @ self.Et).tocsr()

        # ---- W' (27N x 27N), state [phi; u; psi; sigma]
        GB = self.Gamma @ self.B
        self.Wp = sp.bmat([
            [self.B, Z(9 * N, 3 * N), Z(9 * N, 9 * N), self.E],
            [GB, self.J, Z(3 * N, 9 * N), self.F],
            [self.Et @ GB, self.Et @ self.J, self.Bt, self.Et @ self.F],
            [self.G @ GB, self.G @ self.J, self.Delta @ self.Bt, sp.identity(6 * N) + self.G @ self.F],
        ], format="csr")

        # ---- Sec. 3 (no PML): W = [[J, Phi], [Psi J, I + Psi Phi]], state [u; sigma]
        self.W = sp.bmat([[self.J, self.Phi],
                          [self.Psi @ self.J, sp.identity(6 * N) + self.Psi @ self.Phi]], format="csr")

        # ---- injection and measurement
        third = -1.0 / 3.0
        self.tau_p = sp.vstack([Z(21 * N, N), third * Id, third * Id, third * Id, Z(3 * N, N)], format="csr")
        self.tau = sp.vstack([Z(3 * N, N), third * Id, third * Id, third * Id, Z(3 * N, N)], format="csr")
        base, w = model.receivers()
        L = base.shape[0]
        R = sp.csr_matrix((w.reshape(-1), (np.repeat(np.arange(L), 8), base.reshape(-1))), shape=(L, N))
        self.R = R
        self.Theta_p = sp.hstack([Z(L, 21 * N), -R, -R, -R, Z(L, 3 * N)], format="csr")
        self.Theta = sp.hstack([Z(L, 3 * N), -R, -R, -R, Z(L, 3 * N)], format="csr")
        self.L = L

    def H_dense(self, M: int, pml: bool = True) -> np.ndarray:
        """Explicit H (LM x N), row blocks p_0 ... p_{M-1} (eq. H / eq. HPML)."""
        W = self.Wp if pml else self.W
        tau = self.tau_p if pml else self.tau
        Th = self.Theta_p if pml else self.Theta
        X = tau.toarray()
        rows = [Th @ X]
        for _ in range(1, M):
            X = W @ X
            rows.append(Th @ X)
        return np.vstack(rows)
