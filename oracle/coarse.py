"""Two-level preconditioner: Jacobi plus the coarse term of Eq. 6 -- plain
numpy oracle.

Test infrastructure only (used by the test-suite); the product package never
imports it.

Eq. 6 of the paper adds to the local solves a coarse correction
R_0^T A_0^{-1} R_0 on a problem with few unknowns that spans the whole
domain.  With single-node subdomains the local sum is the Jacobi
preconditioner D^{-1}, so this oracle computes

    M^{-1} r = D^{-1} r + P C(A_0) P^T r,

with these choices (the paper leaves them open):

* Coarse space: the trilinear (Q1) hat functions of the element vertices,
  evaluated at the GLL nodes in each element's reference coordinates, set to
  0 at Dirichlet nodes; P is the n_global x n_vertex matrix of their values.
  Every vertex whose masked hat function is not zero is a coarse unknown.
* A_0 = P^T A P (Galerkin), with A the masked assembled operator.
* C(A_0) replaces A_0^{-1}: k steps of Chebyshev iteration for
  D_0^{-1} A_0 z = D_0^{-1} r_0 from z = 0, D_0 = diag(A_0), on the interval
  [a, b] with b the largest absolute row sum of D_0^{-1} A_0 (an upper bound
  of its spectrum) and a = frac * b.  A fixed polynomial, so M is linear; it
  is positive on (0, b], so M is symmetric positive definite.

Vectors are E-vectors: P^T r sums over unique nodes (local sum weighted by
1/mult) and P z0 is continuous.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class CoarseOracle:
    def __init__(self, mesh, k: int = 20, frac: float = 0.01, h1=None, h2=None):
        self.m = mesh
        self.k, self.frac = int(k), float(frac)
        self.h1, self.h2 = h1, h2
        N, P = mesh.N, mesh.P
        nx, ny, nz = mesh.nel
        per = mesh.periodic
        self.vdims = (nx + 1 - per[0], ny + 1 - per[1], nz + 1 - per[2])
        vx, vy, vz = self.vdims
        self.nvert = vx * vy * vz
        gid = mesh.numbering()
        l = np.stack([(1.0 - mesh.xi) / 2.0, (1.0 + mesh.xi) / 2.0])  # [corner side, i]
        rows, cols, vals = [], [], []
        self.evert = np.zeros((mesh.E, 8), dtype=np.int64)
        for e in range(mesh.E):
            ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
            g = gid[e * P ** 3:(e + 1) * P ** 3]
            for c in range(8):
                cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
                v = ((ex + cx) % vx) + vx * (((ey + cy) % vy) + vy * ((ez + cz) % vz))
                self.evert[e, c] = v
                phi = np.einsum("k,j,i->kji", l[cz], l[cy], l[cx]).reshape(-1)
                rows.append(g)
                cols.append(np.full(P ** 3, v))
                vals.append(phi)
        # every copy of a node carries the same hat value: keep one per node
        coo = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                            shape=(mesh.nglob, self.nvert))
        Pm = coo.tocsr()
        Pm.sum_duplicates()
        mult = np.bincount(gid, minlength=mesh.nglob).astype(float)
        live = (mesh.global_mask() == 0).astype(float)
        self.P = (sp.diags(live / mult) @ Pm).tocsc()
        self.A0 = self._galerkin()
        self.keep = np.abs(np.diag(self.A0)) > 0
        self.A0k = self.A0[np.ix_(self.keep, self.keep)]
        self.D0 = np.diag(self.A0k).copy()
        self.b = float(np.max(np.sum(np.abs(self.A0k / self.D0[:, None]), axis=1)))
        self.a = self.frac * self.b
        self.inv = mesh.jacobi(h1, h2)

    # -- pieces -----------------------------------------------------------------
    def prolong(self, z0):
        """P z0 as a continuous, masked E-vector (z0 over all vertices)."""
        return (self.P @ z0)[self.m.numbering()]

    def restrict(self, r):
        """P^T r for a continuous E-vector r (over all vertices)."""
        g = np.zeros(self.m.nglob)
        g[self.m.numbering()] = r
        return self.P.T @ g

    def _galerkin(self):
        A0 = np.zeros((self.nvert, self.nvert))
        for v in range(self.nvert):
            e = np.zeros(self.nvert)
            e[v] = 1.0
            A0[:, v] = self.restrict(self.m.apply(self.prolong(e), self.h1, self.h2))
        return A0

    def chebyshev(self, r0k):
        """k steps of Chebyshev iteration for D0^-1 A0 z = D0^-1 r0 (kept vertices)."""
        theta, delta = (self.b + self.a) / 2.0, (self.b - self.a) / 2.0
        sigma = theta / delta
        rho = 1.0 / sigma
        z = np.zeros_like(r0k)
        res = r0k.copy()
        d = (res / self.D0) / theta
        for _ in range(self.k):
            z = z + d
            res = res - self.A0k @ d
            rho_new = 1.0 / (2.0 * sigma - rho)
            d = rho_new * rho * d + (2.0 * rho_new / delta) * (res / self.D0)
            rho = rho_new
        return z

    def coarse(self, r):
        """P C(A0) P^T r."""
        r0 = self.restrict(r)
        z0 = np.zeros(self.nvert)
        z0[self.keep] = self.chebyshev(r0[self.keep])
        return self.prolong(z0)

    def apply(self, r):
        """M^{-1} r = D^{-1} r + P C(A0) P^T r."""
        return self.inv * r + self.coarse(r)
