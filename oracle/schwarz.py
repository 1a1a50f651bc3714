"""Overlapping additive Schwarz preconditioner (Eq. 6, its sum over local
subdomains) -- plain numpy oracle.

Test infrastructure only (used by the test-suite); the product package never
imports it.

Eq. 6 of the paper writes the pressure preconditioner as a coarse term plus
a sum of local solves on overlapping subdomains,
    M^{-1} = R_0^T A_0^{-1} R_0 + sum_k R_k^T A_k^{-1} R_k .
This oracle implements the sum over the local subdomains (the coarse term is
not part of it), with the following choices, which the paper leaves open:

* Subdomain k is element k extended by one node layer into every neighbour
  (minimal overlap): extended indices (i, j, k) in [-1, N+1]^3, where -1 is
  the previous neighbour's node N-1 and N+1 the next neighbour's node 1, also
  across periodic faces.  Nodes beyond a non-periodic face do not exist; nodes
  on a Dirichlet face are not unknowns.
* A_k is the separable approximation of the local stiffness on a box with the
  element's mean edge lengths l_r, l_s, l_t (the fast-diagonalisation form):
      A_k = B_t x B_s x A_r + B_t x A_s x B_r + A_t x B_s x B_r
  with A_d, B_d the 1-D GLL stiffness and lumped mass of the element (length
  l_d) and of a copy of it on each side that has a neighbour, assembled on the
  3N+1 nodes of the three and restricted to the subdomain's nodes in that
  direction (x: Kronecker product, the r index fastest).  On an affine mesh of
  equal box elements this is exactly R_k A R_k^T.
* z = sum_k R_k^T A_k^{-1} R_k r, each local system solved densely here;
  Dirichlet nodes of z are 0.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np
from scipy.linalg import cho_factor, cho_solve

INTERIOR, DIRICHLET, NEUMANN = 0, 1, 2


def one_d(N: int, xi, w, D, ell: float, left: int, right: int) -> Tuple[np.ndarray, np.ndarray, List[int]]:
    """1-D stiffness and lumped mass of the extended element of length ell;
    returns (A1, B1 diagonal, kept extended indices in [-1, N+1])."""
    P = N + 1
    Ke = (2.0 / ell) * (D.T @ np.diag(w) @ D)
    Me = (ell / 2.0) * w
    n = 3 * N + 1
    K = np.zeros((n, n))
    M = np.zeros(n)
    parts = [1]
    if left == INTERIOR:
        parts.append(0)
    if right == INTERIOR:
        parts.append(2)
    for p in parts:
        sl = slice(p * N, p * N + P)
        K[sl, sl] += Ke
        M[sl] += Me
    lo = -1 if left == INTERIOR else (0 if left == NEUMANN else 1)
    hi = N + 1 if right == INTERIOR else (N if right == NEUMANN else N - 1)
    kept = list(range(lo, hi + 1))
    g = [N + i for i in kept]
    return K[np.ix_(g, g)], M[g], kept


class SchwarzOracle:
    def __init__(self, mesh):
        self.m = mesh
        self.N, self.P = mesh.N, mesh.P
        self.nel = mesh.nel
        self.gid = mesh.numbering()
        self.lmask = mesh.local_mask()
        x, y, z = mesh.coords()
        self.X = np.stack([x, y, z], axis=-1)
        self._chol = {}

    # -- geometry of the subdomains -----------------------------------------
    def elem_xyz(self, e):
        P = self.P
        return self.X[e * P ** 3:(e + 1) * P ** 3].reshape(P, P, P, 3)  # [k, j, i, :]

    def lengths(self, e):
        """Mean straight edge length of the element along r, s, t."""
        Xe = self.elem_xyz(e)
        N = self.N
        c = [0, N]
        lr = np.mean([np.linalg.norm(Xe[k, j, N] - Xe[k, j, 0]) for k in c for j in c])
        ls = np.mean([np.linalg.norm(Xe[k, N, i] - Xe[k, 0, i]) for k in c for i in c])
        lt = np.mean([np.linalg.norm(Xe[N, j, i] - Xe[0, j, i]) for j in c for i in c])
        return lr, ls, lt

    def elem_pos(self, e):
        nx, ny, _ = self.nel
        return e % nx, (e // nx) % ny, e // (nx * ny)

    def sides(self, e):
        """(left, right) kind per direction r, s, t."""
        pos = self.elem_pos(e)
        out = []
        for d in range(3):
            kinds = []
            for hi_side in (0, 1):
                at_edge = pos[d] == (self.nel[d] - 1 if hi_side else 0)
                if not at_edge or self.m.periodic[d]:
                    kinds.append(INTERIOR)
                elif (self.m.dirichlet >> (2 * d + hi_side)) & 1:
                    kinds.append(DIRICHLET)
                else:
                    kinds.append(NEUMANN)
            out.append(tuple(kinds))
        return out

    def ext_gid(self, e, i, j, k):
        """Global id of extended node (i, j, k) of element e, or -1."""
        N, P = self.N, self.P
        pos = list(self.elem_pos(e))
        loc = []
        for d, v in enumerate((i, j, k)):
            if v == -1:
                pos[d] -= 1
                loc.append(N - 1)
            elif v == N + 1:
                pos[d] += 1
                loc.append(1)
            else:
                loc.append(v)
            if pos[d] < 0 or pos[d] >= self.nel[d]:
                if not self.m.periodic[d]:
                    return -1
                pos[d] %= self.nel[d]
        nx, ny, _ = self.nel
        en = pos[0] + nx * (pos[1] + ny * pos[2])
        return int(self.gid[en * P ** 3 + loc[0] + P * (loc[1] + P * loc[2])])

    def local_system(self, e):
        """(dense A_k over the kept nodes, their global ids)."""
        lr, ls, lt = self.lengths(e)
        (l0, r0), (l1, r1), (l2, r2) = self.sides(e)
        m = self.m
        Ar, Br, kr = one_d(self.N, m.xi, m.w, m.D, lr, l0, r0)
        As, Bs, ks = one_d(self.N, m.xi, m.w, m.D, ls, l1, r1)
        At, Bt, kt = one_d(self.N, m.xi, m.w, m.D, lt, l2, r2)
        Dr, Ds, Dt = np.diag(Br), np.diag(Bs), np.diag(Bt)
        A = np.kron(Dt, np.kron(Ds, Ar)) + np.kron(Dt, np.kron(As, Dr)) + np.kron(At, np.kron(Ds, Dr))
        ids = np.array([self.ext_gid(e, i, j, k) for k in kt for j in ks for i in kr], dtype=np.int64)
        return A, ids

    # -- application -----------------------------------------------------------
    def apply(self, r):
        """z = sum_k R_k^T A_k^{-1} R_k r for a continuous E-vector r; returns
        the continuous, masked E-vector z."""
        gm = self.m.global_mask()
        rg = np.zeros(self.m.nglob)
        rg[self.gid] = r
        rg[gm == 1] = 0.0
        zg = np.zeros(self.m.nglob)
        for e in range(self.m.E):
            if e not in self._chol:
                A, ids = self.local_system(e)
                assert np.all(ids >= 0)
                self._chol[e] = (cho_factor(A), ids)
            cf, ids = self._chol[e]
            y = cho_solve(cf, rg[ids])
            np.add.at(zg, ids, y)
        zg[gm == 1] = 0.0
        return zg[self.gid]


def pcg(mesh, b, precond, tol: float = 1e-10, max_iter: int = 5000, x0=None):
    """Preconditioned CG on the masked assembled system with unique-dof inner
    products; stops when the recursive residual is <= tol ||b||.  Returns
    (x, iterations)."""
    x = np.zeros(mesh.nloc) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = b - mesh.apply(x)
    bn = np.sqrt(mesh.dot(b, b))
    if np.sqrt(mesh.dot(r, r)) <= tol * bn:
        return x, 0
    z = precond(r)
    p = z.copy()
    rz = mesh.dot(r, z)
    for it in range(1, max_iter + 1):
        w = mesh.apply(p)
        alpha = rz / mesh.dot(p, w)
        x += alpha * p
        r -= alpha * w
        if np.sqrt(mesh.dot(r, r)) <= tol * bn:
            return x, it
        z = precond(r)
        rz_new = mesh.dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, max_iter
