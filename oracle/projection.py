"""Projection onto previous solutions -- plain numpy oracle.

Test infrastructure only (used by the test-suite); the product package never
imports it.

Section 2 of the paper accelerates the successive solves of a time step by
projecting the current solution onto the space spanned by earlier ones
(Fischer's projection method, cited there).  For A symmetric positive
definite and a basis x_1..x_l of earlier solutions kept A-orthonormal
(x_i^T A x_j = delta_ij), the element of their span closest to the solution
of A x = b in the A-norm is

    xbar = sum_i (x_i^T b) x_i,

so the remaining solve is A d = b - A xbar from d = 0, and x = xbar + d
(equivalently: the solve of A x = b started from xbar).  A
new solution enters the basis by Gram-Schmidt in the A-inner product (done
twice for stability) and A-normalisation; a vector whose A-norm after the
orthogonalisation is below drop_tol (1e-8) times its A-norm before is
dropped -- such a remainder is made of the earlier solves' own errors, and
keeping it would steer the next guesses with noise -- and a full basis
restarts from the new vector alone.

All inner products are the unique-dof inner product of the E-vectors
(``OracleMesh.dot``) and A is the masked assembled operator
(``OracleMesh.apply``), so x^T A y = dot(x, apply(y)) for continuous x, y.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np


class ProjectionSpace:
    def __init__(self, mesh, max_vectors: int, h1=None, h2=None, drop_tol: float = 1e-8):
        if max_vectors < 1:
            raise ValueError("max_vectors must be >= 1")
        self.mesh = mesh
        self.max_vectors = int(max_vectors)
        self.h1, self.h2 = h1, h2
        self.drop_tol = drop_tol
        self.X: List[np.ndarray] = []   # A-orthonormal basis
        self.AX: List[np.ndarray] = []  # A applied to each basis vector

    def __len__(self):
        return len(self.X)

    def reset(self):
        self.X, self.AX = [], []

    def _A(self, v):
        return self.mesh.apply(v, self.h1, self.h2)

    def project(self, b) -> np.ndarray:
        """xbar = sum_i (x_i . b) x_i."""
        xbar = np.zeros(self.mesh.nloc)
        for xi in self.X:
            xbar += self.mesh.dot(xi, b) * xi
        return xbar

    def add(self, x) -> bool:
        """A-orthogonalise x against the basis (two passes), A-normalise and
        append it; returns False when it was dropped as dependent."""
        if len(self.X) >= self.max_vectors:
            self.reset()
        v = np.array(x, dtype=np.float64, copy=True)
        Av = self._A(v)
        n0 = self.mesh.dot(v, Av)
        if not n0 > 0.0:
            return False
        for _ in range(2):
            coef = [self.mesh.dot(xi, Av) for xi in self.X]
            for c, xi, axi in zip(coef, self.X, self.AX):
                v -= c * xi
                Av -= c * axi
        n2 = self.mesh.dot(v, Av)
        if not n2 > (self.drop_tol ** 2) * n0:
            return False
        s = 1.0 / np.sqrt(n2)
        self.X.append(v * s)
        self.AX.append(Av * s)
        return True

    def solve(self, b, tol: float = 1e-10, max_iter: int = 5000):
        """Projection, then PCG on A x = b started from xbar (the same iterates
        as PCG on A d = b - A xbar from d = 0), then the solution joins the
        basis.  Returns (x, PCG result)."""
        xbar = self.project(b)
        x, res = self.mesh.pcg(b, x0=xbar, tol=tol, max_iter=max_iter, h1=self.h1, h2=self.h2)
        self.add(x)
        return x, res
