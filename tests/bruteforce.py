"""Independent dense brute-force SEM assembly for tiny meshes (test pin).

Written separately from the oracle, with different formulations throughout, so
that a mistake in the oracle (a transposed D, a wrong g-factor pairing, a wrong
numbering) shows up as a disagreement:
  * GLL nodes from numpy's Legendre roots, weights from the closed form;
  * Lagrange derivative matrix from explicit polynomial products;
  * node coordinates from a numpy trilinear / pipe map;
  * physical gradients grad phi = J^{-T} grad_ref phi at each quadrature point
    (no G factors);
  * global numbering by matching node coordinates (plus the periodic shift).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


def gll_numpy(N):
    cP = np.zeros(N + 1)
    cP[N] = 1.0
    interior = np.sort(np.real(npleg.legroots(npleg.legder(cP))))
    xi = np.concatenate([[-1.0], interior, [1.0]])
    PN = npleg.legval(xi, cP)
    w = 2.0 / (N * (N + 1) * PN ** 2)
    return xi, w


def lagrange_deriv(xi):
    """Dm[i, l] = derivative of the l-th Lagrange polynomial at xi_i."""
    P = len(xi)
    Dm = np.zeros((P, P))
    for l in range(P):
        coef = np.array([1.0])
        for m in range(P):
            if m != l:
                coef = nppoly.polymul(coef, np.array([-xi[m], 1.0]) / (xi[l] - xi[m]))
        Dm[:, l] = nppoly.polyval(xi, nppoly.polyder(coef))
    return Dm


def node_coords(N, nel, lo, hi, vertices=None, pipe=False):
    """Coordinates of every local node, E-vector order (i fastest, then j, k, e)."""
    xi, _ = gll_numpy(N)
    P = N + 1
    nx, ny, nz = nel
    h = [(hi[d] - lo[d]) / nel[d] for d in range(3)]
    X = np.zeros((nx * ny * nz, P, P, P, 3))  # [e, k, j, i, d]
    t = 0.5 * (xi + 1.0)
    T, S, R = np.meshgrid(t, t, t, indexing="ij")  # [k, j, i]
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                e = ex + nx * (ey + ny * ez)
                if pipe:
                    Xs = lo[0] + (ex + R) * h[0]
                    Ys = lo[1] + (ey + S) * h[1]
                    Zs = lo[2] + (ez + T) * h[2]
                    X[e, ..., 0] = Xs * np.sqrt(1 - Ys ** 2 / 2)
                    X[e, ..., 1] = Ys * np.sqrt(1 - Xs ** 2 / 2)
                    X[e, ..., 2] = Zs
                    continue
                acc = np.zeros((P, P, P, 3))
                for c in range(8):
                    vx, vy, vz = ex + (c & 1), ey + ((c >> 1) & 1), ez + ((c >> 2) & 1)
                    if vertices is not None:
                        V = vertices[vx + (nx + 1) * (vy + (ny + 1) * vz)]
                    else:
                        V = np.array([lo[0] + vx * h[0], lo[1] + vy * h[1], lo[2] + vz * h[2]])
                    wgt = ((R if c & 1 else 1 - R) * (S if (c >> 1) & 1 else 1 - S)
                           * (T if (c >> 2) & 1 else 1 - T))
                    acc += wgt[..., None] * V
                X[e] = acc
    return X.reshape(-1, 3)


def number_by_coords(X, period=None, tol=1e-9):
    """Global ids by coordinate matching (periodic along z when period given)."""
    key = X.copy()
    if period is not None:
        key[:, 2] = np.mod(key[:, 2], period)
        key[np.abs(key[:, 2] - period) < tol, 2] = 0.0
    q = np.round(key / tol).astype(np.int64)
    _, inv = np.unique(q, axis=0, return_inverse=True)
    return inv.reshape(-1)


def element_stiffness(N, Xe, drop=None):
    """Dense element stiffness sum_q W_q detJ_q grad phi_a . grad phi_b (and the
    lumped mass W detJ) from physical gradients; Xe is (P^3, 3)."""
    xi, w = gll_numpy(N)
    P = N + 1
    Dm = lagrange_deriv(xi)
    I = np.eye(P)
    # index = i + P j + P^2 k  ->  kron(k-factor, j-factor, i-factor)
    Dr = np.kron(I, np.kron(I, Dm))
    Ds = np.kron(I, np.kron(Dm, I))
    Dt = np.kron(Dm, np.kron(I, I))
    W = np.kron(w, np.kron(w, w))  # weight of point i + P j + P^2 k
    J = np.stack([np.stack([Dr @ Xe[:, a], Ds @ Xe[:, a], Dt @ Xe[:, a]], axis=-1)
                  for a in range(3)], axis=1)  # [q, a(x,y,z), b(r,s,t)]
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)  # [q, (r,s,t), (x,y,z)]
    ref = [Dr, Ds, Dt]
    wq = W * detJ
    if drop is not None:
        wq = np.where(drop, 0.0, wq)
    Ae = np.zeros((P ** 3, P ** 3))
    for d in range(3):  # physical direction x, y, z
        Gd = sum(Jinv[:, b, d][:, None] * ref[b] for b in range(3))
        Ae += Gd.T @ (wq[:, None] * Gd)
    return Ae, wq


def assemble(N, X, gid, drop=None):
    """Assembled dense stiffness A_G (nglob x nglob) and lumped mass B_G."""
    P3 = (N + 1) ** 3
    E = X.shape[0] // P3
    ng = int(gid.max()) + 1
    A = np.zeros((ng, ng))
    Bg = np.zeros(ng)
    for e in range(E):
        sl = slice(e * P3, (e + 1) * P3)
        Ae, wq = element_stiffness(N, X[sl], None if drop is None else drop[sl])
        g = gid[sl]
        A[np.ix_(g, g)] += Ae
        np.add.at(Bg, g, wq)
    return A, Bg
