"""Conditioning of the pipe's geometric factors next to the map's singular corners.

The square-to-disk map has det J = 0 where the square's corners are; the nodes
next to them have small det J, and the factors W det(J) J^{-1} J^{-T} computed
from FP64 node coordinates by differentiation lose digits there.  This test
evaluates the same isoparametric factors in 80-bit extended precision on the
corner elements and shows that the oracle and the library are both within a
stated bound of it -- so a difference between the two of that size is rounding,
not a defect, and the pipe tolerances elsewhere in the suite follow from it.
"""
import numpy as np
import pytest

from libhost import host_setup

LD = np.longdouble


def _gll_ld(N):
    """GLL nodes/weights in extended precision by Newton on P'_N."""
    def leg(n, x):
        p0, p1 = np.ones_like(x), x.copy()
        d0, d1 = np.zeros_like(x), np.ones_like(x)
        for m in range(1, n):
            p2 = ((2 * m + 1) * x * p1 - m * p0) / (m + 1)
            d2 = d0 + (2 * m + 1) * p1
            p0, p1, d0, d1 = p1, p2, d1, d2
        return p1, d1
    x = -np.cos(np.pi * np.arange(N + 1, dtype=LD) / N)
    for _ in range(60):
        p, dp = leg(N, x[1:-1])
        ddp = (2 * x[1:-1] * dp - N * (N + 1) * p) / (1 - x[1:-1] ** 2)
        x[1:-1] -= dp / ddp
    x[0], x[-1] = LD(-1), LD(1)
    p, _ = leg(N, x)
    w = LD(2) / (N * (N + 1) * p * p)
    D = np.zeros((N + 1, N + 1), dtype=LD)
    for i in range(N + 1):
        for l in range(N + 1):
            if i != l:
                D[i, l] = p[i] / (p[l] * (x[i] - x[l]))
    D[0, 0], D[N, N] = -LD(N * (N + 1)) / 4, LD(N * (N + 1)) / 4
    return x, w, D


def _geom_ld(N, nel, elems):
    """Extended-precision factors for the listed elements of the pipe."""
    xi, w, D = _gll_ld(N)
    P = N + 1
    nx, ny, nz = nel
    h = [LD(2) / nx, LD(2) / ny, LD(10) / nz]
    t = (xi + 1) / 2
    out = []
    for e in elems:
        ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
        T, S, R = np.meshgrid(t, t, t, indexing="ij")
        Xs, Ys, Zs = -1 + (ex + R) * h[0], -1 + (ey + S) * h[1], (ez + T) * h[2]
        X = [Xs * np.sqrt(1 - Ys * Ys / 2), Ys * np.sqrt(1 - Xs * Xs / 2), Zs]  # [k,j,i]
        J = np.zeros((3, 3, P, P, P), dtype=LD)
        for a in range(3):
            J[a, 0] = np.einsum("il,kjl->kji", D, X[a])
            J[a, 1] = np.einsum("jl,kli->kji", D, X[a])
            J[a, 2] = np.einsum("kl,lji->kji", D, X[a])
        C = np.zeros_like(J)
        C[0, 0] = J[1, 1] * J[2, 2] - J[1, 2] * J[2, 1]
        C[0, 1] = J[1, 2] * J[2, 0] - J[1, 0] * J[2, 2]
        C[0, 2] = J[1, 0] * J[2, 1] - J[1, 1] * J[2, 0]
        C[1, 0] = J[0, 2] * J[2, 1] - J[0, 1] * J[2, 2]
        C[1, 1] = J[0, 0] * J[2, 2] - J[0, 2] * J[2, 0]
        C[1, 2] = J[0, 1] * J[2, 0] - J[0, 0] * J[2, 1]
        C[2, 0] = J[0, 1] * J[1, 2] - J[0, 2] * J[1, 1]
        C[2, 1] = J[0, 2] * J[1, 0] - J[0, 0] * J[1, 2]
        C[2, 2] = J[0, 0] * J[1, 1] - J[0, 1] * J[1, 0]
        det = J[0, 0] * C[0, 0] + J[0, 1] * C[0, 1] + J[0, 2] * C[0, 2]
        W = w[:, None, None] * w[None, :, None] * w[None, None, :]
        pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
        g = np.stack([W * sum(C[a, b] * C[a, c] for a in range(3)) / det for b, c in pairs])
        g = g.reshape(6, -1)
        # dropped quadrature points at the square's corners
        sing = np.zeros((P, P, P), dtype=bool)
        for j in range(P):
            for i in range(P):
                xe = (ex == 0 and i == 0) or (ex == nx - 1 and i == N)
                ye = (ey == 0 and j == 0) or (ey == ny - 1 and j == N)
                sing[:, j, i] = xe and ye
        g[:, sing.reshape(-1)] = 0
        out.append(g)
    return np.concatenate(out, axis=1)


@pytest.mark.skipif(np.finfo(np.longdouble).eps > 1e-18, reason="needs 80-bit long double")
@pytest.mark.parametrize("N", [7, 9])
def test_pipe_geometry_rounding_is_conditioning(oracle_mod, N):
    nel = (48, 48, 1)
    nx, ny, _ = nel
    corners = [0, nx - 1, nx * (ny - 1), nx * ny - 1]
    neighbours = [1, nx, nx + 1]
    elems = np.array(sorted(set(corners + neighbours)), dtype=np.int64)
    exact = _geom_ld(N, nel, elems).astype(np.float64)
    om = oracle_mod.pipe_mesh(*nel, N=N)
    Go, _ = om.geom(elems)
    h = host_setup(N=N, nel=nel, periodic=(0, 0, 1), lo=(-1, -1, 0), hi=(1, 1, 10), mapping=1)
    P3 = (N + 1) ** 3
    Gl = np.concatenate([h["G"][:, e * P3:(e + 1) * P3] for e in elems], axis=1)
    nrm = np.linalg.norm(exact)
    err_o = np.linalg.norm(Go - exact) / nrm
    err_l = np.linalg.norm(Gl - exact) / nrm
    diff = np.linalg.norm(Go - Gl) / nrm
    # both FP64 evaluations carry a rounding error of the same order, set by the
    # conditioning near the corners; their difference is bounded by the sum
    bound = {7: 2e-11, 9: 2e-10}[N]
    assert err_o < bound and err_l < bound, (err_o, err_l)
    assert diff <= err_o + err_l + 1e-15
    # away from the corner elements both are accurate to ~1e-13
    far = np.array([nx // 2 + nx * (ny // 2)], dtype=np.int64)
    ex_far = _geom_ld(N, nel, far).astype(np.float64)
    Gf = h["G"][:, far[0] * P3:(far[0] + 1) * P3]
    assert np.linalg.norm(Gf - ex_far) <= 1e-13 * np.linalg.norm(ex_far)
    assert np.linalg.norm(om.geom(far)[0] - ex_far) <= 1e-13 * np.linalg.norm(ex_far)
