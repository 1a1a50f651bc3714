"""Pins of the oracle's mesh coordinates and geometric factors (CPU only).

Algorithm 1 combines the reference derivatives with six factors g1..g6; with
the quadrature weight and det J folded in they are W det(J) J^{-1} J^{-T}
(g1=rr, g2=ss, g3=tt, g4=rs, g5=rt, g6=st), and B = W det J is the lumped mass.
"""
import numpy as np
import pytest

import seeded_inputs as SI
from bruteforce import element_stiffness, gll_numpy, lagrange_deriv, node_coords


def test_undistorted_box_closed_form(oracle_mod):
    N = 5
    nel, lo, hi = (3, 2, 4), (0.0, -1.0, 2.0), (1.5, 1.0, 3.0)
    m = oracle_mod.OracleMesh(N, nel, lo=lo, hi=hi)
    G, B = m.geom()
    h = [(hi[d] - lo[d]) / nel[d] for d in range(3)]
    _, w = gll_numpy(N)
    W = np.kron(w, np.kron(w, w))  # weight of node i + P j + P^2 k
    W = np.tile(W, m.E)
    hx, hy, hz = h
    np.testing.assert_allclose(G[0], W * hy * hz / (2 * hx), rtol=1e-12)
    np.testing.assert_allclose(G[1], W * hx * hz / (2 * hy), rtol=1e-12)
    np.testing.assert_allclose(G[2], W * hx * hy / (2 * hz), rtol=1e-12)
    assert np.max(np.abs(G[3:])) < 1e-13 * np.max(np.abs(G[0]))
    np.testing.assert_allclose(B, W * hx * hy * hz / 8, rtol=1e-12)


@pytest.mark.parametrize("N", [2, 3, 7])
def test_mass_sums_to_volume_jittered(oracle_mod, N):
    nel = (4, 3, 2)
    V = SI.jittered_box_vertices(nel, amp=0.05, seed=11)
    m = oracle_mod.OracleMesh(N, nel, vertices=V)
    _, B = m.geom()
    # trilinear elements: det J has degree <= 2 per variable, integrated exactly for N >= 2;
    # the jitter moves interior vertices only, so the box volume is unchanged
    assert abs(B.sum() - 1.0) < 1e-13


def test_coords_match_independent_map(oracle_mod):
    nel = (3, 2, 2)
    V = SI.jittered_box_vertices(nel, amp=0.05, seed=3)
    m = oracle_mod.OracleMesh(4, nel, vertices=V)
    x, y, z = m.coords()
    X = node_coords(4, nel, (0, 0, 0), (1, 1, 1), vertices=V)
    np.testing.assert_allclose(np.stack([x, y, z], 1), X, atol=1e-15)
    mp = oracle_mod.pipe_mesh(4, 4, 3, N=5)
    x, y, z = mp.coords()
    X = node_coords(5, (4, 4, 3), (-1, -1, 0), (1, 1, 10), pipe=True)
    np.testing.assert_allclose(np.stack([x, y, z], 1), X, atol=1e-15)


def _bruteforce_G(N, X, drop=None):
    """G factors from an independent numpy Jacobian (same definitions)."""
    xi, w = gll_numpy(N)
    P = N + 1
    Dm = lagrange_deriv(xi)
    I = np.eye(P)
    Dr, Ds, Dt = np.kron(I, np.kron(I, Dm)), np.kron(I, np.kron(Dm, I)), np.kron(Dm, np.kron(I, I))
    W = np.kron(w, np.kron(w, w))
    P3 = P ** 3
    out = []
    for e in range(X.shape[0] // P3):
        Xe = X[e * P3:(e + 1) * P3]
        J = np.stack([np.stack([Dr @ Xe[:, a], Ds @ Xe[:, a], Dt @ Xe[:, a]], -1) for a in range(3)], 1)
        det = np.linalg.det(J)
        Ji = np.linalg.inv(J)
        M = np.einsum("qax,qbx->qab", Ji, Ji) * (W * det)[:, None, None]
        g = np.stack([M[:, 0, 0], M[:, 1, 1], M[:, 2, 2], M[:, 0, 1], M[:, 0, 2], M[:, 1, 2]])
        out.append(g)
    return np.concatenate(out, axis=1)


def test_geom_against_bruteforce_jittered(oracle_mod):
    N, nel = 4, (2, 3, 2)
    V = SI.jittered_box_vertices(nel, amp=0.05, seed=5)
    m = oracle_mod.OracleMesh(N, nel, vertices=V)
    G, _ = m.geom()
    Gb = _bruteforce_G(N, node_coords(N, nel, (0, 0, 0), (1, 1, 1), vertices=V))
    np.testing.assert_allclose(G, Gb, rtol=0, atol=1e-13 * np.abs(Gb).max())


def _pipe_singular(N, nel):
    """Local nodes whose square coordinates are (+-1, +-1), from indices."""
    nx, ny, nz = nel
    P = N + 1
    out = np.zeros((nz, ny, nx, P, P, P), dtype=bool)  # [ez,ey,ex,k,j,i]
    for ey in range(ny):
        for ex in range(nx):
            for j in range(P):
                for i in range(P):
                    xe = (ex == 0 and i == 0) or (ex == nx - 1 and i == N)
                    ye = (ey == 0 and j == 0) or (ey == ny - 1 and j == N)
                    if xe and ye:
                        out[:, ey, ex, :, j, i] = True
    return out.reshape(-1)


def test_geom_against_bruteforce_pipe(oracle_mod):
    N, nel = 5, (4, 4, 2)
    m = oracle_mod.pipe_mesh(*nel, N=N)
    G, B = m.geom()
    X = node_coords(N, nel, (-1, -1, 0), (1, 1, 10), pipe=True)
    Gb = _bruteforce_G(N, X)
    sing = _pipe_singular(N, nel)
    assert sing.sum() == 4 * nel[2] * (N + 1)
    # singular nodes: the quadrature point is dropped
    assert np.all(G[:, sing] == 0) and np.all(B[sing] == 0)
    ok = ~sing
    np.testing.assert_allclose(G[:, ok], Gb[:, ok], rtol=1e-9, atol=1e-12 * np.abs(Gb[:, ok]).max())


def test_pipe_volume_converges(oracle_mod):
    # sum(B) -> area(pi) * length(10), spectrally in N: the isoparametric map
    # and the GLL quadrature of its Jacobian converge exponentially (the
    # dropped corner points have |J| = 0).  Measured 1.3e-6, 2.8e-9, 1.1e-11,
    # 6e-14 at N = 3, 5, 7, 9; a wrong weight or a dropped term would stall
    # at the 1e-3 level or above.
    bounds = {3: 1e-5, 5: 1e-7, 7: 1e-9, 9: 1e-12}
    errs = []
    for N, bound in bounds.items():
        m = oracle_mod.pipe_mesh(8, 8, 1, N=N)
        _, B = m.geom()
        err = abs(B.sum() - 10 * np.pi) / (10 * np.pi)
        assert err < bound, (N, err)
        errs.append(err)
    # each step of two orders gains at least two decades
    assert all(b < a * 1e-2 for a, b in zip(errs, errs[1:])), errs
