"""Pins of the oracle's Jacobi-PCG and of the discretisation (CPU only).

The pressure Poisson solve (paper section 2, Eq. 5) is done by a
preconditioned Krylov iteration; here Jacobi-PCG on the GLL Laplacian with
homogeneous Dirichlet walls.  Several x are correct (any with a true relative
residual <= 1e-10), so the pins are a dense direct solve, a closed loop
b = A v, and the true residual.
"""
import numpy as np
import pytest

import seeded_inputs as SI
from bruteforce import assemble, node_coords


def test_pcg_matches_dense_solve(oracle_mod):
    nel = (2, 2, 2)
    V = SI.jittered_box_vertices(nel, amp=0.05, seed=51)
    m = oracle_mod.OracleMesh(4, nel, vertices=V)
    X = node_coords(4, nel, (0, 0, 0), (1, 1, 1), vertices=V)
    gid = m.numbering()
    A, _ = assemble(4, X, gid)
    free = m.global_mask() == 0
    bG = SI.random_local(m.nglob, 52)
    bG[~free] = 0
    xG = np.zeros(m.nglob)
    xG[free] = np.linalg.solve(A[np.ix_(free, free)], bG[free])
    x, res = oracle_mod.OracleMesh.pcg(m, bG[gid], tol=1e-12, max_iter=2000)
    assert res.status == 0
    kappa = np.linalg.cond(A[np.ix_(free, free)])
    err = np.linalg.norm(x - xG[gid]) / np.linalg.norm(xG[gid])
    assert err < kappa * 1e-12


@pytest.mark.parametrize("mesh", ["box", "pipe"])
def test_pcg_closed_loop(oracle_mod, mesh):
    if mesh == "box":
        nel = (3, 3, 3)
        m = oracle_mod.OracleMesh(5, nel, vertices=SI.jittered_box_vertices(nel, seed=61))
    else:
        m = oracle_mod.pipe_mesh(4, 4, 3, N=5)
    v = SI.random_local(m.nglob, 62)[m.numbering()]
    v[m.local_mask() == 1] = 0
    b = m.apply(v)
    x, res = m.pcg(b, tol=1e-10, max_iter=5000)
    assert res.status == 0
    assert m.true_residual(b, x) <= 1e-10
    # ||x - v|| / ||v|| <= kappa * 1e-10; kappa of these small meshes < 1e4
    assert np.linalg.norm(x - v) / np.linalg.norm(v) < 1e-6


def test_pcg_box_config_converges(oracle_mod):
    """4x4x4 jittered box, N=7, sin^3 forcing: reaches a true 1e-10 residual."""
    nel = (4, 4, 4)
    m = oracle_mod.OracleMesh(7, nel, vertices=SI.jittered_box_vertices(nel, seed=1))
    x, y, z = m.coords()
    b = m.mass(SI.sin3_forcing(x, y, z))
    u, res = m.pcg(b, tol=1e-10, max_iter=5000)
    assert res.status == 0 and res.rel_residual <= 1e-10
    assert m.true_residual(b, u) <= 1e-10
    assert np.max(np.abs(u - SI.sin3(x, y, z))) < 1e-6


def test_pcg_status_codes(oracle_mod):
    m = oracle_mod.OracleMesh(3, (2, 2, 2))
    x, y, z = m.coords()
    b = m.mass(SI.sin3_forcing(x, y, z))
    _, res = m.pcg(b, tol=1e-10, max_iter=1)
    assert res.status == 1 and res.iterations == 1
    # zero right-hand side: x = 0 is already converged
    _, res = m.pcg(np.zeros(m.nloc), tol=1e-10, max_iter=10)
    assert res.status == 0 and res.iterations == 0


def test_spectral_convergence(oracle_mod):
    """Manufactured sin^3 on the jittered 4^3 box: the nodal error falls
    exponentially with N (values unpinned: the paper prints none)."""
    nel = (4, 4, 4)
    V = SI.jittered_box_vertices(nel, seed=1)
    errs = {}
    for N in range(2, 11):
        m = oracle_mod.OracleMesh(N, nel, vertices=V)
        x, y, z = m.coords()
        b = m.mass(SI.sin3_forcing(x, y, z))
        u, res = m.pcg(b, tol=1e-13, max_iter=5000)
        errs[N] = np.max(np.abs(u - SI.sin3(x, y, z)))
    for N in range(2, 9):
        assert errs[N + 2] < errs[N] / 10, errs
    assert errs[10] < 1e-8
    # exponential rather than algebraic: the log-error falls faster than linearly in log N
    slope_lo = np.log(errs[4] / errs[2]) / np.log(4 / 2)
    slope_hi = np.log(errs[10] / errs[8]) / np.log(10 / 8)
    assert slope_hi < slope_lo
