"""Pins of the two-level (Jacobi + coarse term of Eq. 6) oracle.

* The hat functions form a partition of unity on the unmasked nodes.
* On an affine box the coarse prolongation equals trilinear interpolation of
  the vertex values at the physical node coordinates (an independent
  construction), and A_0 equals P^T A P with A from the brute-force dense
  assembly.
* The Chebyshev step equals the closed-form polynomial evaluated through an
  eigendecomposition.
* The preconditioner is symmetric positive definite and cuts PCG iterations
  below Jacobi's."""
import numpy as np
import pytest

import bruteforce as BF
import seeded_inputs as SI
from oracle.coarse import CoarseOracle
from oracle.schwarz import pcg


@pytest.fixture(scope="module")
def affine(oracle_mod):
    return oracle_mod.OracleMesh(3, (3, 2, 2))


def test_partition_of_unity(oracle_mod):
    nel = (3, 2, 2)
    m = oracle_mod.OracleMesh(3, nel, vertices=SI.jittered_box_vertices(nel, seed=2), periodic=(0, 0, 1))
    C = CoarseOracle(m)
    s = C.prolong(np.ones(C.nvert))
    live = m.local_mask() == 0
    assert np.allclose(s[live], 1.0, atol=1e-14) and np.all(s[~live] == 0.0)


def test_affine_box_against_brute_force(affine):
    m = affine
    C = CoarseOracle(m)
    nx, ny, nz = m.nel
    X = BF.node_coords(m.N, m.nel, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    gid = m.numbering()
    # trilinear interpolation of each vertex's indicator at the physical coordinates
    vx, vy, vz = C.vdims
    xg = np.zeros((m.nglob, 3))
    xg[gid] = X
    hx = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
    live = m.global_mask() == 0
    for v in range(C.nvert):
        a, b, c = v % vx, (v // vx) % vy, v // (vx * vy)
        hat = np.prod([np.clip(1.0 - np.abs(xg[:, d] / hx[d] - idx), 0.0, None)
                       for d, idx in enumerate((a, b, c))], axis=0)
        col = C.P[:, v].toarray().ravel()
        assert np.max(np.abs(col - hat * live)) <= 1e-13, v
    A, _ = BF.assemble(m.N, X, gid)
    A = A * np.outer(live, live)
    Pd = C.P.toarray()
    A0 = Pd.T @ A @ Pd
    assert np.max(np.abs(C.A0 - A0)) <= 1e-12 * np.max(np.abs(A0))
    assert np.max(np.abs(C.A0 - C.A0.T)) <= 1e-12 * np.max(np.abs(A0))


def test_chebyshev_closed_form(affine):
    C = CoarseOracle(affine, k=7, frac=0.05)
    A, D = C.A0k, C.D0
    S = A / np.sqrt(np.outer(D, D))
    lam, V = np.linalg.eigh(S)
    theta, delta = (C.b + C.a) / 2, (C.b - C.a) / 2
    x0 = theta / delta
    # residual polynomial r_k(l) = T_k((theta - l)/delta) / T_k(theta/delta); z = (1 - r_k(l))/l applied
    T = lambda x: np.polynomial.chebyshev.chebval(x, [0] * C.k + [1])
    p = (1.0 - T((theta - lam) / delta) / T(x0)) / lam
    r0 = SI.random_local(len(D), 4)
    ref = (V @ (p * (V.T @ (r0 / np.sqrt(D))))) / np.sqrt(D)
    got = C.chebyshev(r0)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_spd_and_fewer_iterations(oracle_mod):
    nel = (4, 4, 4)
    m = oracle_mod.OracleMesh(5, nel, vertices=SI.jittered_box_vertices(nel, seed=1))
    C = CoarseOracle(m)
    g = m.numbering()
    x = SI.uniform_global_values(m.nglob, 1)[g]
    y = SI.uniform_global_values(m.nglob, 2)[g]
    x[m.local_mask() == 1] = 0.0
    y[m.local_mask() == 1] = 0.0
    Mx, My = C.apply(x), C.apply(y)
    assert abs(m.dot(x, My) - m.dot(y, Mx)) <= 1e-12 * abs(m.dot(x, My))
    assert m.dot(x, Mx) > 0
    xs_, ys_, zs_ = m.coords()
    b = m.mass(SI.sin3_forcing(xs_, ys_, zs_))
    _, rj = m.pcg(b, tol=1e-10)
    xs, its = pcg(m, b, C.apply, tol=1e-10)
    assert m.true_residual(b, xs) <= 1e-10
    assert its < 0.8 * rj.iterations, (its, rj.iterations)
