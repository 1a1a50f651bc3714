"""Pins of the projection oracle (projection onto previous solutions, the
acceleration section 2 of the paper applies to successive solves).

Checked against what the method fixes: the basis is A-orthonormal; a right-hand
side whose solution lies in the span is solved exactly by the projection; the
projected residual is A-orthogonal... i.e. orthogonal to the span; the
projection equals the brute-force normal-equations solution over the raw
vectors; dependent vectors are dropped; a full basis restarts."""
import numpy as np
import pytest

import seeded_inputs as SI
from oracle.projection import ProjectionSpace


@pytest.fixture(scope="module")
def mesh(oracle_mod):
    nel = (3, 2, 2)
    return oracle_mod.OracleMesh(5, nel, vertices=SI.jittered_box_vertices(nel, seed=3))


def _continuous(m, seed):
    """A continuous, masked E-vector (one value per global node)."""
    v = SI.uniform_global_values(m.nglob, seed)[m.numbering()]
    v[m.local_mask() == 1] = 0.0
    return v


def _Adot(m, a, b):
    return m.dot(a, m.apply(b))


def test_basis_is_A_orthonormal(mesh):
    ps = ProjectionSpace(mesh, 6)
    for s in range(5):
        assert ps.add(_continuous(mesh, 10 + s))
    G = np.array([[_Adot(mesh, xi, xj) for xj in ps.X] for xi in ps.X])
    assert np.max(np.abs(G - np.eye(len(ps)))) <= 1e-12
    # the stored A x_i are A applied to the basis vectors
    for xi, axi in zip(ps.X, ps.AX):
        ref = mesh.apply(xi)
        assert np.linalg.norm(axi - ref) <= 1e-12 * np.linalg.norm(ref)


def test_projection_exact_on_span(mesh):
    ps = ProjectionSpace(mesh, 6)
    vs = [_continuous(mesh, 20 + s) for s in range(4)]
    for v in vs:
        ps.add(v)
    c = np.array([0.7, -1.3, 0.25, 2.0])
    x = sum(ci * vi for ci, vi in zip(c, vs))
    b = mesh.apply(x)
    xbar = ps.project(b)
    assert np.linalg.norm(xbar - x) <= 1e-10 * np.linalg.norm(x)
    # the solve then needs no iteration
    ps2 = ProjectionSpace(mesh, 6)
    for v in vs:
        ps2.add(v)
    xs, res = ps2.solve(b, tol=1e-10)
    assert res.iterations == 0 and np.linalg.norm(xs - x) <= 1e-10 * np.linalg.norm(x)


def test_residual_orthogonal_to_span_and_brute_force(mesh):
    vs = [_continuous(mesh, 30 + s) for s in range(4)]
    ps = ProjectionSpace(mesh, 8)
    for v in vs:
        ps.add(v)
    x, y, z = mesh.coords()
    b = mesh.mass(SI.sin3_forcing(x, y, z))
    xbar = ps.project(b)
    r = b - mesh.apply(xbar)
    bn = np.sqrt(mesh.dot(b, b))
    for v in vs:
        assert abs(mesh.dot(v, r)) <= 1e-12 * bn * np.sqrt(mesh.dot(v, v))
    # brute force: Galerkin over the raw vectors, G c = V^T b with G = V^T A V
    G = np.array([[_Adot(mesh, vi, vj) for vj in vs] for vi in vs])
    rhs = np.array([mesh.dot(vi, b) for vi in vs])
    c = np.linalg.solve(G, rhs)
    xbf = sum(ci * vi for ci, vi in zip(c, vs))
    assert np.linalg.norm(xbar - xbf) <= 1e-9 * np.linalg.norm(xbf)


def test_dependent_vector_dropped_and_restart(mesh):
    ps = ProjectionSpace(mesh, 3)
    v1, v2 = _continuous(mesh, 40), _continuous(mesh, 41)
    assert ps.add(v1) and ps.add(v2)
    assert not ps.add(2.0 * v1 - 0.5 * v2)
    assert len(ps) == 2
    v3, v4 = _continuous(mesh, 42), _continuous(mesh, 43)
    assert ps.add(v3) and len(ps) == 3
    # full: the next vector restarts the basis from itself, A-normalised
    assert ps.add(v4) and len(ps) == 1
    x0 = ps.X[0]
    nv4 = np.sqrt(_Adot(mesh, v4, v4))
    assert np.linalg.norm(x0 - v4 / nv4) <= 1e-13 * np.linalg.norm(x0)
    assert abs(_Adot(mesh, x0, x0) - 1.0) <= 1e-13


def test_successive_solves_need_fewer_iterations(mesh):
    x, y, z = mesh.coords()
    ps = ProjectionSpace(mesh, 8)
    plain, proj = [], []
    for t in range(6):
        b = mesh.mass(SI.travelling_forcing(x, y, z, float(t)))
        _, r0 = mesh.pcg(b, tol=1e-10)
        xs, r1 = ps.solve(b, tol=1e-10)
        assert mesh.true_residual(b, xs) <= 1e-10
        plain.append(r0.iterations)
        proj.append(r1.iterations)
    assert proj[0] == plain[0]
    assert all(p < q for p, q in zip(proj[2:], plain[2:])), (proj, plain)
