"""Pins of the overlapping Schwarz oracle (Eq. 6, sum over local subdomains).

* On an affine mesh of equal box elements the separable local matrix equals
  the restriction of the brute-force assembled stiffness to the extended
  element (this fixes the 1-D assembly, the overlap layer, the side handling
  and the Kronecker order) -- with at least three elements along periodic
  directions, where the two neighbours of an element are distinct.
* The preconditioner is symmetric positive definite.
* A single affine element with Dirichlet faces: the local solve is the exact
  inverse, so PCG converges in one iteration.
* It takes fewer iterations than Jacobi on a jittered box."""
import numpy as np
import pytest

import bruteforce as BF
import seeded_inputs as SI
from oracle.schwarz import SchwarzOracle, pcg


@pytest.mark.parametrize("N,nel,periodic", [(3, (3, 3, 2), (0, 0, 0)), (3, (3, 3, 3), (1, 0, 1)),
                                            (2, (3, 4, 3), (1, 1, 1))])
def test_local_matrix_is_restricted_stiffness_on_affine_boxes(oracle_mod, N, nel, periodic):
    m = oracle_mod.OracleMesh(N, nel, periodic=periodic)
    S = SchwarzOracle(m)
    X = BF.node_coords(N, nel, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    A, _ = BF.assemble(N, X, m.numbering())
    for e in range(m.E):
        Ak, ids = S.local_system(e)
        assert np.all(ids >= 0) and len(set(ids.tolist())) == len(ids)
        ref = A[np.ix_(ids, ids)]
        assert np.max(np.abs(Ak - ref)) <= 1e-13 * np.max(np.abs(ref)), e


def _continuous(m, seed):
    v = SI.uniform_global_values(m.nglob, seed)[m.numbering()]
    v[m.local_mask() == 1] = 0.0
    return v


def test_preconditioner_spd(oracle_mod):
    nel = (3, 2, 2)
    m = oracle_mod.OracleMesh(3, nel, vertices=SI.jittered_box_vertices(nel, seed=4))
    S = SchwarzOracle(m)
    x, y = _continuous(m, 1), _continuous(m, 2)
    Mx, My = S.apply(x), S.apply(y)
    assert abs(m.dot(x, My) - m.dot(y, Mx)) <= 1e-12 * abs(m.dot(x, My))
    assert m.dot(x, Mx) > 0 and m.dot(y, My) > 0
    # the output is continuous and masked
    assert np.all(Mx[m.local_mask() == 1] == 0.0)
    g = m.numbering()
    first = np.zeros(m.nglob)
    first[g] = Mx
    assert np.array_equal(first[g], Mx)


def test_single_affine_element_is_exact(oracle_mod):
    m = oracle_mod.OracleMesh(5, (1, 1, 1))
    S = SchwarzOracle(m)
    x, y, z = m.coords()
    b = m.mass(SI.sin3_forcing(x, y, z))
    xs, its = pcg(m, b, S.apply, tol=1e-12)
    assert its == 1
    assert m.true_residual(b, xs) <= 1e-12


def test_fewer_iterations_than_jacobi(oracle_mod):
    nel = (3, 3, 3)
    m = oracle_mod.OracleMesh(5, nel, vertices=SI.jittered_box_vertices(nel, seed=1))
    x, y, z = m.coords()
    b = m.mass(SI.sin3_forcing(x, y, z))
    _, rj = m.pcg(b, tol=1e-10)
    xs, its = pcg(m, b, SchwarzOracle(m).apply, tol=1e-10)
    assert m.true_residual(b, xs) <= 1e-10
    assert its < 0.6 * rj.iterations, (its, rj.iterations)


def test_element_lengths_on_a_distorted_element(oracle_mod):
    """The local problem's length per direction is the mean of the four
    straight edges of the element along that direction.  On one trilinear
    element with hand-placed vertices whose four edges differ in every
    direction, the oracle's lengths equal the means computed here directly
    from the vertex coordinates (so averaging two edges, mixing directions or
    measuring along the curve would all fail)."""
    V = np.array([[0.00, 0.00, 0.00], [1.00, 0.05, 0.00], [0.10, 1.20, 0.05], [1.30, 1.10, 0.10],
                  [0.05, 0.10, 0.90], [0.90, 0.20, 1.00], [0.00, 1.00, 1.10], [1.20, 1.05, 1.30]])
    m = oracle_mod.OracleMesh(3, (1, 1, 1), vertices=V.reshape(-1))
    S = SchwarzOracle(m)
    d = lambda a, b: float(np.linalg.norm(V[a] - V[b]))
    edges = {
        "r": [(0, 1), (2, 3), (4, 5), (6, 7)],
        "s": [(0, 2), (1, 3), (4, 6), (5, 7)],
        "t": [(0, 4), (1, 5), (2, 6), (3, 7)],
    }
    want = [np.mean([d(a, b) for a, b in edges[x]]) for x in "rst"]
    for x in "rst":
        lens = [d(a, b) for a, b in edges[x]]
        assert max(lens) - min(lens) > 0.05, x  # the four edges really differ
    got = S.lengths(0)
    assert np.allclose(got, want, rtol=1e-14, atol=0.0), (got, want)


def test_element_lengths_on_jittered_elements(oracle_mod):
    """The same rule on every element of a jittered 3x2x2 box, from the
    vertex array passed to the mesh."""
    nel = (3, 2, 2)
    V = SI.jittered_box_vertices(nel, seed=8)
    m = oracle_mod.OracleMesh(3, nel, vertices=V)
    S = SchwarzOracle(m)
    VV = np.asarray(V).reshape(nel[2] + 1, nel[1] + 1, nel[0] + 1, 3)
    for e in range(m.E):
        ex, ey, ez = e % nel[0], (e // nel[0]) % nel[1], e // (nel[0] * nel[1])
        c = lambda dx, dy, dz: VV[ez + dz, ey + dy, ex + dx]
        lr = np.mean([np.linalg.norm(c(1, y, z) - c(0, y, z)) for y in (0, 1) for z in (0, 1)])
        ls = np.mean([np.linalg.norm(c(x, 1, z) - c(x, 0, z)) for x in (0, 1) for z in (0, 1)])
        lt = np.mean([np.linalg.norm(c(x, y, 1) - c(x, y, 0)) for x in (0, 1) for y in (0, 1)])
        assert np.allclose(S.lengths(e), (lr, ls, lt), rtol=1e-13, atol=0.0), e
