"""Pins of the oracle's local operator (Algorithm 1), gather-scatter, numbering
and Jacobi diagonal (CPU only).

The matrix-free operator is a faster way to apply the assembled stiffness
matrix (paper section 2: global face exchange plus local matrix-free work), so
it is pinned against an independent dense assembly, exact-integration special
cases and invariants.
"""
import numpy as np
import pytest

import seeded_inputs as SI
from bruteforce import assemble, element_stiffness, node_coords, number_by_coords


def _tiny_cases(oracle_mod):
    cases = []
    nel = (2, 2, 2)
    V = SI.jittered_box_vertices(nel, amp=0.05, seed=21)
    cases.append(("jitter_N3", oracle_mod.OracleMesh(3, nel, vertices=V),
                  node_coords(3, nel, (0, 0, 0), (1, 1, 1), vertices=V), None))
    nel = (2, 1, 2)
    V = SI.jittered_box_vertices(nel, lo=(0, 0, 0), hi=(2, 1, 1), amp=0.05, seed=22)
    cases.append(("jitter_N4", oracle_mod.OracleMesh(4, nel, hi=(2, 1, 1), vertices=V),
                  node_coords(4, nel, (0, 0, 0), (2, 1, 1), vertices=V), None))
    nel = (3, 3, 2)
    cases.append(("pipe_N3", oracle_mod.pipe_mesh(*nel, N=3),
                  node_coords(3, nel, (-1, -1, 0), (1, 1, 10), pipe=True), 10.0))
    return cases


def _continuous(m, seed):
    v = SI.random_local(m.nglob, seed)
    return v[m.numbering()]


def test_numbering_matches_coordinate_matching(oracle_mod):
    for name, m, X, period in _tiny_cases(oracle_mod):
        gid = m.numbering()
        gb = number_by_coords(X, period=period)
        # same partition of local nodes into global nodes
        pairs = np.unique(np.stack([gid, gb], 1), axis=0)
        assert len(pairs) == len(np.unique(gid)) == len(np.unique(gb)) == m.nglob, name


def test_element_operator_against_dense(oracle_mod):
    """A_L u element by element equals the dense element stiffness times u_e."""
    for name, m, X, _ in _tiny_cases(oracle_mod):
        P3 = m.P ** 3
        u = SI.random_local(m.nloc, 5)
        w = m.ax(u)
        G, B = m.geom()
        drop = (B == 0)
        for e in range(m.E):
            sl = slice(e * P3, (e + 1) * P3)
            Ae, _ = element_stiffness(m.N, X[sl], drop[sl])
            ref = Ae @ u[sl]
            err = np.max(np.abs(w[sl] - ref)) / np.max(np.abs(ref))
            assert err < 1e-12, (name, e, err)


def test_assembled_operator_against_dense(oracle_mod):
    """mask(Q Q^T A_L Q u_G) equals Q mask(A_G u_G) with A_G densely assembled."""
    for name, m, X, _ in _tiny_cases(oracle_mod):
        gid = m.numbering()
        _, B = m.geom()
        A, _ = assemble(m.N, X, gid, drop=(B == 0))
        uG = SI.random_local(m.nglob, 7)
        ref = A @ uG
        ref[m.global_mask() == 1] = 0.0
        got = m.apply(uG[gid])
        err = np.max(np.abs(got - ref[gid])) / np.max(np.abs(ref))
        assert err < 1e-12, (name, err)


def test_symmetry_and_neumann_nullspace(oracle_mod):
    for name, m, X, _ in _tiny_cases(oracle_mod):
        u, v = _continuous(m, 1), _continuous(m, 2)
        mk = m.local_mask() == 1
        u[mk] = 0
        v[mk] = 0
        a = m.dot(v, m.apply(u))
        b = m.dot(u, m.apply(v))
        assert abs(a - b) < 1e-12 * max(abs(a), 1.0), name
        # constants are in the null space of the unmasked (Neumann) operator
        one = np.ones(m.nloc)
        assert np.max(np.abs(m.apply(one, masked=False))) < 1e-12, name


@pytest.mark.parametrize("N", [2, 3, 5, 7])
def test_linear_functions_harmonic(oracle_mod, N):
    """A(c.x) = 0 at every non-wall node: the quadrature is exact for it on
    affine and trilinear elements."""
    nel = (3, 2, 2)
    V = SI.jittered_box_vertices(nel, amp=0.05, seed=31)
    for m in (oracle_mod.OracleMesh(N, nel), oracle_mod.OracleMesh(N, nel, vertices=V)):
        x, y, z = m.coords()
        u = 0.3 * x - 1.1 * y + 0.7 * z + 2.0
        w = m.apply(u)
        assert np.max(np.abs(w)) < 1e-12


@pytest.mark.parametrize("N,jitter", [(2, False), (4, False), (3, True), (5, True), (7, True)])
def test_quadratic_gives_minus_six_mass(oracle_mod, N, jitter):
    """A(x^2+y^2+z^2) = -6 Q Q^T B at non-wall nodes (weak Laplacian of a
    quadratic, integrated exactly: N >= 2 affine, N >= 3 trilinear)."""
    nel = (2, 3, 2)
    V = SI.jittered_box_vertices(nel, amp=0.05, seed=41) if jitter else None
    m = oracle_mod.OracleMesh(N, nel, vertices=V)
    x, y, z = m.coords()
    _, B = m.geom()
    w = m.apply(x * x + y * y + z * z)
    ref = -6.0 * m.gs(B)
    assert np.max(np.abs(w - ref)) < 1e-12 * np.max(np.abs(ref))


def test_gs_invariants(oracle_mod):
    for name, m, X, _ in _tiny_cases(oracle_mod):
        mult = m.local_mult()
        np.testing.assert_array_equal(m.gs(np.ones(m.nloc), masked=False), mult)
        assert abs(np.sum(1.0 / mult) - m.nglob) < 1e-9
        a, b = SI.random_local(m.nloc, 3), SI.random_local(m.nloc, 4)
        # Q Q^T is symmetric; so is mask * Q Q^T * mask
        assert abs(a @ m.gs(b) - m.gs(a) @ b) < 1e-12 * m.nloc
        # idempotent up to multiplicity: gs(gs(a)) = mult * gs(a)
        np.testing.assert_allclose(m.gs(m.gs(a, masked=False), masked=False),
                                   mult * m.gs(a, masked=False), rtol=1e-14, atol=1e-13)


def _mult_1d(n_el, N, periodic):
    ext = n_el * N + (0 if periodic else 1)
    mlt = np.ones(ext, dtype=np.int64)
    for a in range(ext):
        if a % N == 0:
            if periodic or (0 < a < ext - 1):
                mlt[a] = 2
    if periodic and n_el == 1:
        mlt[0] = 2
    return mlt


def _hist_closed_form(nel, N, periodic):
    """Multiplicity histogram over global nodes: product of 1-D multiplicities."""
    m1 = [_mult_1d(nel[d], N, periodic[d]) for d in range(3)]
    prod = np.multiply.outer(np.multiply.outer(m1[2], m1[1]), m1[0]).reshape(-1)
    return {k: int(np.sum(prod == k)) for k in (1, 2, 4, 8)}


@pytest.mark.parametrize("case", [
    ((4, 4, 4), 7, (0, 0, 0)),
    ((3, 2, 5), 5, (0, 0, 1)),
    ((2, 2, 2), 4, (1, 1, 1)),
])
def test_multiplicity_histogram_small(oracle_mod, case):
    nel, N, per = case
    m = oracle_mod.OracleMesh(N, nel, periodic=per)
    gm = m.global_mult()
    got = {k: int(np.sum(gm == k)) for k in (1, 2, 4, 8)}
    assert got == _hist_closed_form(nel, N, per)
    assert gm.sum() == m.nloc


def test_multiplicity_histogram_box_config():
    # the 4x4x4, N=7 box: 29^3 global nodes
    assert _hist_closed_form((4, 4, 4), 7, (0, 0, 0)) == {1: 17576, 2: 6084, 4: 702, 8: 27}


@pytest.mark.slow
@pytest.mark.parametrize("nel,N,hist", [
    ((48, 48, 96), 7, {1: 48441600, 2: 23775360, 4: 3889344, 8: 212064}),
    ((48, 48, 48), 9, {1: 57214464, 2: 21084864, 4: 2589888, 8: 106032}),
])
def test_multiplicity_histogram_pipe(oracle_mod, nel, N, hist):
    """Full-size pipe numbering: histogram equals the closed form."""
    assert _hist_closed_form(nel, N, (0, 0, 1)) == hist
    m = oracle_mod.pipe_mesh(*nel, N=N)
    gm = m.global_mult()
    got = {k: int(np.sum(gm == k)) for k in (1, 2, 4, 8)}
    assert got == hist


def test_jacobi_against_dense_diagonal(oracle_mod):
    for name, m, X, _ in _tiny_cases(oracle_mod):
        gid = m.numbering()
        _, B = m.geom()
        A, _ = assemble(m.N, X, gid, drop=(B == 0))
        inv = m.jacobi()
        ref = 1.0 / np.diag(A)
        ref[m.global_mask() == 1] = 0.0
        np.testing.assert_allclose(inv, ref[gid], rtol=1e-12, atol=0)


def test_helmholtz_against_dense(oracle_mod):
    """Helmholtz form h1 (grad, grad) + h2 (B .): per-point h1 weights the
    stiffness quadrature, h2 B adds the lumped mass."""
    name, m, X, _ = _tiny_cases(oracle_mod)[0]
    P3 = m.P ** 3
    rng = np.random.default_rng(9)
    h1 = rng.uniform(0.5, 2.0, m.nloc)
    h2 = rng.uniform(0.0, 3.0, m.nloc)
    u = SI.random_local(m.nloc, 10)
    w = m.ax(u, h1=h1, h2=h2)
    _, B = m.geom()
    from bruteforce import gll_numpy, lagrange_deriv
    xi, wq = gll_numpy(m.N)
    Dm = lagrange_deriv(xi)
    I = np.eye(m.P)
    ref_ops = [np.kron(I, np.kron(I, Dm)), np.kron(I, np.kron(Dm, I)), np.kron(Dm, np.kron(I, I))]
    W = np.kron(wq, np.kron(wq, wq))
    for e in range(m.E):
        sl = slice(e * P3, (e + 1) * P3)
        Xe = X[sl]
        J = np.stack([np.stack([R @ Xe[:, a] for R in ref_ops], -1) for a in range(3)], 1)
        Ji = np.linalg.inv(J)
        wdet = W * np.linalg.det(J) * h1[sl]
        Ae = np.zeros((P3, P3))
        for d in range(3):
            Gd = sum(Ji[:, b, d][:, None] * ref_ops[b] for b in range(3))
            Ae += Gd.T @ (wdet[:, None] * Gd)
        ref = Ae @ u[sl] + h2[sl] * B[sl] * u[sl]
        assert np.max(np.abs(w[sl] - ref)) < 1e-12 * np.max(np.abs(ref))
    # Jacobi diagonal of the Helmholtz form
    inv = m.jacobi(h1=h1, h2=h2)
    diag = np.zeros(m.nloc)
    for e in range(m.E):
        sl = slice(e * P3, (e + 1) * P3)
        Xe = X[sl]
        J = np.stack([np.stack([R @ Xe[:, a] for R in ref_ops], -1) for a in range(3)], 1)
        Ji = np.linalg.inv(J)
        wdet = W * np.linalg.det(J) * h1[sl]
        for d in range(3):
            Gd = sum(Ji[:, b, d][:, None] * ref_ops[b] for b in range(3))
            diag[sl] += np.einsum("qa,q,qa->a", Gd, wdet, Gd)
        diag[sl] += h2[sl] * B[sl]
    ref = m.gs(diag)
    mk = m.local_mask() == 1
    np.testing.assert_allclose(inv[~mk], 1.0 / ref[~mk], rtol=1e-12)
    assert np.all(inv[mk] == 0)
