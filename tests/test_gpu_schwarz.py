"""Overlapping Schwarz local solves of Eq. 6 on the GPU (fast
diagonalisation on each element extended by one node layer) against the
oracle (oracle/schwarz.py, pinned in test_oracle_schwarz.py): M^-1 r element
by element, alone and with the coarse term, and whole CG runs (iterations,
fixed-step iterates, true residual), on boxes with Dirichlet, free and
periodic faces and on the pipe."""
import numpy as np
import pytest
import torch

import seeded_inputs as SI
from oracle.coarse import CoarseOracle
from oracle.schwarz import SchwarzOracle, pcg

pytestmark = pytest.mark.gpu

K, FRAC = 4, 0.05


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b), np.max(np.abs(a - b)) / np.max(np.abs(b))


class _Op:
    def __init__(self, om, h1=None, h2=None):
        self.om, self.h1, self.h2 = om, h1, h2
        self.nloc = om.nloc

    def apply(self, x):
        return self.om.apply(x, self.h1, self.h2)

    def dot(self, a, b):
        return self.om.dot(a, b)


def _meshes(semlib, oracle_mod, kind, N, nel, periodic, seed, dirichlet=None):
    if kind == "pipe":
        return (semlib.pipe_mesh(*nel, N=N, length=2.0, with_fp32=True),
                oracle_mod.pipe_mesh(*nel, N=N, length=2.0))
    V = SI.jittered_box_vertices(nel, seed=seed)
    kw = {} if dirichlet is None else {"dirichlet_faces": dirichlet}
    return (semlib.box_mesh(N, nel, vertices=V, periodic=periodic, with_fp32=True, **kw),
            oracle_mod.OracleMesh(N, nel, vertices=V, periodic=periodic, dirichlet=dirichlet))


def _continuous(om, seed):
    g = SI.uniform_global_values(om.nglob, seed=seed)
    return g[om.numbering()] * (om.local_mask() == 0)


# the local solves invert matrices whose condition grows like N^4 / h^2; the
# FDM and the oracle's Cholesky agree to a few thousand ulps
TOL = 1e-11

CASES = [
    ("box", 3, (3, 3, 3), (0, 0, 0), 1, None),
    ("box", 5, (3, 3, 4), (0, 0, 1), 2, None),
    ("box", 4, (3, 4, 3), (1, 0, 1), 3, None),
    ("box", 2, (4, 3, 3), (0, 0, 0), 4, None),
    ("box", 2, (3, 3, 3), (1, 1, 1), 5, None),  # fully periodic: every subdomain has all neighbours
    ("box", 5, (3, 3, 3), (0, 0, 0), 6, 0b000110),  # Dirichlet on x-high and y-low only, free elsewhere
    ("pipe", 7, (4, 4, 3), None, 7, None),
    ("box", 9, (3, 2, 2), (0, 0, 0), 8, None),
]


@pytest.mark.parametrize("kind,N,nel,periodic,seed,dirichlet", CASES)
def test_schwarz_apply(semlib, oracle_mod, kind, N, nel, periodic, seed, dirichlet):
    print(f"case: schwarz apply {kind} N={N} nel={nel} periodic={periodic} dirichlet={dirichlet}", flush=True)
    m, om = _meshes(semlib, oracle_mod, kind, N, nel, periodic, seed, dirichlet)
    S = SchwarzOracle(om)
    m.set_schwarz(True)
    info = m.schwarz_info()
    assert info["enabled"] and 1 <= info["n_factors"] <= 3 * om.E
    live = om.local_mask() == 0
    for s in range(2):
        r = _continuous(om, 100 * seed + s)
        z = _host(m.precond(_dev(r)))
        ref = S.apply(r)
        e2, einf = _relerr(z, ref)
        assert e2 <= TOL and einf <= TOL, (s, e2, einf)
        assert np.all(z[~live] == 0.0)
        # every copy of a shared node holds the same bits
        zg = np.zeros(om.nglob)
        zg[om.numbering()] = z
        assert np.array_equal(zg[om.numbering()], z)
    # with the coarse term: M^-1 r = Schwarz(r) + P C(A0) P^T r
    m.set_coarse(K, FRAC)
    C = CoarseOracle(om, k=K, frac=FRAC)
    r = _continuous(om, 100 * seed + 7)
    e2, einf = _relerr(_host(m.precond(_dev(r))), S.apply(r) + C.coarse(r))
    assert e2 <= TOL and einf <= TOL, (e2, einf)
    # removing it restores Jacobi (+ coarse)
    m.set_schwarz(False)
    assert not m.schwarz_info()["enabled"]
    e2, _ = _relerr(_host(m.precond(_dev(r))), C.apply(r))
    assert e2 <= 1e-12
    m.close()


PCG_CASES = [
    ("box", 5, (3, 3, 3), (0, 0, 0), 21, None),
    ("pipe", 5, (6, 6, 5), None, 22, None),
    ("box", 4, (3, 3, 4), (0, 0, 1), 23, 0b000101),
]


@pytest.mark.parametrize("coarse", [False, True])
@pytest.mark.parametrize("kind,N,nel,periodic,seed,dirichlet", PCG_CASES)
def test_schwarz_pcg(semlib, oracle_mod, kind, N, nel, periodic, seed, dirichlet, coarse):
    print(f"case: schwarz pcg {kind} N={N} nel={nel} coarse={coarse}", flush=True)
    m, om = _meshes(semlib, oracle_mod, kind, N, nel, periodic, seed, dirichlet)
    x, y, z = om.coords()
    b = om.mass(SI.sin3_forcing(x, y, z))
    S = SchwarzOracle(om)
    if coarse:
        C = CoarseOracle(om, k=K, frac=FRAC)
        M = lambda r: S.apply(r) + C.coarse(r)  # noqa: E731
        m.set_coarse(K, FRAC)
    else:
        M = S.apply
    m.set_schwarz(True)
    _, it_o = pcg(_Op(om), b, M, tol=1e-10)
    _, rj = om.pcg(b, tol=1e-10)
    assert it_o < rj.iterations
    for graph, poll in ((True, 16), (False, 5)):
        xg, res = m.solve(_dev(b), tol=1e-10, use_graph=graph, poll_every=poll)
        assert res.ok, res
        assert abs(res.iterations - it_o) <= max(3, 0.05 * it_o), (graph, res.iterations, it_o)
        assert om.true_residual(b, _host(xg)) <= 1e-10
    for steps in (1, 5):
        xs, _ = pcg(_Op(om), b, M, tol=1e-30, max_iter=steps)
        xg, res = m.solve(_dev(b), fixed_iters=steps)
        assert res.iterations == steps
        e2, einf = _relerr(_host(xg), xs)
        assert e2 <= 1e-9 and einf <= 1e-9, (steps, e2, einf)
    m.close()


def test_schwarz_helmholtz_pcg(semlib, oracle_mod):
    """Helmholtz operator, Poisson-form local solves (plus the coarse term of
    the Helmholtz operator): CG against the oracle with the same M."""
    print("case: schwarz helmholtz pcg box 3x3x3 N=5", flush=True)
    m, om = _meshes(semlib, oracle_mod, "box", 5, (3, 3, 3), (0, 0, 0), 31)
    h1 = SI.uniform_local(om.nloc, 32, 0.5, 2.0)
    h2 = SI.uniform_local(om.nloc, 33, 0.0, 3.0)
    m.set_helmholtz(_dev(h1), _dev(h2))
    m.set_schwarz(True)
    m.set_coarse(K, FRAC)
    S = SchwarzOracle(om)
    C = CoarseOracle(om, k=K, frac=FRAC, h1=h1, h2=h2)
    x, y, z = om.coords()
    b = om.mass(SI.sin3_forcing(x, y, z))
    _, it_o = pcg(_Op(om, h1, h2), b, lambda r: S.apply(r) + C.coarse(r), tol=1e-10)
    xg, res = m.solve(_dev(b), tol=1e-10)
    assert res.ok and abs(res.iterations - it_o) <= max(3, 0.05 * it_o), (res, it_o)
    assert om.true_residual(b, _host(xg), h1, h2) <= 1e-10
    m.close()


def test_schwarz_errors(semlib):
    print("case: schwarz error paths", flush=True)
    L = semlib._lib
    # N = 1: the one-node overlap spans the neighbours, interior local problems are singular
    m1 = semlib.box_mesh(1, (3, 3, 3))
    with pytest.raises(L.SemError) as e:
        m1.set_schwarz(True)
    assert e.value.status == L.SEM_EUNSUPPORTED
    m1.close()
    m = semlib.box_mesh(3, (2, 2, 2), with_fp32=True)
    m.set_schwarz(True)
    b = m.zeros()
    b.fill_(1.0)
    with pytest.raises(L.SemError) as e:
        m.solve(b, precision="mixed")
    assert e.value.status == L.SEM_EUNSUPPORTED
    batch = semlib.Batch(max_slots=2)
    with pytest.raises(L.SemError) as e:
        batch.admit(m, b)
    assert e.value.status == L.SEM_EUNSUPPORTED
    batch.close()
    m.set_schwarz(False)
    assert not m.schwarz_info()["enabled"]
    m.close()


@pytest.mark.parametrize("N,nel,periodic,seed", [(3, (1, 3, 2), (0, 0, 0), 71), (4, (2, 3, 2), (1, 0, 0), 72),
                                                 (2, (3, 2, 2), (0, 0, 1), 73)])
def test_schwarz_degenerate_lattices(semlib, oracle_mod, N, nel, periodic, seed):
    """A single element across an axis (no neighbour on either side) and
    periodic axes with two elements (both neighbours are the same element):
    M^-1 r against the oracle."""
    print(f"case: schwarz degenerate N={N} nel={nel} periodic={periodic}", flush=True)
    m, om = _meshes(semlib, oracle_mod, "box", N, nel, periodic, seed)
    S = SchwarzOracle(om)
    m.set_schwarz(True)
    r = _continuous(om, 800 + seed)
    z = _host(m.precond(_dev(r)))
    e2, einf = _relerr(z, S.apply(r))
    assert e2 <= TOL and einf <= TOL, (e2, einf)
    zg = np.zeros(om.nglob)
    zg[om.numbering()] = z
    assert np.array_equal(zg[om.numbering()], z)
    m.close()
