"""Two-level preconditioner (Jacobi plus the coarse term of Eq. 6) on the GPU
against the oracle (oracle/coarse.py, pinned in test_oracle_coarse.py):
coarse-space sizes and Chebyshev interval, M^-1 r element by element, whole
CG runs (iterations, the iterate after a fixed number of steps, the true
residual), the Helmholtz form, rebuilds, and the error paths."""
import numpy as np
import pytest
import torch

import seeded_inputs as SI
from oracle.coarse import CoarseOracle
from oracle.schwarz import pcg

pytestmark = pytest.mark.gpu

K, FRAC = 10, 0.01


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b), np.max(np.abs(a - b)) / np.max(np.abs(b))


class _Op:
    """The oracle mesh with a fixed Helmholtz form, for oracle.schwarz.pcg."""

    def __init__(self, om, h1=None, h2=None):
        self.om, self.h1, self.h2 = om, h1, h2
        self.nloc = om.nloc

    def apply(self, x):
        return self.om.apply(x, self.h1, self.h2)

    def dot(self, a, b):
        return self.om.dot(a, b)


def _meshes(semlib, oracle_mod, kind, N, nel, periodic, seed):
    if kind == "pipe":
        return (semlib.pipe_mesh(*nel, N=N, length=2.0, with_fp32=True),
                oracle_mod.pipe_mesh(*nel, N=N, length=2.0))
    V = SI.jittered_box_vertices(nel, seed=seed)
    return (semlib.box_mesh(N, nel, vertices=V, periodic=periodic, with_fp32=True),
            oracle_mod.OracleMesh(N, nel, vertices=V, periodic=periodic))


def _continuous(om, seed):
    g = SI.uniform_global_values(om.nglob, seed=seed)
    return g[om.numbering()] * (om.local_mask() == 0)


CASES = [
    ("box", 3, (3, 2, 2), (0, 0, 0), 1),
    ("box", 5, (3, 3, 4), (0, 0, 1), 2),
    ("box", 4, (2, 3, 2), (1, 0, 1), 3),
    ("box", 2, (5, 4, 3), (0, 0, 0), 4),
    ("pipe", 5, (4, 4, 3), None, 5),
    ("box", 9, (2, 2, 2), (0, 0, 0), 6),
]


@pytest.mark.parametrize("kind,N,nel,periodic,seed", CASES)
def test_coarse_space_and_apply(semlib, oracle_mod, kind, N, nel, periodic, seed):
    print(f"case: coarse apply {kind} N={N} nel={nel} periodic={periodic}", flush=True)
    m, om = _meshes(semlib, oracle_mod, kind, N, nel, periodic, seed)
    C = CoarseOracle(om, k=K, frac=FRAC)
    m.set_coarse(K, FRAC)
    info = m.coarse_info()
    assert info["n_vertices"] == C.nvert
    assert info["n_coarse"] == int(C.keep.sum())
    assert info["chebyshev_steps"] == K
    assert abs(info["b"] - C.b) <= 1e-12 * C.b, (info["b"], C.b)
    assert abs(info["a"] - FRAC * info["b"]) <= 1e-15 * info["b"]
    # stored entries: at least the non-zeros of A0's kept rows, at most 27 per row
    assert int(np.count_nonzero(C.A0[C.keep])) <= info["nnz"] <= 27 * info["n_coarse"]
    for s in range(2):
        r = _continuous(om, 100 * seed + s)
        z = _host(m.precond(_dev(r)))
        ref = C.apply(r)
        e2, einf = _relerr(z, ref)
        assert e2 <= 1e-12 and einf <= 1e-12, (s, e2, einf)
        # z is continuous and masked
        live = om.local_mask() == 0
        assert np.all(z[~live] == 0.0)
        zg = np.zeros(om.nglob)
        zg[om.numbering()] = z
        assert np.max(np.abs(zg[om.numbering()] - z)) <= 1e-13 * np.max(np.abs(z))
    # removing the coarse space leaves Jacobi: exactly invdiag * r
    m.set_coarse(0)
    assert m.coarse_info()["chebyshev_steps"] == 0
    r = _continuous(om, 7 * seed)
    _, _, inv = m.export_geom()
    assert np.array_equal(_host(m.precond(_dev(r))), inv * r)
    m.close()


def test_coarse_symmetric_positive(semlib, oracle_mod):
    """<M^-1 r1, r2> = <r1, M^-1 r2> and <r, M^-1 r> > 0 (unique-dof products)."""
    print("case: coarse symmetry pipe 6x6x5 N=7", flush=True)
    m = semlib.pipe_mesh(6, 6, 5, N=7, length=2.0)
    om = oracle_mod.pipe_mesh(6, 6, 5, N=7, length=2.0)
    m.set_coarse(K, FRAC)
    r1, r2 = _continuous(om, 11), _continuous(om, 12)
    z1, z2 = _host(m.precond(_dev(r1))), _host(m.precond(_dev(r2)))
    a, b = om.dot(z1, r2), om.dot(r1, z2)
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))
    assert om.dot(r1, z1) > 0 and om.dot(r2, z2) > 0
    m.close()


PCG_CASES = [
    ("box", 5, (4, 4, 3), (0, 0, 0), 21),
    ("pipe", 5, (6, 6, 5), None, 22),
    ("box", 7, (3, 3, 4), (0, 0, 1), 23),
    ("box", 4, (3, 3, 3), (0, 0, 0), 24),  # even N: the FP32 update takes one node per lane
]


@pytest.mark.parametrize("kind,N,nel,periodic,seed", PCG_CASES)
def test_coarse_pcg(semlib, oracle_mod, kind, N, nel, periodic, seed):
    print(f"case: coarse pcg {kind} N={N} nel={nel}", flush=True)
    m, om = _meshes(semlib, oracle_mod, kind, N, nel, periodic, seed)
    x, y, z = om.coords()
    b = om.mass(SI.sin3_forcing(x, y, z))
    C = CoarseOracle(om, k=K, frac=FRAC)
    xo, it_o = pcg(_Op(om), b, C.apply, tol=1e-10)
    _, rj = om.pcg(b, tol=1e-10)
    assert it_o < rj.iterations
    m.set_coarse(K, FRAC)
    for graph, poll in ((True, 16), (False, 5)):
        xg, res = m.solve(_dev(b), tol=1e-10, use_graph=graph, poll_every=poll)
        assert res.ok, res
        assert abs(res.iterations - it_o) <= max(3, 0.05 * it_o), (graph, res.iterations, it_o)
        assert om.true_residual(b, _host(xg)) <= 1e-10
    # mixed precision: FP32 inner CG with the same coarse term (FP64 coarse solve)
    xg, res = m.solve(_dev(b), tol=1e-10, precision="mixed")
    assert res.ok, res
    assert om.true_residual(b, _host(xg)) <= 1e-10
    assert res.iterations < rj.iterations, (res.iterations, rj.iterations)
    # the same Krylov iterate after a fixed number of steps
    for steps in (1, 6):
        xs, _ = pcg(_Op(om), b, C.apply, tol=1e-30, max_iter=steps)
        xg, res = m.solve(_dev(b), fixed_iters=steps)
        assert res.iterations == steps
        e2, einf = _relerr(_host(xg), xs)
        assert e2 <= 1e-10 and einf <= 1e-10, (steps, e2, einf)
    m.close()


def test_coarse_helmholtz_and_rebuild(semlib, oracle_mod):
    """The coarse space follows the operator: set before sem_set_helmholtz it
    is rebuilt for the Helmholtz form; back to Poisson with both NULL."""
    print("case: coarse helmholtz box 3x3x2 N=5", flush=True)
    nel = (3, 3, 2)
    m, om = _meshes(semlib, oracle_mod, "box", 5, nel, (0, 0, 0), 31)
    h1 = SI.uniform_local(om.nloc, 32, 0.5, 2.0)
    h2 = SI.uniform_local(om.nloc, 33, 0.0, 3.0)
    m.set_coarse(K, FRAC)
    b_poisson = m.coarse_info()["b"]
    m.set_helmholtz(_dev(h1), _dev(h2))
    C = CoarseOracle(om, k=K, frac=FRAC, h1=h1, h2=h2)
    assert abs(m.coarse_info()["b"] - C.b) <= 1e-12 * C.b
    r = _continuous(om, 34)
    e2, einf = _relerr(_host(m.precond(_dev(r))), C.apply(r))
    assert e2 <= 1e-12 and einf <= 1e-12, (e2, einf)
    x, y, z = om.coords()
    b = om.mass(SI.sin3_forcing(x, y, z))
    _, it_o = pcg(_Op(om, h1, h2), b, C.apply, tol=1e-10)
    xg, res = m.solve(_dev(b), tol=1e-10)
    assert res.ok and abs(res.iterations - it_o) <= max(3, 0.05 * it_o), (res, it_o)
    assert om.true_residual(b, _host(xg), h1, h2) <= 1e-10
    m.set_helmholtz(None, None)
    assert abs(m.coarse_info()["b"] - b_poisson) <= 1e-14 * b_poisson
    m.close()


def test_coarse_periodic_helmholtz(semlib, oracle_mod):
    """Fully periodic box: no Dirichlet node; h2 B keeps A and A0 definite."""
    print("case: coarse periodic helmholtz box 3x3x3 N=4", flush=True)
    nel = (3, 3, 3)
    m, om = _meshes(semlib, oracle_mod, "box", 4, nel, (1, 1, 1), 41)
    h1 = np.ones(om.nloc)
    h2 = SI.uniform_local(om.nloc, 42, 0.5, 1.5)
    m.set_helmholtz(None, _dev(h2))
    m.set_coarse(K, FRAC)
    C = CoarseOracle(om, k=K, frac=FRAC, h1=None, h2=h2)
    assert m.coarse_info()["n_vertices"] == 27 == C.nvert
    r = _continuous(om, 43)
    e2, einf = _relerr(_host(m.precond(_dev(r))), C.apply(r))
    assert e2 <= 1e-12 and einf <= 1e-12, (e2, einf)
    x, y, z = om.coords()
    b = om.mass(SI.sin3_forcing(x, y, z))
    xg, res = m.solve(_dev(b), tol=1e-10)
    assert res.ok
    assert om.true_residual(b, _host(xg), h1, h2) <= 1e-10
    m.close()


def test_coarse_errors(semlib):
    print("case: coarse error paths", flush=True)
    m = semlib.box_mesh(3, (2, 2, 2), with_fp32=True)
    L = semlib._lib
    for steps, frac in ((-1, 0.1), (1001, 0.1), (5, 0.0), (5, 1.0), (5, float("nan"))):
        with pytest.raises(L.SemError) as e:
            m.set_coarse(steps, frac)
        assert e.value.status == L.SEM_EINVAL
    m.set_coarse(5, 0.05)
    b = m.zeros()
    b.fill_(1.0)
    batch = semlib.Batch(max_slots=2)
    # batched slots take the coarse term, not the Schwarz local solves
    m.set_schwarz(True)
    with pytest.raises(L.SemError) as e:
        batch.admit(m, b)
    assert e.value.status == L.SEM_EUNSUPPORTED
    m.set_schwarz(False)
    batch.close()
    r = m.zeros()
    with pytest.raises(ValueError):
        m.precond(r, r)
    m.set_coarse(0)
    m.close()


def test_coarse_helmholtz_mixed_and_projection(semlib, oracle_mod):
    """The coarse term in the FP32 inner solves of a mixed Helmholtz solve, and
    in solves started from the projection onto previous solutions: both meet
    the true residual (measured by the oracle) with fewer iterations than
    without the coarse term."""
    print("case: coarse helmholtz mixed + projection box 4x4x3 N=5", flush=True)
    nel = (4, 4, 3)
    m, om = _meshes(semlib, oracle_mod, "box", 5, nel, (0, 0, 0), 51)
    h1 = SI.uniform_local(om.nloc, 52, 0.5, 2.0)
    h2 = SI.uniform_local(om.nloc, 53, 0.0, 3.0)
    m.set_helmholtz(_dev(h1), _dev(h2))
    x, y, z = om.coords()
    b = om.mass(SI.sin3_forcing(x, y, z))
    _, plain = m.solve(_dev(b), tol=1e-10, precision="mixed")
    m.set_coarse(K, FRAC)
    xg, res = m.solve(_dev(b), tol=1e-10, precision="mixed")
    assert res.ok and res.iterations < plain.iterations, (res, plain)
    assert om.true_residual(b, _host(xg), h1, h2) <= 1e-10
    # projection: successive right-hand sides (a forcing travelling in time)
    proj = semlib.Projection(m, max_vectors=4)
    iters = []
    for t in range(4):
        bt = om.mass(SI.travelling_forcing(x, y, z, 0.1 * t))
        xt, rt = proj.solve(_dev(bt), tol=1e-10)
        assert rt.ok
        assert om.true_residual(bt, _host(xt), h1, h2) <= 1e-10
        iters.append(rt.iterations)
    assert iters[-1] < iters[0], iters
    proj.close()
    m.close()


DEGENERATE = [
    ("box", 3, (1, 3, 2), (0, 0, 0), 61),   # one element across x
    ("box", 4, (2, 1, 3), (1, 1, 0), 62),   # periodic x with two elements, periodic y with one
    ("box", 2, (3, 2, 1), (0, 0, 1), 63),   # periodic z with one element: its two z-faces are one
]


@pytest.mark.parametrize("kind,N,nel,periodic,seed", DEGENERATE)
def test_coarse_degenerate_lattices(semlib, oracle_mod, kind, N, nel, periodic, seed):
    """Lattices where periodic images of a vertex coincide within one element
    or an axis has a single element: the vertex space, A0 and M^-1 r against
    the oracle."""
    print(f"case: coarse degenerate {kind} N={N} nel={nel} periodic={periodic}", flush=True)
    m, om = _meshes(semlib, oracle_mod, kind, N, nel, periodic, seed)
    C = CoarseOracle(om, k=K, frac=FRAC)
    m.set_coarse(K, FRAC)
    info = m.coarse_info()
    assert info["n_vertices"] == C.nvert and info["n_coarse"] == int(C.keep.sum())
    assert abs(info["b"] - C.b) <= 1e-12 * C.b
    r = _continuous(om, 700 + seed)
    e2, einf = _relerr(_host(m.precond(_dev(r))), C.apply(r))
    assert e2 <= 1e-12 and einf <= 1e-12, (e2, einf)
    m.close()


def test_coarse_cg_with_odd_grids(semlib, oracle_mod):
    """The coarse-corrected operator sizes its grid to whole rounds of its
    resident workgroups and reports it for the dot partials: CG (FP64 and
    mixed) and the operator's u.w agree with the oracle under odd grid caps
    and several tile shapes."""
    print("case: coarse cg with odd grid caps box 5x4x3 N=5", flush=True)
    nel = (5, 4, 3)
    m, om = _meshes(semlib, oracle_mod, "box", 5, nel, (0, 0, 0), 91)
    x, y, z = om.coords()
    b = om.mass(SI.sin3_forcing(x, y, z))
    C = CoarseOracle(om, k=K, frac=FRAC)
    _, it_o = pcg(_Op(om), b, C.apply, tol=1e-10)
    m.set_coarse(K, FRAC)
    u = SI.random_local(om.nloc, 92)
    ref_dot = float(np.sum(u * om.ax(u)))
    for epw, grid in ((1, 7), (2, 13), (3, 1000), (1, 0)):
        m.set_operator_config(epw, grid)
        for prec in ("fp64", "mixed"):
            xg, res = m.solve(_dev(b), tol=1e-10, precision=prec)
            assert res.ok, (epw, grid, prec, res)
            assert om.true_residual(b, _host(xg)) <= 1e-10
            if prec == "fp64":
                assert abs(res.iterations - it_o) <= max(3, 0.05 * it_o), (epw, grid, res.iterations, it_o)
        _, d = m.ax(_dev(u), dot=True)
        assert abs(float(d.item()) - ref_dot) <= 1e-12 * abs(ref_dot), (epw, grid)
    m.close()
