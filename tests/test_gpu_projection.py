"""Projection onto previous solutions (sem_proj_*) against the projection
oracle: the same basis gives the same guess, and sequences of solves agree
in iterations and reach the tolerance measured by the oracle."""
import numpy as np
import pytest
import torch

import seeded_inputs as SI
from oracle.projection import ProjectionSpace

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _continuous(om, seed):
    v = SI.uniform_global_values(om.nglob, seed)[om.numbering()]
    v[om.local_mask() == 1] = 0.0
    return v


def _box(semlib, oracle_mod, N, nel, seed):
    V = SI.jittered_box_vertices(nel, seed=seed)
    return semlib.box_mesh(N, nel, vertices=V, with_fp32=True), oracle_mod.OracleMesh(N, nel, vertices=V)


def test_project_add_drop_restart(semlib, oracle_mod):
    print("case: projection basis, box 3x2x2 N=5", flush=True)
    m, om = _box(semlib, oracle_mod, 5, (3, 2, 2), 3)
    P = semlib.Projection(m, max_vectors=5)
    ref = ProjectionSpace(om, 5)
    vs = [_continuous(om, 50 + s) for s in range(4)]
    for v in vs:
        assert P.add(_dev(v)) == ref.add(v)
    assert len(P) == len(ref) == 4
    b = om.mass(SI.sin3_forcing(*om.coords()))
    xg, xo = _host(P.project(_dev(b))), ref.project(b)
    assert np.linalg.norm(xg - xo) <= 1e-11 * np.linalg.norm(xo)
    # exact on the span
    x = 0.5 * vs[0] - 2.0 * vs[3]
    xb = _host(P.project(_dev(om.apply(x))))
    assert np.linalg.norm(xb - x) <= 1e-10 * np.linalg.norm(x)
    # a dependent vector is dropped, a full basis restarts
    assert not P.add(_dev(vs[1] + vs[2]))
    assert len(P) == 4
    assert P.add(_dev(_continuous(om, 60))) and len(P) == 5
    assert P.add(_dev(_continuous(om, 61))) and len(P) == 1
    P.reset()
    assert len(P) == 0
    assert not np.any(_host(P.project(_dev(b))))
    P.close()
    m.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_projected_solve_sequence(semlib, oracle_mod, prec):
    print(f"case: projected solves {prec}, box 4x4x4 N=7", flush=True)
    m, om = _box(semlib, oracle_mod, 7, (4, 4, 4), 1)
    x, y, z = om.coords()
    P = semlib.Projection(m, max_vectors=8)
    ref = ProjectionSpace(om, 8)
    its = []
    for t in range(6):
        b = om.mass(SI.travelling_forcing(x, y, z, float(t)))
        xg, r = P.solve(_dev(b), tol=1e-10, precision=prec)
        xo, ro = ref.solve(b, tol=1e-10)
        assert r.ok, r
        assert om.true_residual(b, _host(xg)) <= 1e-10, (t, r)
        if prec == "fp64":
            assert abs(r.iterations - ro.iterations) <= max(3, 0.1 * ro.iterations), (t, r.iterations, ro.iterations)
        its.append(r.iterations)
    assert its[-1] < its[0] / 3, its
    # changing the operator empties the basis
    assert len(P) > 0
    m.set_helmholtz(None, _dev(np.ones(om.nloc)))
    assert len(P) == 0
    P.close()
    m.close()
