"""Helmholtz form of the operator (Eq. 4 with Algorithm 1's per-point h1):
h1-weighted stiffness plus h2 B, its Jacobi diagonal and CG, against the
oracle (whose Helmholtz operator and diagonal are pinned by dense assembly)."""
import numpy as np
import pytest
import torch

import seeded_inputs as SI

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b), np.max(np.abs(a - b)) / np.max(np.abs(b))


def _case(semlib, oracle_mod, N, nel, seed, periodic=(0, 0, 0)):
    V = SI.jittered_box_vertices(nel, seed=seed)
    m = semlib.box_mesh(N, nel, vertices=V, periodic=periodic, with_fp32=True)
    om = oracle_mod.OracleMesh(N, nel, vertices=V, periodic=periodic)
    h1 = SI.uniform_local(om.nloc, 40 + seed, 0.5, 2.0)
    h2 = SI.uniform_local(om.nloc, 60 + seed, 0.0, 3.0)
    return m, om, h1, h2


@pytest.mark.parametrize("N", [1, 3, 5, 7, 8, 9, 10, 12])
def test_helmholtz_operator_and_diagonal(semlib, oracle_mod, N):
    nel = (3, 2, 2) if N <= 9 else (2, 1, 2)
    print(f"case: helmholtz ax N={N} nel={nel}", flush=True)
    m, om, h1, h2 = _case(semlib, oracle_mod, N, nel, seed=N)
    m.set_helmholtz(_dev(h1), _dev(h2))
    u = SI.random_local(om.nloc, 300 + N)
    ref = om.ax(u, h1=h1, h2=h2)
    e2, einf = _relerr(_host(m.ax(_dev(u))), ref)
    assert e2 <= 1e-12 and einf <= 1e-12, (e2, einf)
    # FP32: the coefficients and factors carry FP32 rounding as well
    u32 = u.astype(np.float32)
    e2, einf = _relerr(_host(m.ax(_dev(u32, torch.float32))), om.ax(u32.astype(np.float64), h1=h1, h2=h2))
    assert e2 <= 2e-6 and einf <= 2e-5, (e2, einf)
    # Jacobi preconditioner of the Helmholtz operator
    _, _, inv = m.export_geom()
    invo = om.jacobi(h1=h1, h2=h2)
    assert np.max(np.abs(inv - invo)) <= 1e-12 * np.abs(invo).max()
    # h1 only, h2 only
    m.set_helmholtz(_dev(h1), None)
    e2, _ = _relerr(_host(m.ax(_dev(u))), om.ax(u, h1=h1))
    assert e2 <= 1e-12
    m.set_helmholtz(None, _dev(h2))
    e2, _ = _relerr(_host(m.ax(_dev(u))), om.ax(u, h2=h2))
    assert e2 <= 1e-12
    m.close()


def test_helmholtz_pcg_dirichlet_box(semlib, oracle_mod):
    print("case: helmholtz pcg box 4x4x4 N=7", flush=True)
    m, om, h1, h2 = _case(semlib, oracle_mod, 7, (4, 4, 4), seed=5)
    x, y, z = om.coords()
    b = om.mass(SI.sin3_forcing(x, y, z))
    _, ro = om.pcg(b, tol=1e-10, h1=h1, h2=h2)
    m.set_helmholtz(_dev(h1), _dev(h2))
    for prec in ("fp64", "mixed"):
        xg, res = m.solve(_dev(b), tol=1e-10, precision=prec)
        assert res.ok, (prec, res)
        assert om.true_residual(b, _host(xg), h1, h2) <= 1e-10, (prec, res)
        if prec == "fp64":
            assert abs(res.iterations - ro.iterations) <= max(3, 0.05 * ro.iterations), (res, ro)
    m.close()


def test_helmholtz_pcg_periodic_box(semlib, oracle_mod):
    """Fully periodic box: no Dirichlet node, the h2 B term makes A definite."""
    print("case: helmholtz pcg periodic box 3x3x3 N=5", flush=True)
    m, om, h1, h2 = _case(semlib, oracle_mod, 5, (3, 3, 3), seed=6, periodic=(1, 1, 1))
    h2 = h2 + 0.5
    vg = SI.uniform_global_values(om.nglob, 8)
    b = om.mass(vg[om.numbering()])
    _, ro = om.pcg(b, tol=1e-10, h1=h1, h2=h2)
    m.set_helmholtz(_dev(h1), _dev(h2))
    xg, res = m.solve(_dev(b), tol=1e-10)
    assert res.ok, res
    assert om.true_residual(b, _host(xg), h1, h2) <= 1e-10
    assert abs(res.iterations - ro.iterations) <= max(3, 0.05 * ro.iterations), (res, ro)
    m.close()


def test_helmholtz_restore_and_batch(semlib, oracle_mod):
    print("case: helmholtz restore + batch rejection", flush=True)
    m, om, h1, h2 = _case(semlib, oracle_mod, 5, (2, 3, 2), seed=7)
    u = SI.random_local(om.nloc, 11)
    m.set_helmholtz(_dev(h1), _dev(h2))
    B = semlib.Batch(max_slots=2)
    with pytest.raises(semlib.SemError) as ei:
        B.admit(m, _dev(om.mass(np.ones(om.nloc))))
    assert ei.value.status == 7  # SEM_EUNSUPPORTED
    B.close()
    m.set_helmholtz(None, None)
    e2, einf = _relerr(_host(m.ax(_dev(u))), om.ax(u))
    assert e2 <= 1e-12 and einf <= 1e-12
    _, _, inv = m.export_geom()
    invo = om.jacobi()
    assert np.max(np.abs(inv - invo)) <= 1e-12 * np.abs(invo).max()
    m.close()
