"""Failure and degenerate cases of the solvers: each ends with its status and
a usable x, never with a hang (the iteration limits and breakdown flags are
checked on the device and read by the host)."""
import numpy as np
import pytest
import torch

import seeded_inputs as SI

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def box(semlib, oracle_mod):
    nel = (3, 3, 2)
    V = SI.jittered_box_vertices(nel, seed=9)
    m = semlib.box_mesh(5, nel, vertices=V, with_fp32=True)
    om = oracle_mod.OracleMesh(5, nel, vertices=V)
    x, y, z = om.coords()
    b = om.mass(SI.sin3_forcing(x, y, z))
    yield m, om, b
    m.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_iteration_limit(semlib, box, prec):
    print(f"case: iteration limit {prec}", flush=True)
    m, om, b = box
    xg, res = m.solve(_dev(b), tol=1e-10, max_iter=5, precision=prec, raise_on_error=False)
    assert res.status == 4 and not res.ok  # SEM_ENOCONV
    assert res.iterations <= 5
    # x holds the last iterate (finite, nonzero, not converged; CG after a few
    # steps need not have a smaller residual norm than x = 0)
    xh = _host(xg)
    assert np.all(np.isfinite(xh)) and np.any(xh)
    assert om.true_residual(b, xh) > 1e-10
    with pytest.raises(semlib.SemError) as ei:
        m.solve(_dev(b), tol=1e-10, max_iter=5, precision=prec)
    assert ei.value.status == 4


def test_zero_rhs(semlib, box):
    print("case: zero right-hand side", flush=True)
    m, om, b = box
    for prec in ("fp64", "mixed"):
        x0 = _dev(np.full(om.nloc, 3.0))
        xg, res = m.solve(_dev(np.zeros(om.nloc)), x0, tol=1e-10, precision=prec, initial_guess=False)
        assert res.ok and res.iterations == 0
        assert not np.any(_host(xg))


def test_breakdown_on_indefinite_operator(semlib, box):
    """h1 < 0 makes A negative definite: p.Ap < 0 at the first step."""
    print("case: CG breakdown", flush=True)
    m, om, b = box
    m.set_helmholtz(_dev(np.full(om.nloc, -1.0)), None)
    try:
        _, res = m.solve(_dev(b), tol=1e-10, raise_on_error=False)
        assert res.status == 5  # SEM_EBREAKDOWN
        _, res = m.solve(_dev(b), tol=1e-10, precision="mixed", raise_on_error=False)
        assert res.status == 5
    finally:
        m.set_helmholtz(None, None)
    _, res = m.solve(_dev(b), tol=1e-10)
    assert res.ok


def test_initial_guess_is_used(semlib, box):
    print("case: initial guess", flush=True)
    m, om, b = box
    xs, r0 = m.solve(_dev(b), tol=1e-10)
    # starting from the solution takes no iteration
    x1, r1 = m.solve(_dev(b), xs.clone(), tol=1e-10, initial_guess=True)
    assert r1.ok and r1.iterations == 0
    assert om.true_residual(b, _host(x1)) <= 1e-10
    # starting from a perturbed continuous guess converges in fewer iterations than from zero
    g = np.zeros(om.nglob)
    g[om.numbering()] = _host(xs)
    g += 1e-4 * SI.uniform_global_values(om.nglob, 5)
    guess = g[om.numbering()]
    guess[om.local_mask() == 1] = 0.0
    x2, r2 = m.solve(_dev(b), _dev(guess), tol=1e-10, initial_guess=True)
    assert r2.ok and 0 < r2.iterations < r0.iterations
    assert om.true_residual(b, _host(x2)) <= 1e-10
