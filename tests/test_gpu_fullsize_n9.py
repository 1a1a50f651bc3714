"""Full-size parity at N = 9: the 48x48x48 pipe (110,592 elements, 110.6M
local nodes; order 9 probes the LDS/register balance of the operator).

  * maps and multiplicities bit-exact against the oracle's numbering;
  * on the oracle's own geometric factors (sem_load_geometry): the operator
    on sampled elements, the corner columns included, and the fused Ax+gs on
    the whole mesh against the oracle's assembled apply, at 1e-12 norm-wise
    and max-norm;
  * FP64 and mixed solves of the seeded noise right-hand side whose true
    residual the oracle measures on the whole mesh (<= 1e-10), with the
    mixed solve's difference from the FP64 solve reported.
"""
import numpy as np
import pytest
import torch

import seeded_inputs as SI

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

NEL = (48, 48, 48)
N = 9


@pytest.fixture(scope="module")
def pipe9(semlib, oracle_mod):
    print("case: pipe 48x48x48 N=9 setup on the oracle's geometry", flush=True)
    om = oracle_mod.pipe_mesh(*NEL, N=N)
    m = semlib.pipe_mesh(*NEL, N=N, with_fp32=True)
    gid, mult, mask = m.export_maps()
    assert np.array_equal(gid, om.numbering())
    assert np.array_equal(mult, om.local_mult())
    assert np.array_equal(mask, om.local_mask())
    del gid, mult, mask
    G, B = om.geom()
    m.load_geometry(G, B)
    del G, B
    yield m, om
    m.close()


def test_n9_ax_axgs_on_oracle_geometry(pipe9):
    m, om = pipe9
    print("case: pipe N=9 ax sampled + axgs whole", flush=True)
    assert m.info.n_shared_local == 53377536 and m.info.n_shared_global == 23780784
    rng = np.random.default_rng(9)
    nx, ny, nz = NEL
    corners = [ex + nx * (ey + ny * ez) for ez in (0, nz // 2, nz - 1)
               for ex in (0, 1, nx - 1) for ey in (0, 1, ny - 1)]
    elems = np.unique(np.concatenate([rng.integers(0, om.E, 48), corners, [0, om.E - 1]])).astype(np.int64)
    u = SI.random_local(om.nloc, 29)
    ud = torch.from_numpy(u).cuda()
    w = m.ax(ud).cpu().numpy()
    P3 = (N + 1) ** 3
    ref = om.ax(np.concatenate([u[e * P3:(e + 1) * P3] for e in elems]), elems=elems)
    for q, e in enumerate(elems):
        a, b = w[e * P3:(e + 1) * P3], ref[q * P3:(q + 1) * P3]
        err = max(np.linalg.norm(a - b) / np.linalg.norm(b), np.max(np.abs(a - b)) / np.max(np.abs(b)))
        assert err <= 1e-12, (int(e), err)
    del w, ref
    refg = om.apply(u)
    for fused in (False, True):
        m.set_axgs_config(fused)
        wg = m.axgs(ud).cpu().numpy()
        e2 = np.linalg.norm(wg - refg) / np.linalg.norm(refg)
        einf = np.max(np.abs(wg - refg)) / np.max(np.abs(refg))
        print(f"  axgs (fused={fused}) whole mesh: {e2:.2e} norm-wise, {einf:.2e} max-norm", flush=True)
        assert e2 <= 1e-12 and einf <= 1e-12, (fused, e2, einf)
    m.set_axgs_config(False)


def test_n9_solves_on_oracle_geometry(pipe9):
    m, om = pipe9
    gid = om.numbering()
    b = SI.uniform_global_values(om.nglob, 2)[gid]
    b[om.local_mask() == 1] = 0.0
    bd = torch.from_numpy(b).cuda()
    xs = {}
    for prec in ("fp64", "mixed"):
        print(f"case: pipe N=9 solve {prec}", flush=True)
        x, res = m.solve(bd, tol=1e-10, max_iter=40000, precision=prec, poll_every=50)
        xh = x.cpu().numpy()
        rel = om.true_residual(b, xh)
        print(f"  {prec}: iterations {res.iterations}, outer {res.outer_iterations}, "
              f"oracle residual {rel:.3e}", flush=True)
        assert res.ok and rel <= 1e-10, (prec, rel)
        xs[prec] = xh
    d = np.sqrt(om.dot(xs["mixed"] - xs["fp64"], xs["mixed"] - xs["fp64"]) / om.dot(xs["fp64"], xs["fp64"]))
    print(f"  mixed vs fp64 solution: {d:.2e}", flush=True)
