"""GPU tests of the fused operator and gather-scatter (sem_axgs with the face
sums a workgroup holds done in the operator's epilogue, the rest by a
residual plan).

Bars: the fused result is the same bits as sem_ax followed by sem_gs (both add
each node's copies in ascending local index from 0), for every tile shape and
line count tried, FP64 and FP32; against the FP64 oracle the operator bar
(1e-12 norm-wise and max-norm relative); solves through the fused CG reach a
true relative residual <= 1e-10 measured by the oracle.
"""
import numpy as np
import pytest
import torch

import seeded_inputs as SI

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _unfused(m, u):
    w = m.ax(u)
    m.gs(w)
    torch.cuda.synchronize()
    return w


def _fused(m, u):
    w = torch.full_like(u, float("nan"))  # every entry must be written
    m.axgs(u, w)
    torch.cuda.synchronize()
    return w


def _same_bits(a, b):
    return torch.equal(a.view(torch.int64) if a.dtype == torch.float64 else a.view(torch.int32),
                       b.view(torch.int64) if b.dtype == torch.float64 else b.view(torch.int32))


# (N, nel, periodic, dirichlet_faces, jitter): boxes with ragged line counts,
# periodic seams on every axis and Neumann faces (dirichlet_faces bitmask:
# bit 2a = low face of axis a, bit 2a+1 = high face)
CASES = [
    (7, (4, 4, 4), (0, 0, 0), -1, True),
    (7, (5, 3, 4), (0, 0, 1), -1, True),
    (5, (6, 5, 3), (1, 0, 0), -1, True),
    (4, (3, 4, 5), (0, 1, 0), -1, False),
    (3, (4, 4, 3), (1, 1, 1), -1, False),
    (6, (5, 4, 3), (0, 0, 0), 0b010110, True),   # x-low, y-high, z-low Neumann
    (2, (7, 3, 2), (0, 0, 0), 0, True),          # pure Neumann
    (7, (1, 3, 2), (0, 0, 0), -1, True),         # one element per line
    (7, (2, 1, 2), (1, 1, 0), -1, False),        # two-element periodic line, one line per plane
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("shape", [(0, 0), (1, 1), (2, 2), (3, 3), (4, 5), (1, 1000)])
def test_fused_equals_operator_then_gs(semlib, oracle_mod, case, shape):
    N, nel, per, faces, jit = CASES[case]
    epw, lines = shape
    if epw * (N + 1) ** 2 > 512:
        pytest.skip("tile wider than a workgroup")
    print(f"case: fused N={N} nel={nel} periodic={per} faces={faces} epw={epw} lines={lines}", flush=True)
    V = SI.jittered_box_vertices(nel, seed=11 + case) if jit and not any(per) else None
    m = semlib.box_mesh(N, nel, vertices=V, periodic=per, dirichlet_faces=faces, with_fp32=True)
    n_lines = nel[1] * nel[2]
    m.set_axgs_config(True, epw, min(lines, n_lines) if lines else 0)
    info = m.axgs_info()
    assert info["enabled"] == 1
    assert info["residual_ids"] <= m.info.n_shared_global
    u = _dev(SI.random_local(m.n_local, 300 + case))
    for dt in (torch.float64, torch.float32):
        uu = u.to(dt)
        wf, wu = _fused(m, uu), _unfused(m, uu)
        assert not torch.isnan(wf).any()
        assert _same_bits(wf, wu), (dt, (wf - wu).abs().max().item())
    # the FP64 result against the oracle
    om = oracle_mod.OracleMesh(N, nel, vertices=V, periodic=per, dirichlet=None if faces < 0 else faces)
    ref = om.apply(u.cpu().numpy())
    w = _fused(m, u).cpu().numpy()
    assert np.linalg.norm(w - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.max(np.abs(w - ref)) <= 1e-12 * np.max(np.abs(ref))
    m.close()


@pytest.mark.parametrize("N", list(range(2, 13)))
def test_fused_all_orders(semlib, N):
    nel = (3, 3, 2) if N <= 9 else (2, 3, 2)
    print(f"case: fused orders N={N} nel={nel}", flush=True)
    V = SI.jittered_box_vertices(nel, seed=N)
    m = semlib.box_mesh(N, nel, vertices=V, with_fp32=True)
    for lines in (0, 2):
        m.set_axgs_config(True, 0, lines)
        assert m.axgs_info()["enabled"] == 1
        u = _dev(SI.random_local(m.n_local, 500 + N))
        for dt in (torch.float64, torch.float32):
            uu = u.to(dt)
            assert _same_bits(_fused(m, uu), _unfused(m, uu)), (N, lines, dt)
    m.close()


def test_fused_not_used_where_it_does_not_apply(semlib):
    print("case: fused availability", flush=True)
    m = semlib.box_mesh(1, (3, 3, 3))
    m.set_axgs_config(True)
    assert m.axgs_info()["enabled"] == 0  # order 1: no interior t-plane
    m.close()
    m = semlib.box_mesh(7, (3, 3, 3))
    assert m.axgs_info()["enabled"] == 0  # opt-in
    m.set_axgs_config(False)
    assert m.axgs_info()["enabled"] == 0
    u = _dev(SI.random_local(m.n_local, 9))
    w = _fused(m, u)  # the two launches run
    assert _same_bits(w, _unfused(m, u))
    m.set_axgs_config(True)
    assert m.axgs_info()["enabled"] == 1
    with pytest.raises(semlib.SemError):
        m.set_axgs_config(True, 9, 0)  # 9 * 64 lanes > 512
    with pytest.raises(semlib.SemError):
        m.set_axgs_config(True, -1, 0)
    m.close()


def test_fused_helmholtz(semlib):
    print("case: fused helmholtz", flush=True)
    nel = (4, 3, 3)
    V = SI.jittered_box_vertices(nel, seed=4)
    m = semlib.box_mesh(7, nel, vertices=V, with_fp32=True)
    rng = np.random.default_rng(8)
    h1 = _dev(1.0 + rng.random(m.n_local))
    h2 = _dev(rng.random(m.n_local))
    m.set_helmholtz(h1, h2)
    for lines in (1, 3):
        m.set_axgs_config(True, 0, lines)
        u = _dev(SI.random_local(m.n_local, 31))
        for dt in (torch.float64, torch.float32):
            uu = u.to(dt)
            assert _same_bits(_fused(m, uu), _unfused(m, uu)), (lines, dt)
    m.close()


@pytest.mark.parametrize("lines", [1, 2, 5])
def test_fused_cg_solves(semlib, oracle_mod, lines):
    """FP64 and mixed solves whose CG iterations run the fused operator reach
    the oracle's true residual; iteration counts match the two-launch path to
    within rounding drift (the dot partials follow the workgroups)."""
    nel = (4, 4, 4)
    print(f"case: fused cg lines={lines}", flush=True)
    V = SI.jittered_box_vertices(nel, seed=1)
    m = semlib.box_mesh(7, nel, vertices=V, with_fp32=True)
    om = oracle_mod.OracleMesh(7, nel, vertices=V)
    x, y, z = om.coords()
    b = om.mass(SI.sin3_forcing(x, y, z))
    bd = _dev(b)
    its = {}
    for fused in (True, False):
        m.set_axgs_config(fused, 0, lines if fused else 0)
        for prec in ("fp64", "mixed"):
            xs, res = m.solve(bd, tol=1e-10, precision=prec)
            rel = om.true_residual(b, xs.cpu().numpy())
            assert res.ok and rel <= 1e-10, (fused, prec, res, rel)
            its[(fused, prec)] = res.iterations
    for prec in ("fp64", "mixed"):
        assert abs(its[(True, prec)] - its[(False, prec)]) <= max(2, its[(False, prec)] // 50), its
    m.close()


def test_fused_graph_replays_match_eager(semlib):
    """Fixed-count CG runs through the fused path: graph replays and eager
    launches give the same bits."""
    nel = (4, 4, 4)
    print("case: fused graph vs eager", flush=True)
    V = SI.jittered_box_vertices(nel, seed=1)
    m = semlib.box_mesh(7, nel, vertices=V)
    m.set_axgs_config(True, 0, 3)
    b = m.scatter(_dev(np.random.default_rng(3).uniform(-1, 1, m.n_global)))
    xs = []
    for graph in (True, False, True):
        x, res = m.solve(b, tol=1e-30, max_iter=40, fixed_iters=40, use_graph=graph, poll_every=8,
                         raise_on_error=False)
        xs.append(x.clone())
    assert torch.equal(xs[0], xs[1]) and torch.equal(xs[0], xs[2])
    m.close()


def test_fused_pipe_full_size(semlib):
    """The 48x48x96 pipe at N = 7 in the shape the bench times: the fused
    apply is the same bits as operator + gather-scatter, FP64 and FP32."""
    print("case: fused pipe 48x48x96 N=7", flush=True)
    m = semlib.pipe_mesh(48, 48, 96, 7, with_fp32=True)
    m.set_axgs_config(True, 4, 9)
    info = m.axgs_info()
    assert info["enabled"] == 1 and info["y_onchip"] == 1 and info["lines_per_wg"] == 9
    print(f"shape {info}", flush=True)
    u = torch.empty(m.n_local, dtype=torch.float64, device="cuda")
    g = torch.Generator(device="cuda").manual_seed(5)
    u.uniform_(-1.0, 1.0, generator=g)
    for dt in (torch.float64, torch.float32):
        uu = u.to(dt)
        wf = _fused(m, uu)
        wu = _unfused(m, uu)
        assert _same_bits(wf, wu), dt
        del wf, wu, uu
    m.close()
