"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Bars: bit-exact for index maps, multiplicities and the gather-scatter on
identical input; FP64 operator within 1e-12 relative (norm-wise and max-norm);
solves reach a true relative residual <= 1e-10 measured by the oracle.
"""
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
    n = np.linalg.norm(b)
    return np.linalg.norm(a - b) / n, np.max(np.abs(a - b)) / np.max(np.abs(b))


def _box(semlib, oracle_mod, N, nel, seed=1, **kw):
    V = SI.jittered_box_vertices(nel, seed=seed)
    m = semlib.box_mesh(N, nel, vertices=V, **kw)
    om = oracle_mod.OracleMesh(N, nel, vertices=V,
                               periodic=kw.get("periodic", (0, 0, 0)))
    return m, om


def test_box_config_maps_and_geometry(semlib, oracle_mod):
    print("case: box 4x4x4 N=7 maps", flush=True)
    m, om = _box(semlib, oracle_mod, 7, (4, 4, 4), with_fp32=True)
    gid, mult, mask = m.export_maps()
    assert np.array_equal(gid, om.numbering())
    assert np.array_equal(mult, om.local_mult())
    assert np.array_equal(mask, om.local_mask())
    G, B, inv = m.export_geom()
    Go, Bo = om.geom()
    assert np.linalg.norm(G - Go) <= 1e-13 * np.linalg.norm(Go)
    assert np.max(np.abs(B - Bo)) <= 1e-13 * np.abs(Bo).max()
    invo = om.jacobi()
    assert np.max(np.abs(inv - invo)) <= 1e-12 * np.abs(invo).max()
    assert m.info.n_global == 29 ** 3 and m.info.n_unmasked_global == 27 ** 3


def _nel_for(N):
    return (3, 2, 3) if N <= 9 else ((2, 2, 2) if N <= 12 else (2, 1, 2))


def _order_scale(N):
    """Growth with the order of the difference between two FP64 evaluations
    that start from differently rounded geometric factors: the factors come
    from differentiating node coordinates with D, whose entries grow like N^2
    (|D_00| = N(N+1)/4), and each output sums 3(N+1) products with D again;
    the tolerances on each side's own geometry hold up to N = 12 and are
    scaled by ((N+1)/13)^2 beyond.  The operator's own rounding stays within
    the unscaled bar (the extended-precision test below), and on identical
    factors so does its difference from the oracle."""
    return max(1.0, ((N + 1) / 13.0) ** 2)


@pytest.mark.parametrize("N", list(range(1, 18)))
def test_ax_fp64_all_orders(semlib, oracle_mod, N):
    """Ragged element counts (not a multiple of the elements per workgroup).
    On the library's own geometry the result differs from the oracle's by the
    two FP64 geometries' rounding, which grows with the order (the factors
    come from differentiating coordinates with D, |D| ~ N^2); on the oracle's
    factors, loaded through sem_load_geometry, the 1e-12 bar holds at every
    order."""
    nel = _nel_for(N)
    print(f"case: ax fp64 N={N} nel={nel}", flush=True)
    m, om = _box(semlib, oracle_mod, N, nel, seed=N)
    u = SI.random_local(om.nloc, 100 + N)
    ref = om.ax(u)
    e2, einf = _relerr(_host(m.ax(_dev(u))), ref)
    tol = 1e-12 * _order_scale(N)
    assert e2 <= tol and einf <= tol, (e2, einf)
    m.load_geometry(*om.geom())
    e2, einf = _relerr(_host(m.ax(_dev(u))), ref)
    assert e2 <= 1e-12 and einf <= 1e-12, (e2, einf)


def _ax_extended(N, D, G, u, E):
    """A_L u in 80-bit extended precision from the library's own FP64 D and
    factors (exact inputs): the reference against which the rounding of the
    FP64 operator itself is measured."""
    LD = np.longdouble
    P = N + 1
    P3 = P ** 3
    D = D.astype(LD)
    out = np.zeros(E * P3, dtype=LD)
    for e in range(E):
        U = u[e * P3:(e + 1) * P3].astype(LD).reshape(P, P, P)  # [k, j, i]
        g = G[:, e * P3:(e + 1) * P3].astype(LD).reshape(6, P, P, P)
        ur = np.einsum("il,kjl->kji", D, U)
        us = np.einsum("jl,kli->kji", D, U)
        ut = np.einsum("kl,lji->kji", D, U)
        fr = g[0] * ur + g[3] * us + g[4] * ut
        fs = g[3] * ur + g[1] * us + g[5] * ut
        ft = g[4] * ur + g[5] * us + g[2] * ut
        w = (np.einsum("li,kjl->kji", D, fr) + np.einsum("lj,kli->kji", D, fs)
             + np.einsum("lk,lji->kji", D, ft))
        out[e * P3:(e + 1) * P3] = w.reshape(-1)
    return out


@pytest.mark.parametrize("N", [2, 7, 12, 13, 15, 17])
def test_ax_fp64_against_extended_precision(semlib, N):
    """The rounding of the FP64 operator itself, measured against an 80-bit
    evaluation on identical inputs (the library's D and factors): within the
    1e-12 bar at every order up to the LDS limit, so the order-scaled
    tolerance of the comparisons on the library's own geometry covers the
    two geometries' rounding, not the operator's."""
    nel = _nel_for(N)
    print(f"case: ax fp64 vs extended precision N={N} nel={nel}", flush=True)
    V = SI.jittered_box_vertices(nel, seed=N)
    m = semlib.box_mesh(N, nel, vertices=V)
    _, _, D = semlib.export_gll(N)
    G, _, _ = m.export_geom()
    u = SI.random_local(m.n_local, 100 + N)
    w = _host(m.ax(_dev(u)))
    ref = _ax_extended(N, D, G, u, m.E)
    d = (w.astype(np.longdouble) - ref)
    e2 = float(np.sqrt(np.sum(d * d) / np.sum(ref * ref)))
    einf = float(np.max(np.abs(d)) / np.max(np.abs(ref)))
    print(f"  N={N}: {e2:.2e} norm-wise, {einf:.2e} max-norm", flush=True)
    assert e2 <= 1e-12 and einf <= 1e-12, (e2, einf)
    m.close()


@pytest.mark.parametrize("N", list(range(1, 18)))
def test_ax_fp32_all_orders(semlib, oracle_mod, N):
    """FP32 operator (geometric factors rounded to FP32) at every order against
    the oracle applied to the FP32-rounded input: the error is FP32 rounding
    of O(N) operations per output."""
    nel = _nel_for(N)
    print(f"case: ax fp32 N={N} nel={nel}", flush=True)
    m, om = _box(semlib, oracle_mod, N, nel, seed=N, with_fp32=True)
    u32 = SI.random_local(om.nloc, 200 + N).astype(np.float32)
    w = _host(m.ax(_dev(u32, torch.float32)))
    ref = om.ax(u32.astype(np.float64))
    e2, einf = _relerr(w, ref)
    sc = _order_scale(N)
    assert e2 <= 2e-6 * sc and einf <= 2e-5 * sc, (e2, einf)


@pytest.mark.parametrize("N,nel", [(8, (2, 2, 2)), (9, (2, 2, 2)), (10, (2, 1, 2)), (12, (1, 2, 1)),
                                   (14, (2, 1, 1)), (17, (1, 2, 1))])
def test_pcg_high_order(semlib, oracle_mod, N, nel):
    """CG at the orders whose operator reads D rows from LDS."""
    print(f"case: pcg fp64 + mixed box N={N} nel={nel}", flush=True)
    m, om = _box(semlib, oracle_mod, N, nel, seed=30 + N, with_fp32=True)
    x, y, z = om.coords()
    b = om.mass(SI.sin3_forcing(x, y, z))
    _, ro = om.pcg(b, tol=1e-10)
    for prec in ("fp64", "mixed"):
        xg, res = m.solve(_dev(b), tol=1e-10, precision=prec)
        assert res.ok, (prec, res)
        assert om.true_residual(b, _host(xg)) <= 1e-10, (prec, res)
        if prec == "fp64":
            assert abs(res.iterations - ro.iterations) <= max(3, 0.05 * ro.iterations), (res, ro)


@pytest.mark.parametrize("N,epws", [(5, (1, 3, 7, 14)), (7, (1, 2, 4, 8)), (9, (1, 2, 5)), (3, (1, 4, 32))])
def test_operator_config_does_not_change_results(semlib, oracle_mod, N, epws):
    """Elements per workgroup (up to 512 lanes) change the launch, not the
    bits of A_L u; a configuration beyond the lane limit is refused."""
    nel = (5, 3, 2)
    print(f"case: operator configs N={N} epw={epws}", flush=True)
    m, om = _box(semlib, oracle_mod, N, nel, seed=3 + N)
    u = _dev(SI.random_local(om.nloc, 70 + N))
    outs = []
    for e in epws:
        m.set_operator_config(e, 0)
        assert m.operator_config()[0] == e
        outs.append(_host(m.ax(u)))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    e2, _ = _relerr(outs[0], om.ax(_host(u)))
    assert e2 <= 1e-12
    with pytest.raises(semlib.SemError):
        m.set_operator_config(512 // (N + 1) ** 2 + 1, 0)


def test_ax_dot_and_fp32(semlib, oracle_mod):
    print("case: ax dot + fp32, box 4x4x4 N=7", flush=True)
    m, om = _box(semlib, oracle_mod, 7, (4, 4, 4), with_fp32=True)
    u = SI.random_local(om.nloc, 5)
    w, dot = m.ax(_dev(u), dot=True)
    ref = om.ax(u)
    assert abs(float(dot.item()) - float(u @ ref)) <= 1e-12 * abs(float(u @ ref)) + 1e-12 * np.abs(u * ref).sum()
    w32 = _host(m.ax(_dev(u, torch.float32)))
    u32 = u.astype(np.float32).astype(np.float64)
    e2, einf = _relerr(w32, om.ax(u32))
    assert e2 <= 2e-6 and einf <= 2e-5, (e2, einf)


def test_gs_bit_exact(semlib, oracle_mod):
    for N, nel, per in ((7, (4, 4, 4), (0, 0, 0)), (5, (3, 2, 5), (0, 0, 1)), (3, (2, 2, 1), (1, 1, 1))):
        print(f"case: gs N={N} nel={nel} periodic={per}", flush=True)
        m, om = _box(semlib, oracle_mod, N, nel, periodic=per, with_fp32=True)
        v = SI.random_local(om.nloc, 9)
        got = _host(m.gs(_dev(v)))
        assert np.array_equal(got, om.gs(v))
        # FP32: same order, FP32 sums
        v32 = v.astype(np.float32)
        got32 = _host(m.gs(_dev(v32, torch.float32)))
        ref32 = om.gs(v32.astype(np.float64))
        assert np.max(np.abs(got32 - ref32)) <= 4e-7 * np.abs(ref32).max()


def test_axgs_mass_scatter(semlib, oracle_mod):
    print("case: axgs / mass / scatter, box 4x4x4 N=7", flush=True)
    m, om = _box(semlib, oracle_mod, 7, (4, 4, 4))
    u = SI.random_local(om.nloc, 11)
    w = _host(m.axgs(_dev(u)))
    e2, einf = _relerr(w, om.apply(u))
    assert e2 <= 1e-12 and einf <= 1e-12
    x, y, z = om.coords()
    f = SI.sin3_forcing(x, y, z)
    b = _host(m.mass(_dev(f)))
    bo = om.mass(f)
    assert np.max(np.abs(b - bo)) <= 1e-13 * np.abs(bo).max()
    vg = SI.uniform_global_values(om.nglob, 3)
    ul = _host(m.scatter(_dev(vg)))
    ref = vg[om.numbering()]
    ref[om.local_mask() == 1] = 0
    assert np.array_equal(ul, ref)


def test_pipe_small_operator(semlib, oracle_mod):
    print("case: pipe 6x6x4 N=7 axgs", flush=True)
    m = semlib.pipe_mesh(6, 6, 4, N=7)
    om = oracle_mod.pipe_mesh(6, 6, 4, N=7)
    gid, mult, mask = m.export_maps()
    assert np.array_equal(gid, om.numbering()) and np.array_equal(mask, om.local_mask())
    u = SI.random_local(om.nloc, 12)
    w = _host(m.axgs(_dev(u)))
    e2, einf = _relerr(w, om.apply(u))
    # the two geometries differ by rounding near the pipe's singular corners
    assert e2 <= 1e-11 and einf <= 1e-10, (e2, einf)


def test_pcg_box_config(semlib, oracle_mod):
    """4x4x4 jittered box, N=7, sin^3 forcing, Jacobi-PCG to 1e-10."""
    print("case: pcg fp64 box 4x4x4 N=7", flush=True)
    m, om = _box(semlib, oracle_mod, 7, (4, 4, 4), with_fp32=True)
    x, y, z = om.coords()
    b = om.mass(SI.sin3_forcing(x, y, z))
    uo, ro = om.pcg(b, tol=1e-10)
    xg, res = m.solve(_dev(b), tol=1e-10)
    xh = _host(xg)
    assert res.ok and res.rel_residual <= 1e-10
    assert om.true_residual(b, xh) <= 1e-10
    assert abs(res.iterations - ro.iterations) <= max(3, 0.05 * ro.iterations), (res.iterations, ro.iterations)
    assert np.linalg.norm(xh - uo) <= 1e-7 * np.linalg.norm(uo)
    # graph replay and plain launches give the same bits
    xg2, res2 = m.solve(_dev(b), tol=1e-10, use_graph=False)
    assert np.array_equal(_host(xg2), xh) and res2.iterations == res.iterations
    # mixed precision: FP32 inner, FP64 refinement
    print("case: pcg mixed box 4x4x4 N=7", flush=True)
    xm, rm = m.solve(_dev(b), tol=1e-10, precision="mixed")
    xmh = _host(xm)
    assert rm.ok and om.true_residual(b, xmh) <= 1e-10, rm
    assert np.linalg.norm(xmh - uo) <= 1e-7 * np.linalg.norm(uo)


def test_pcg_pipe_small(semlib, oracle_mod):
    print("case: pcg fp64 + mixed pipe 8x8x4 N=7", flush=True)
    m = semlib.pipe_mesh(8, 8, 4, N=7, with_fp32=True)
    om = oracle_mod.pipe_mesh(8, 8, 4, N=7)
    # the oracle's own factors: its residual is then measured on the operator solved
    m.load_geometry(*om.geom())
    vg = SI.uniform_global_values(om.nglob, 2)
    b = vg[om.numbering()]
    b[om.local_mask() == 1] = 0
    for prec in ("fp64", "mixed"):
        xg, res = m.solve(_dev(b), tol=1e-10, precision=prec, max_iter=20000)
        xh = _host(xg)
        assert res.ok, res
        assert om.true_residual(b, xh) <= 1e-10, (prec, res)
