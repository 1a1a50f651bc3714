"""The lattice gather-scatter (no plan read) against the CSR plan and the
oracle, through the C ABI.

Bar: bit-exact.  The lattice kernel sums a node's copies in ascending local
index from 0, as the plan does, so FP64 and FP32 results must be the same
bits as the plan's, signed zeros included (an unmasked node with a single
copy is left untouched by both); FP64 results must equal the oracle's
assembled sum on inputs without negative zeros.  Meshes span every
periodicity pattern, Dirichlet face subsets (none, some, all), one element
along a non-periodic axis, orders 1 to 12, and the pipe map; a periodic axis
of one element takes the plan (the lattice kernel declines it).  The
"stream" kind runs the row-streaming kernel for the nodes off the z-planes
at every order 2 to 7 (the default kind only on large order-7 meshes), so
these cases check it against the plan, bit for bit, on every periodicity
and Dirichlet set.
"""
import numpy as np
import pytest
import torch

import seeded_inputs as SI

pytestmark = pytest.mark.gpu

CASES = [
    # N, nel, periodic, dirichlet faces (-1: every non-periodic face)
    (1, (2, 2, 2), (0, 0, 0), -1),
    (2, (3, 2, 4), (1, 0, 0), -1),
    (3, (1, 2, 2), (0, 1, 0), -1),
    (4, (2, 3, 2), (1, 1, 1), -1),
    (5, (1, 1, 3), (0, 0, 0), 0),
    (6, (3, 3, 2), (0, 0, 0), 0b000101),
    (7, (4, 3, 5), (0, 0, 1), 0b001010),
    (7, (2, 2, 2), (1, 0, 1), 0b001100),
    (9, (2, 3, 2), (0, 1, 1), -1),
    (12, (2, 2, 2), (0, 0, 1), -1),
]


def _bits(t):
    torch.cuda.synchronize()
    a = t.detach().cpu().numpy()
    return a.view(np.uint64 if a.dtype == np.float64 else np.uint32)


def _with_signed_zeros(v, seed):
    rng = np.random.default_rng(seed)
    v = v.copy()
    v[rng.random(v.size) < 0.05] = -0.0
    v[rng.random(v.size) < 0.02] = 0.0
    return v


def _mesh(semlib, N, nel, per, faces, pipe=False):
    if pipe:
        return semlib.pipe_mesh(*nel, N=N, with_fp32=True)
    V = SI.jittered_box_vertices(nel, seed=N)
    return semlib.box_mesh(N, nel, vertices=V, periodic=per, dirichlet_faces=faces, with_fp32=True)


def _check_against_plan(m, v):
    for dt in (torch.float64, torch.float32):
        src = torch.from_numpy(v).to(device="cuda", dtype=dt)
        m.set_gs_kind("plan")
        ref = _bits(m.gs(src.clone()))
        for kind in ("auto", "stream"):
            m.set_gs_kind(kind)
            got = _bits(m.gs(src.clone()))
            assert np.array_equal(got, ref), (dt, kind, int(np.count_nonzero(got != ref)))
        m.set_gs_kind("auto")


@pytest.mark.parametrize("N,nel,per,faces", CASES)
def test_lattice_gs_bit_exact(semlib, oracle_mod, N, nel, per, faces):
    print(f"case: lattice gs N={N} nel={nel} periodic={per} faces={faces}", flush=True)
    m = _mesh(semlib, N, nel, per, faces)
    try:
        assert m.gs_kind() == ("auto", True)
        n = m.info.n_local
        _check_against_plan(m, _with_signed_zeros(SI.random_local(n, 40 + N), N))
        om = oracle_mod.OracleMesh(N, nel, vertices=SI.jittered_box_vertices(nel, seed=N), periodic=per,
                                   dirichlet=None if faces < 0 else faces)
        gid, mult, mask = m.export_maps()
        assert np.array_equal(gid, om.numbering()) and np.array_equal(mask, om.local_mask())
        v = SI.random_local(n, 60 + N)
        got = m.gs(torch.from_numpy(v).cuda()).cpu().numpy()
        assert np.array_equal(got, om.gs(v))
    finally:
        m.close()


def test_lattice_gs_pipe_and_solve(semlib, oracle_mod):
    """Pipe map (periodic z, Dirichlet wall): bit-exact with the plan and the
    oracle; a solve with either kernel takes the same iterations and returns
    the same bits (the CG sums do not depend on which kernel summed)."""
    print("case: lattice gs pipe 6x6x4 N=7", flush=True)
    m = _mesh(semlib, 7, (6, 6, 4), None, None, pipe=True)
    om = oracle_mod.pipe_mesh(6, 6, 4, N=7)
    try:
        assert m.gs_kind() == ("auto", True)
        n = m.info.n_local
        _check_against_plan(m, _with_signed_zeros(SI.random_local(n, 71), 7))
        v = SI.random_local(n, 72)
        assert np.array_equal(m.gs(torch.from_numpy(v).cuda()).cpu().numpy(), om.gs(v))
        gid = om.numbering()
        b = SI.uniform_global_values(om.nglob, 3)[gid]
        b[om.local_mask() == 1] = 0.0
        bd = torch.from_numpy(b).cuda()
        out = {}
        for kind in ("plan", "auto", "stream"):
            m.set_gs_kind(kind)
            for prec in ("fp64", "mixed"):
                x, res = m.solve(bd, tol=1e-10, max_iter=5000, precision=prec)
                assert res.ok
                out[kind, prec] = (_bits(x), res.iterations)
        m.set_gs_kind("auto")
        for kind in ("auto", "stream"):
            for prec in ("fp64", "mixed"):
                assert out["plan", prec][1] == out[kind, prec][1]
                assert np.array_equal(out["plan", prec][0], out[kind, prec][0]), (kind, prec)
        assert om.true_residual(b, out["auto", "fp64"][0].view(np.float64)) <= 1e-10
    finally:
        m.close()


def test_lattice_gs_declines_single_periodic_element(semlib):
    """A periodic axis of one element puts two copies of a node in the same
    element: the plan runs, with the same results."""
    print("case: lattice gs declined, nel_z = 1 periodic", flush=True)
    m = _mesh(semlib, 4, (2, 2, 1), (0, 0, 1), -1)
    try:
        assert m.gs_kind() == ("auto", False)
        _check_against_plan(m, SI.random_local(m.info.n_local, 5))
    finally:
        m.close()


def test_gs_kind_validation(semlib):
    m = _mesh(semlib, 3, (2, 2, 2), (0, 0, 0), -1)
    try:
        with pytest.raises(ValueError):
            m.set_gs_kind("atomic")
        m.set_gs_kind("plan")
        assert m.gs_kind() == ("plan", False)
        m.set_gs_kind("stream")
        assert m.gs_kind() == ("stream", True)
        m.set_gs_kind("auto")
        assert m.gs_kind() == ("auto", True)
    finally:
        m.close()


def test_batched_slots_lattice_vs_plan(semlib, oracle_mod):
    """Batched slots sum with the lattice kernel when their mesh does: the same
    bits as with the plan, FP64 and mixed, and the oracle's true residual."""
    print("case: batched slots, lattice vs plan gather-scatter", flush=True)
    cases = []
    for N, nel, per in ((5, (3, 4, 2), (0, 0, 0)), (7, (2, 3, 4), (0, 0, 1)), (9, (2, 2, 2), (1, 0, 0))):
        V = None if any(per) else SI.jittered_box_vertices(nel, seed=N)
        m = semlib.box_mesh(N, nel, vertices=V, periodic=per, with_fp32=True)
        om = oracle_mod.OracleMesh(N, nel, vertices=V, periodic=per)
        b = SI.uniform_global_values(om.nglob, 50 + N)[om.numbering()]
        b[om.local_mask() == 1] = 0.0
        cases.append((m, om, b))
    B = semlib.Batch(max_slots=8)
    try:
        meshes = [c[0] for c in cases]
        bs = [torch.from_numpy(c[2]).cuda() for c in cases]
        for prec in ("fp64", "mixed"):
            out = {}
            for kind in ("auto", "plan"):
                for m in meshes:
                    m.set_gs_kind(kind)
                xs, res = B.solve(meshes, bs, tol=1e-10, precision=prec)
                out[kind] = (xs, [r.iterations for r in res])
            assert out["auto"][1] == out["plan"][1], prec
            for (m, om, b), xa, xp in zip(cases, out["auto"][0], out["plan"][0]):
                assert torch.equal(xa, xp), (prec, m.N)
                assert om.true_residual(b, xa.cpu().numpy()) <= 1e-10
    finally:
        for m in meshes:
            m.set_gs_kind("auto")
        B.close()
        for m, _, _ in cases:
            m.close()
