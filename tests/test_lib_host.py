"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
and its host-side set-up (GLL rule, geometry, numbering, gather-scatter plan,
Jacobi diagonal) agrees with the oracle.  No compute call touches a GPU."""
import ctypes as C

import numpy as np
import pytest

import seeded_inputs as SI
from libhost import apply_plan, header_functions, host_setup, make_desc


@pytest.fixture(scope="module")
def L():
    from paper_2109_03592_amd import _lib
    _lib.load()
    return _lib


def test_every_declared_symbol_is_exported(L):
    names = header_functions()
    assert len(names) >= 15
    lib = L.load()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares exactly the header's functions
    assert sorted(L.SIGNATURES) == names


def test_version_and_error_text(L):
    lib = L.load()
    assert b"gfx950" in lib.sem_version()
    d, _ = make_desc(L, 0, (1, 1, 1))
    info = L.MeshInfo()
    st = lib.sem_host_setup(C.byref(d), C.byref(info), *([None] * 8))
    assert st == L.SEM_EINVAL
    assert b"N must be" in lib.sem_last_error()
    d, _ = make_desc(L, 3, (0, 1, 1))
    assert lib.sem_host_setup(C.byref(d), C.byref(info), *([None] * 8)) == L.SEM_EINVAL
    d, _ = make_desc(L, 3, (1, 1, 1), lo=(0, 0, 0), hi=(0, 1, 1))
    assert lib.sem_host_setup(C.byref(d), C.byref(info), *([None] * 8)) == L.SEM_EINVAL
    d, _ = make_desc(L, 3, (1, 1, 1), mapping=7)
    assert lib.sem_host_setup(C.byref(d), C.byref(info), *([None] * 8)) == L.SEM_EINVAL
    # a null descriptor is an error, not a crash
    assert lib.sem_host_setup(None, None, *([None] * 8)) == L.SEM_EINVAL
    assert lib.sem_info(None, None) == L.SEM_EINVAL
    assert lib.sem_set_helmholtz(None, None, None, None) == L.SEM_EINVAL


def test_inverted_element_rejected(L):
    # swap two vertex layers so one element is inside out
    nel = (1, 1, 1)
    V = SI.jittered_box_vertices(nel, amp=0.0)
    V = V.reshape(2, 2, 2, 3)[:, :, ::-1, :].reshape(-1, 3)
    d, keep = make_desc(L, 2, nel, vertices=V)
    info = L.MeshInfo()
    assert L.load().sem_host_setup(C.byref(d), C.byref(info), *([None] * 8)) == L.SEM_EINVAL


@pytest.mark.parametrize("N", list(range(1, 18)))
def test_gll_matches_oracle(L, oracle_mod, N):
    xi, w, D = (np.zeros(N + 1), np.zeros(N + 1), np.zeros((N + 1, N + 1)))
    L.check(L.load().sem_export_gll(N, xi.ctypes.data, w.ctypes.data, D.ctypes.data), "gll")
    xo, wo = oracle_mod.gll(N)
    Do = oracle_mod.deriv(N, xo)
    np.testing.assert_allclose(xi, xo, atol=2e-16 * 4)
    np.testing.assert_allclose(w, wo, rtol=2e-14)
    np.testing.assert_allclose(D, Do, atol=5e-14 * N * N)


def _cases(oracle_mod):
    nel = (4, 4, 4)
    V = SI.jittered_box_vertices(nel, seed=1)
    yield "box4_N7", dict(N=7, nel=nel, vertices=V), oracle_mod.OracleMesh(7, nel, vertices=V)
    nel = (3, 2, 5)
    V = SI.jittered_box_vertices(nel, lo=(0, 0, 0), hi=(1.5, 1.0, 2.0), seed=2)
    yield "box_per_z_N5", dict(N=5, nel=nel, vertices=V, hi=(1.5, 1.0, 2.0), periodic=(0, 0, 1)), \
        oracle_mod.OracleMesh(5, nel, hi=(1.5, 1.0, 2.0), periodic=(0, 0, 1), vertices=V)
    nel = (2, 3, 2)
    yield "box_neumann_x_N4", dict(N=4, nel=nel, dirichlet=0b111100), \
        oracle_mod.OracleMesh(4, nel, dirichlet=0b111100)
    nel = (6, 6, 4)
    yield "pipe_N7", dict(N=7, nel=nel, periodic=(0, 0, 1), lo=(-1, -1, 0), hi=(1, 1, 10), mapping=1), \
        oracle_mod.pipe_mesh(*nel, N=7)
    nel = (4, 4, 3)
    yield "pipe_N9", dict(N=9, nel=nel, periodic=(0, 0, 1), lo=(-1, -1, 0), hi=(1, 1, 10), mapping=1), \
        oracle_mod.pipe_mesh(*nel, N=9)
    nel = (2, 2, 1)
    yield "periodic_all_N3", dict(N=3, nel=nel, periodic=(1, 1, 1)), \
        oracle_mod.OracleMesh(3, nel, periodic=(1, 1, 1))


def test_host_maps_bit_exact(oracle_mod):
    for name, kw, om in _cases(oracle_mod):
        h = host_setup(**kw)
        assert h["info"].n_global == om.nglob, name
        np.testing.assert_array_equal(h["gid"], om.numbering(), err_msg=name)
        np.testing.assert_array_equal(h["mult"], om.local_mult(), err_msg=name)
        np.testing.assert_array_equal(h["mask"], om.local_mask(), err_msg=name)
        gm = om.global_mult()
        assert h["info"].n_shared_global == int(np.sum(gm >= 2)), name
        assert h["info"].n_shared_local == int(np.sum(gm[gm >= 2])), name
        assert h["info"].n_masked_global == int(om.global_mask().sum()), name


def test_host_geometry_matches_oracle(oracle_mod):
    for name, kw, om in _cases(oracle_mod):
        h = host_setup(**kw)
        G, B = om.geom()
        # boxes: norm-wise 1e-13.  Pipes: next to the map's singular corners det J is
        # small and the factors are ill-conditioned functions of the node coordinates,
        # so two correct FP64 evaluations differ by more (see the extended-precision test)
        tol = 1e-10 if name.startswith("pipe") else 1e-13
        assert np.linalg.norm(h["G"] - G) <= tol * np.linalg.norm(G), name
        np.testing.assert_array_equal(h["G"][:, B == 0], 0.0)
        assert np.max(np.abs(h["B"] - B)) <= 1e-13 * np.abs(B).max(), name
        inv = om.jacobi()
        assert np.max(np.abs(h["inv"] - inv)) <= 1e-12 * np.abs(inv).max(), name
        np.testing.assert_array_equal(h["inv"] == 0, inv == 0)


def test_gs_plan_reproduces_oracle_bit_exact(oracle_mod):
    for name, kw, om in _cases(oracle_mod):
        h = host_setup(**kw)
        info = h["info"]
        off, idx = h["off"], h["idx"]
        # plan structure: ids ascending, copies ascending, every shared or masked node listed once
        gid = h["gid"]
        ids = gid[idx[off[:-1]]]
        assert np.all(np.diff(ids[:info.gs_plan_sum_ids]) > 0)
        assert np.all(np.diff(ids[info.gs_plan_sum_ids:]) > 0)
        for a, b in zip(off[:-1][:50], off[1:][:50]):
            seg = idx[a:b]
            assert np.all(np.diff(seg) > 0) and np.all(gid[seg] == gid[seg[0]])
        assert len(np.unique(idx)) == len(idx) == info.gs_plan_len
        v = SI.random_local(om.nloc, 77)
        got = apply_plan(v, off, idx, info.gs_plan_sum_ids)
        ref = om.gs(v)
        assert np.array_equal(got, ref), name


@pytest.mark.slow
def test_host_maps_pipe_full_size(oracle_mod):
    """48x48x96 pipe at N=7: maps bit-exact and plan sizes against the closed form."""
    kw = dict(N=7, nel=(48, 48, 96), periodic=(0, 0, 1), lo=(-1, -1, 0), hi=(1, 1, 10), mapping=1)
    from paper_2109_03592_amd import _lib as L
    d, _ = make_desc(L, **kw)
    info = L.MeshInfo()
    n = 48 * 48 * 96 * 512
    gid = np.zeros(n, np.int64)
    L.check(L.load().sem_host_setup(C.byref(d), C.byref(info), gid.ctypes.data, *([None] * 7)), "host")
    assert info.n_global == 337 * 337 * 672
    assert info.n_shared_local == 64804608 and info.n_shared_global == 27876768
    assert info.n_unmasked_global == 335 * 335 * 672
    om = oracle_mod.pipe_mesh(48, 48, 96, N=7)
    assert np.array_equal(gid, om.numbering())


def _slot_layout(lib, n_local, precision):
    off = np.zeros(7, dtype=np.uint64)
    total = C.c_size_t(0)
    st = lib.sem_batch_slot_layout(C.c_int64(n_local), precision, off.ctypes.data, C.byref(total))
    return st, off.astype(np.int64), int(total.value)


def test_batch_slot_layout_holds_every_vector(L):
    """Every vector a batch slot carves from its buffer lies inside the
    allocation, 256-byte aligned and disjoint from the others, for every
    order the batch takes (2..10) and element counts 1..4096."""
    lib = L.load()
    Es = sorted(set([1, 2, 3, 5, 7, 8, 27, 63, 64, 100, 343, 511, 512, 729, 1000, 2047, 4095, 4096]
                    + list(np.random.default_rng(5).integers(1, 4097, 60))))
    for N in range(2, 11):
        P3 = (N + 1) ** 3
        for E in Es:
            nL = int(E) * P3
            for prec, sizes in ((L.SEM_PREC_FP64, [8, 8, 8]), (L.SEM_PREC_MIXED, [8, 8, 8, 4, 4, 4, 4])):
                st, off, total = _slot_layout(lib, nL, prec)
                assert st == L.SEM_OK
                spans = sorted((int(off[q]), int(off[q]) + nL * sz) for q, sz in enumerate(sizes))
                for a, b in spans:
                    assert a % 256 == 0 and b <= total, (N, E, prec, a, b, total)
                for (a0, b0), (a1, b1) in zip(spans, spans[1:]):
                    assert b0 <= a1, (N, E, prec)
                if prec == L.SEM_PREC_FP64:
                    assert not off[3:].any()


def test_batch_slot_layout_rejects_bad_arguments(L):
    lib = L.load()
    assert _slot_layout(lib, 0, L.SEM_PREC_FP64)[0] == L.SEM_EINVAL
    assert _slot_layout(lib, 64, 7)[0] == L.SEM_EINVAL
    total = C.c_size_t(0)
    assert lib.sem_batch_slot_layout(C.c_int64(64), L.SEM_PREC_FP64, None, C.byref(total)) == L.SEM_EINVAL
