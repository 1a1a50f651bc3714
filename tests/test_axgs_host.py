"""CPU tests of the fused operator's residual plan (host logic only).

The fused kernel sums a shared node itself when every copy of it lies on an
interior t-plane (0 < k < N) of elements that one workgroup walks (whole
x-lines, lines_per_wg consecutive lines) and it does not sit on a periodic x-
or y-seam; Dirichlet nodes are zeroed by each copy.  Every other shared node
must be in the residual plan.  This test derives that set from each node's
copies (element, i, j, k) -- independently of the library's lattice-index rule
-- and compares it with the exported plan, which must also keep the full
plan's ascending-local-index order of copies.
"""
import ctypes as C

import numpy as np
import pytest

from libhost import host_setup, make_desc


def _residual(L, N, nel, lines, y_onchip, **kw):
    lib = L.load()
    d, keep = make_desc(L, N, nel, **kw)
    n_ids, n_cp = C.c_int64(0), C.c_int64(0)
    L.check(lib.sem_host_axgs_residual(C.byref(d), lines, y_onchip, C.byref(n_ids), C.byref(n_cp), None, None),
            "sem_host_axgs_residual")
    off = np.zeros(n_ids.value + 1, np.int32)
    idx = np.zeros(n_cp.value, np.int32)
    L.check(lib.sem_host_axgs_residual(C.byref(d), lines, y_onchip, C.byref(n_ids), C.byref(n_cp),
                                       off.ctypes.data, idx.ctypes.data), "sem_host_axgs_residual")
    del keep
    return off, idx


def _expected(N, nel, periodic, lines, y_onchip, hs):
    """Residual ids from the copies of each summed id of the full plan."""
    P = N + 1
    nx, ny, nz = nel
    off, idx = hs["off"], hs["idx"]
    n_sum = hs["info"].gs_plan_sum_ids
    keep = []
    for t in range(n_sum):
        loc = idx[off[t]:off[t + 1]]
        e, p = loc // P ** 3, loc % P ** 3
        i, j, k = p % P, (p // P) % P, p // (P * P)
        ex, line = e % nx, e // nx
        ey = line % ny
        on = True
        if np.any((k == 0) | (k == N)):
            on = False                      # a t-plane k = 0, N
        if np.unique(line // lines).size > 1:
            on = False                      # copies in two workgroups
        if not y_onchip and np.unique(line).size > 1:
            on = False                      # y-faces not summed in LDS
        if periodic[0] and np.any((ex == 0) & (i == 0)) and np.any((ex == nx - 1) & (i == N)):
            on = False                      # the periodic x seam
        if periodic[1] and np.any((ey == 0) & (j == 0)) and np.any((ey == ny - 1) & (j == N)):
            on = False                      # the periodic y seam
        if not on:
            keep.append(t)
    return keep


CASES = [
    (7, (4, 4, 4), (0, 0, 0), 1, 1),
    (7, (4, 4, 4), (0, 0, 0), 3, 1),
    (7, (4, 4, 4), (0, 0, 0), 3, 0),
    (5, (5, 3, 4), (0, 0, 1), 2, 1),
    (4, (6, 5, 3), (1, 0, 0), 4, 1),
    (3, (3, 4, 5), (0, 1, 0), 6, 1),
    (2, (4, 4, 3), (1, 1, 1), 5, 1),
    (6, (2, 1, 3), (1, 1, 0), 2, 1),
    (1, (3, 3, 3), (0, 0, 0), 2, 1),
    (3, (5, 4, 2), (0, 0, 0), 1000, 1),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_residual_plan_is_the_set_not_finished_in_lds(case):
    from paper_2109_03592_amd import _lib as L
    N, nel, per, lines, yon = CASES[case]
    hs = host_setup(N, nel, periodic=per)
    off, idx = _residual(L, N, nel, lines, yon, periodic=per)
    keep = _expected(N, nel, per, lines, yon, hs)
    # same ids (in order), each with the full plan's copies in the same order
    fo, fi = hs["off"], hs["idx"]
    assert len(off) - 1 == len(keep)
    for r, t in enumerate(keep):
        assert np.array_equal(idx[off[r]:off[r + 1]], fi[fo[t]:fo[t + 1]]), (r, t)
    # on-chip ids exist whenever interior t-planes and shared x-faces exist
    if N >= 2 and nel[0] >= 2:
        assert len(keep) < hs["info"].gs_plan_sum_ids


def test_residual_plan_sizes_on_the_pipe_slab():
    """A 48x48x4 slab of the pipe at N = 7 with nine lines per workgroup: the
    residual holds the t-planes and one y-face in nine."""
    from paper_2109_03592_amd import _lib as L
    nel = (48, 48, 4)
    off, idx = _residual(L, 7, nel, 9, 1, periodic=(0, 0, 1), lo=(-1, -1, 0), hi=(1, 1, 10.0 * 4 / 96),
                         mapping=1)
    hs = host_setup(7, nel, periodic=(0, 0, 1), lo=(-1, -1, 0), hi=(1, 1, 10.0 * 4 / 96), mapping=1)
    n_sum = hs["info"].gs_plan_sum_ids
    frac = (len(off) - 1) / n_sum
    assert 0.2 < frac < 0.6, frac


def test_residual_rejects_bad_arguments():
    from paper_2109_03592_amd import _lib as L
    lib = L.load()
    d, _ = make_desc(L, 3, (2, 2, 2))
    a, b = C.c_int64(0), C.c_int64(0)
    assert lib.sem_host_axgs_residual(C.byref(d), 0, 1, C.byref(a), C.byref(b), None, None) == L.SEM_EINVAL
    assert lib.sem_host_axgs_residual(C.byref(d), 1, 2, C.byref(a), C.byref(b), None, None) == L.SEM_EINVAL
    assert lib.sem_host_axgs_residual(None, 1, 1, C.byref(a), C.byref(b), None, None) == L.SEM_EINVAL
