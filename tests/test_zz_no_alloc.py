"""GPU test of sem_ax_noalloc, the operator entry point that allocates
nothing (its dot partials live in a fixed per-device array): through the C
ABI its outputs are the same bits as sem_ax with the dot product, on two calls
in a row -- the second on a smaller mesh, so the shared array holds the first
call's partials beyond the second's -- and it takes no device memory."""
import ctypes as C

import numpy as np
import pytest
import torch

import seeded_inputs as SI

pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _reference(m, u):
    w = torch.empty_like(u)
    dot = torch.zeros(1, dtype=torch.float64, device="cuda")
    from paper_2109_03592_amd import _lib as L
    L.check(L.load().sem_ax(m._h, m._dt(u), u.data_ptr(), w.data_ptr(), dot.data_ptr(),
                            torch.cuda.current_stream().cuda_stream), "sem_ax")
    torch.cuda.synchronize()
    return w, dot


def _noalloc(m, u):
    from paper_2109_03592_amd import _lib as L
    w = torch.full_like(u, float("nan"))
    dot = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    st = L.load().sem_ax_noalloc(m._h, m._dt(u), C.c_void_p(u.data_ptr()), C.c_void_p(w.data_ptr()),
                                 C.c_void_p(dot.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    L.check(st, "sem_ax_noalloc")
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    return w, dot, free0 - free1


def _bits(t):
    return t.view(torch.int64) if t.dtype == torch.float64 else t.view(torch.int32)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_sem_ax_on_two_calls(semlib, dtype):
    big = semlib.box_mesh(7, (12, 10, 9), vertices=SI.jittered_box_vertices((12, 10, 9), seed=3), with_fp32=True)
    small = semlib.box_mesh(5, (3, 2, 3), vertices=SI.jittered_box_vertices((3, 2, 3), seed=4), with_fp32=True)
    for name, m, seed in (("big", big, 21), ("small", small, 22)):
        print(f"case: noalloc {name} N={m.N} E={m.E} {dtype}", flush=True)
        u = _dev(SI.random_local(m.n_local, seed), dtype)
        wr, dr = _reference(m, u)  # first: loads the same kernels
        w, dot, took = _noalloc(m, u)
        assert torch.equal(_bits(w), _bits(wr)), name
        assert torch.equal(_bits(dot), _bits(dr)), (name, dot.item(), dr.item())
        assert took <= 0, f"device memory fell by {took} bytes"
    big.close()
    small.close()


def test_noalloc_rejects_a_grid_beyond_its_scratch(semlib):
    print("case: noalloc grid beyond scratch", flush=True)
    m = semlib.box_mesh(2, (40, 30, 20))  # 24000 elements, one per workgroup below
    m.set_operator_config(1, 20000)
    u = _dev(SI.random_local(m.n_local, 5))
    with pytest.raises(semlib.SemError, match="exceed"):
        m.ax_noalloc(u, torch.empty_like(u), torch.zeros(1, dtype=torch.float64, device="cuda"))
    m.set_operator_config(1, 4096)
    w, dot = m.ax_noalloc(u, torch.empty_like(u), torch.zeros(1, dtype=torch.float64, device="cuda"))
    wr, dr = _reference(m, u)
    assert torch.equal(_bits(w), _bits(wr)) and torch.equal(_bits(dot), _bits(dr))
    # the library's own argument checks (the binding is bypassed)
    from paper_2109_03592_amd import _lib as L
    lib = L.load()
    dot = torch.zeros(1, dtype=torch.float64, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.sem_ax_noalloc(m._h, L.SEM_FP64, C.c_void_p(u.data_ptr()), C.c_void_p(u.data_ptr()),
                              C.c_void_p(dot.data_ptr()), s) == L.SEM_EINVAL
    assert lib.sem_ax_noalloc(m._h, L.SEM_FP64, C.c_void_p(u.data_ptr()), C.c_void_p(w.data_ptr()), None,
                              s) == L.SEM_EINVAL
    assert lib.sem_ax_noalloc(m._h, 7, C.c_void_p(u.data_ptr()), C.c_void_p(w.data_ptr()),
                              C.c_void_p(dot.data_ptr()), s) == L.SEM_EINVAL
    m.close()
