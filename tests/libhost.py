"""Test helpers around the library's host-only entry points (no GPU needed)."""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sem.h")


def header_functions():
    """Names of the functions declared in include/sem.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sem_[a-z0-9_]+)\s*\(", text)))


def make_desc(L, N, nel, periodic=(0, 0, 0), lo=(0, 0, 0), hi=(1, 1, 1), mapping=0, vertices=None,
              dirichlet=-1, fp32=False):
    d = L.MeshDesc()
    d.N = N
    d.nel[:] = list(nel)
    d.periodic[:] = list(periodic)
    d.lo[:] = [float(v) for v in lo]
    d.hi[:] = [float(v) for v in hi]
    d.mapping = mapping
    keep = None
    if vertices is not None:
        keep = np.ascontiguousarray(vertices, dtype=np.float64)
        d.vertices = keep.ctypes.data_as(C.POINTER(C.c_double))
    d.dirichlet_faces = dirichlet
    d.precision_flags = 1 if fp32 else 0
    return d, keep


def host_setup(N, nel, **kw):
    """Run sem_host_setup and return its products as numpy arrays."""
    from paper_2109_03592_amd import _lib as L
    lib = L.load()
    d, keep = make_desc(L, N, nel, **kw)
    info = L.MeshInfo()
    L.check(lib.sem_host_setup(C.byref(d), C.byref(info), None, None, None, None, None, None, None, None),
            "sem_host_setup")
    n = info.n_local
    out = dict(info=info, gid=np.zeros(n, np.int64), mult=np.zeros(n, np.uint8), mask=np.zeros(n, np.uint8),
               G=np.zeros((6, n)), B=np.zeros(n), inv=np.zeros(n),
               off=np.zeros(info.gs_plan_ids + 1, np.int32), idx=np.zeros(info.gs_plan_len, np.int32))
    L.check(lib.sem_host_setup(C.byref(d), None, out["gid"].ctypes.data, out["mult"].ctypes.data,
                               out["mask"].ctypes.data, out["G"].ctypes.data, out["B"].ctypes.data,
                               out["inv"].ctypes.data, out["off"].ctypes.data, out["idx"].ctypes.data),
            "sem_host_setup")
    del keep
    return out


def apply_plan(v, off, idx, n_sum):
    """The gather-scatter plan applied on the host in the kernel's order
    (copies summed left to right from 0, written back; zeroed ids -> 0)."""
    v = np.array(v, dtype=np.float64, copy=True)
    lens = np.diff(off)
    n_ids = len(lens)
    s = np.zeros(n_sum)
    for pos in range(int(lens.max()) if n_ids else 0):
        ids = np.nonzero(lens[:n_sum] > pos)[0]
        s[ids] = s[ids] + v[idx[off[ids] + pos]]
    for pos in range(int(lens.max()) if n_ids else 0):
        ids = np.nonzero(lens > pos)[0]
        q = idx[off[ids] + pos]
        vals = np.where(ids < n_sum, s[np.minimum(ids, max(n_sum - 1, 0))] if n_sum else 0.0, 0.0)
        v[q] = vals
    return v
