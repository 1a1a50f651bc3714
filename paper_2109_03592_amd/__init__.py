"""MI355X (gfx950) spectral-element Poisson engine: Python binding.

Thin marshalling over the C ABI of ``include/sem.h``: every step of the path
(operator, gather-scatter, dot products, CG updates) runs in the HIP kernels
of ``libsem.so``.  PyTorch provides device memory and streams only.  The
binding checks tensor device, dtype, contiguity and length before passing raw
pointers, because the C ABI cannot.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L
from ._lib import (SEM_FP32, SEM_FP64, SEM_MAP_BOX, SEM_MAP_PIPE_SQ2DISK, SEM_MAX_ORDER,
                   SEM_PREC_FP64, SEM_PREC_MIXED, SemError)

__all__ = ["Mesh", "Batch", "SolveResult", "SemError", "box_mesh", "pipe_mesh", "export_gll", "version",
           "SEM_FP64", "SEM_FP32", "SEM_MAP_BOX", "SEM_MAP_PIPE_SQ2DISK", "SEM_MAX_ORDER"]


def version() -> str:
    return L.load().sem_version().decode()


def _stream_handle(stream) -> Optional[int]:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def export_gll(N: int):
    """(xi, w, D) of the library's own GLL rule and derivative matrix."""
    xi, w, D = np.zeros(N + 1), np.zeros(N + 1), np.zeros((N + 1, N + 1))
    L.check(L.load().sem_export_gll(N, xi.ctypes.data, w.ctypes.data, D.ctypes.data), "sem_export_gll")
    return xi, w, D


@dataclass
class SolveResult:
    status: int
    iterations: int
    outer_iterations: int
    rel_residual: float
    bnorm: float
    seconds: float
    ms_operator: float = 0.0
    ms_gather_scatter: float = 0.0
    ms_update: float = 0.0
    operator_launches: int = 0

    @property
    def ok(self) -> bool:
        return self.status == L.SEM_OK


class Mesh:
    """A structured hexahedral mesh of order N resident on the current GPU."""

    def __init__(self, N: int, nel: Sequence[int], periodic=(0, 0, 0), lo=(0.0, 0.0, 0.0),
                 hi=(1.0, 1.0, 1.0), mapping: int = SEM_MAP_BOX, vertices: Optional[np.ndarray] = None,
                 dirichlet_faces: int = -1, with_fp32: bool = False, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("paper_2109_03592_amd needs a ROCm GPU (gfx950); none is visible")
        self._lib = L.load()
        d = L.MeshDesc()
        d.N = int(N)
        d.nel[:] = [int(v) for v in nel]
        d.periodic[:] = [int(v) for v in periodic]
        d.lo[:] = [float(v) for v in lo]
        d.hi[:] = [float(v) for v in hi]
        d.mapping = int(mapping)
        self._vert = None
        if vertices is not None:
            v = np.ascontiguousarray(vertices, dtype=np.float64).reshape(-1)
            need = (d.nel[0] + 1) * (d.nel[1] + 1) * (d.nel[2] + 1) * 3
            if v.size != need:
                raise ValueError(f"vertices: expected {need} doubles, got {v.size}")
            self._vert = v
            d.vertices = v.ctypes.data_as(C.POINTER(C.c_double))
        d.dirichlet_faces = int(dirichlet_faces)
        d.precision_flags = L.SEM_WITH_FP32 if with_fp32 else 0
        self.desc = d
        self.with_fp32 = bool(with_fp32)
        h = C.c_void_p()
        L.check(self._lib.sem_setup(C.byref(d), _stream_handle(stream), C.byref(h)), "sem_setup")
        self._h = h
        info = L.MeshInfo()
        L.check(self._lib.sem_info(h, C.byref(info)), "sem_info")
        self.info = info
        self.N = info.N
        self.P = self.N + 1
        self.E = int(info.E)
        self.n_local = int(info.n_local)
        self.n_global = int(info.n_global)
        self.device = torch.device("cuda", torch.cuda.current_device())

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.sem_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- argument checks -----------------------------------------------------
    def _vec(self, t: torch.Tensor, name: str, dtype=None, n=None) -> int:
        n = self.n_local if n is None else n
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name}: expected a CUDA tensor")
        if dtype is not None and t.dtype != dtype:
            raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
        if t.dtype not in (torch.float64, torch.float32):
            raise TypeError(f"{name}: expected float64 or float32")
        if not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name}: expected a contiguous tensor of {n} elements")
        if t.device.index != self.device.index:
            raise ValueError(f"{name}: tensor is on another device")
        return t.data_ptr()

    @staticmethod
    def _dt(t: torch.Tensor) -> int:
        if t.dtype == torch.float32:
            return SEM_FP32
        return SEM_FP64

    def empty(self, dtype=torch.float64) -> torch.Tensor:
        return torch.empty(self.n_local, dtype=dtype, device=self.device)

    def zeros(self, dtype=torch.float64) -> torch.Tensor:
        return torch.zeros(self.n_local, dtype=dtype, device=self.device)

    # -- launch configuration -------------------------------------------------
    def set_operator_config(self, epw: int, grid: int = 0):
        """Elements per workgroup and persistent grid size of the operator (0 = default)."""
        L.check(self._lib.sem_set_operator_config(self._h, int(epw), int(grid)), "sem_set_operator_config")

    def operator_config(self):
        e, g = C.c_int(), C.c_int()
        L.check(self._lib.sem_get_operator_config(self._h, C.byref(e), C.byref(g)), "sem_get_operator_config")
        return e.value, g.value

    def set_gs_kind(self, kind: str = "auto"):
        """Gather-scatter kernel: "auto" (the lattice kernel where the mesh
        allows it), "plan" (the CSR plan) or "stream" (auto with the
        row-streaming kernel at every order 2..7); all give the same bits."""
        k = {"auto": 0, "plan": 1, "stream": 2}.get(kind)
        if k is None:
            raise ValueError(f"unknown gather-scatter kind {kind!r}")
        L.check(self._lib.sem_set_gs_config(self._h, k), "sem_set_gs_config")

    def gs_kind(self):
        """(kind, lattice kernel in use)."""
        k, on = C.c_int(), C.c_int()
        L.check(self._lib.sem_get_gs_config(self._h, C.byref(k), C.byref(on)), "sem_get_gs_config")
        return ("auto", "plan", "stream")[k.value], bool(on.value)

    def set_axgs_config(self, enable: bool = True, epw: int = 0, lines_per_wg: int = 0):
        """Fused operator and gather-scatter: on/off, elements per tile and
        x-lines per workgroup (0 = automatic)."""
        L.check(self._lib.sem_set_axgs_config(self._h, int(bool(enable)), int(epw), int(lines_per_wg)),
                "sem_set_axgs_config")

    def axgs_info(self, dtype=torch.float64) -> dict:
        """Shape of the fused operator and gather-scatter for a precision
        (enabled = 0 where the two launches run)."""
        info = L.AxgsInfo()
        dt = SEM_FP32 if dtype == torch.float32 else SEM_FP64
        L.check(self._lib.sem_get_axgs_info(self._h, dt, C.byref(info)), "sem_get_axgs_info")
        return {k: getattr(info, k) for k, _ in L.AxgsInfo._fields_}

    def set_helmholtz(self, h1: Optional[torch.Tensor] = None, h2: Optional[torch.Tensor] = None, stream=None):
        """Helmholtz form h1 (grad, grad) + h2 B of the operator (None: h1 = 1,
        h2 = 0; both None restores Poisson).  h1, h2: FP64 E-vectors."""
        for t, name in ((h1, "h1"), (h2, "h2")):
            if t is not None:
                self._vec(t, name, torch.float64)
        L.check(self._lib.sem_set_helmholtz(self._h, None if h1 is None else h1.data_ptr(),
                                            None if h2 is None else h2.data_ptr(), _stream_handle(stream)),
                "sem_set_helmholtz")

    def set_coarse(self, chebyshev_steps: int = 10, fraction: float = 0.01, stream=None):
        """Add the coarse term of Eq. 6 to the FP64 preconditioner (Jacobi +
        trilinear vertex space, A0 = P^T A P, chebyshev_steps Chebyshev steps
        on [fraction b, b]); chebyshev_steps=0 removes it."""
        L.check(self._lib.sem_set_coarse(self._h, int(chebyshev_steps), float(fraction), _stream_handle(stream)),
                "sem_set_coarse")

    def set_schwarz(self, enable: bool = True, stream=None):
        """Use the overlapping Schwarz local solves of Eq. 6 (FDM on each
        element extended by one node layer) as the local part of the FP64
        preconditioner; enable=False restores Jacobi."""
        L.check(self._lib.sem_set_schwarz(self._h, 1 if enable else 0, _stream_handle(stream)), "sem_set_schwarz")

    def schwarz_info(self) -> dict:
        en, nf = C.c_int(0), C.c_int64(0)
        L.check(self._lib.sem_get_schwarz_info(self._h, C.byref(en), C.byref(nf)), "sem_get_schwarz_info")
        return {"enabled": bool(en.value), "n_factors": int(nf.value)}

    def coarse_info(self) -> dict:
        info = L.CoarseInfo()
        L.check(self._lib.sem_get_coarse_info(self._h, C.byref(info)), "sem_get_coarse_info")
        return {k: getattr(info, k) for k, _ in L.CoarseInfo._fields_}

    def precond(self, r: torch.Tensor, z: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """z = M^-1 r (FP64 E-vectors): Jacobi, plus the coarse term when set."""
        z = torch.empty_like(r) if z is None else z
        pr, pz = self._vec(r, "r", torch.float64), self._vec(z, "z", torch.float64)
        if pr == pz:
            raise ValueError("precond: r and z must be distinct")
        L.check(self._lib.sem_precond_apply(self._h, pr, pz, _stream_handle(stream)), "sem_precond_apply")
        return z

    # -- operators -----------------------------------------------------------
    def ax(self, u: torch.Tensor, w: Optional[torch.Tensor] = None, dot: bool = False, stream=None):
        """w = A_L u (no gather-scatter); with dot=True also returns sum u.w (device scalar)."""
        w = torch.empty_like(u) if w is None else w
        pu, pw = self._vec(u, "u"), self._vec(w, "w", dtype=u.dtype)
        if pu == pw:
            raise ValueError("ax: u and w must be distinct")
        dt = torch.zeros(1, dtype=torch.float64, device=self.device) if dot else None
        L.check(self._lib.sem_ax(self._h, self._dt(u), pu, pw, None if dt is None else dt.data_ptr(),
                                 _stream_handle(stream)), "sem_ax")
        return (w, dt) if dot else w

    def ax_noalloc(self, u: torch.Tensor, w: torch.Tensor, dot: torch.Tensor, stream=None):
        """w = A_L u and dot[0] = sum u.w with caller-owned w and dot (one FP64
        entry); the library allocates nothing (its dot partials use a fixed
        per-device array)."""
        pu, pw = self._vec(u, "u"), self._vec(w, "w", dtype=u.dtype)
        if pu == pw:
            raise ValueError("ax_noalloc: u and w must be distinct")
        if dot.dtype != torch.float64 or dot.device != self.device or dot.numel() < 1:
            raise ValueError("ax_noalloc: dot must be an FP64 tensor on the mesh's device")
        L.check(self._lib.sem_ax_noalloc(self._h, self._dt(u), pu, pw, dot.data_ptr(), _stream_handle(stream)),
                "sem_ax_noalloc")
        return w, dot

    def gs(self, v: torch.Tensor, stream=None) -> torch.Tensor:
        """In-place Q Q^T and Dirichlet mask."""
        L.check(self._lib.sem_gs(self._h, self._dt(v), self._vec(v, "v"), _stream_handle(stream)), "sem_gs")
        return v

    def axgs(self, u: torch.Tensor, w: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """w = mask(Q Q^T A_L u)."""
        w = torch.empty_like(u) if w is None else w
        pu, pw = self._vec(u, "u"), self._vec(w, "w", dtype=u.dtype)
        if pu == pw:
            raise ValueError("axgs: u and w must be distinct")
        L.check(self._lib.sem_axgs(self._h, self._dt(u), pu, pw, _stream_handle(stream)), "sem_axgs")
        return w

    def mass(self, f: torch.Tensor, b: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """b = mask(Q Q^T (B f))."""
        b = torch.empty_like(f) if b is None else b
        L.check(self._lib.sem_mass(self._h, self._vec(f, "f", torch.float64), self._vec(b, "b", torch.float64),
                                   _stream_handle(stream)), "sem_mass")
        return b

    def scatter(self, v_global: torch.Tensor, u: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """u = mask(Q v_global)."""
        u = self.empty() if u is None else u
        pv = self._vec(v_global, "v_global", torch.float64, n=self.n_global)
        L.check(self._lib.sem_scatter(self._h, pv, self._vec(u, "u", torch.float64), _stream_handle(stream)),
                "sem_scatter")
        return u

    # -- solve -----------------------------------------------------------------
    def solve(self, b: torch.Tensor, x: Optional[torch.Tensor] = None, tol: float = 1e-10,
              max_iter: int = 5000, precision: str = "fp64", inner_tol: float = 1e-4,
              inner_max_iter: int = 0, poll_every: int = 16, use_graph: bool = True,
              fixed_iters: int = 0, profile: bool = False, initial_guess: Optional[bool] = None,
              stream=None, raise_on_error: bool = True) -> Tuple[torch.Tensor, SolveResult]:
        """Jacobi-PCG for A x = b.  x receives the solution; it is also the initial
        guess when initial_guess is True (default: whenever x is given)."""
        o = L.SolveOpts()
        self._lib.sem_solve_opts_default(C.byref(o))
        o.tol, o.max_iter = float(tol), int(max_iter)
        o.precision = SEM_PREC_MIXED if precision == "mixed" else SEM_PREC_FP64
        o.inner_tol, o.inner_max_iter = float(inner_tol), int(inner_max_iter)
        o.poll_every, o.use_graph, o.fixed_iters = int(poll_every), int(bool(use_graph)), int(fixed_iters)
        if initial_guess is None:
            initial_guess = x is not None
        o.x0_given = int(bool(initial_guess) and x is not None)
        o.profile = int(bool(profile))
        x = self.zeros() if x is None else x
        st = L.SolveStats()
        status = self._lib.sem_pcg_solve(self._h, self._vec(b, "b", torch.float64), self._vec(x, "x", torch.float64),
                                         C.byref(o), C.byref(st), _stream_handle(stream))
        res = SolveResult(st.status, st.iterations, st.outer_iterations, st.rel_residual, st.bnorm, st.seconds,
                          st.ms_operator, st.ms_gather_scatter, st.ms_update, st.operator_launches)
        if raise_on_error and status != L.SEM_OK:
            raise SemError(status, "sem_pcg_solve")
        return x, res

    # -- exports ---------------------------------------------------------------
    def export_maps(self):
        gid = np.zeros(self.n_local, dtype=np.int64)
        mult = np.zeros(self.n_local, dtype=np.uint8)
        mask = np.zeros(self.n_local, dtype=np.uint8)
        L.check(self._lib.sem_export_maps(self._h, gid.ctypes.data, mult.ctypes.data, mask.ctypes.data),
                "sem_export_maps")
        return gid, mult, mask

    def export_geom(self):
        G = np.zeros((6, self.n_local))
        B = np.zeros(self.n_local)
        inv = np.zeros(self.n_local)
        L.check(self._lib.sem_export_geom(self._h, G.ctypes.data, B.ctypes.data, inv.ctypes.data), "sem_export_geom")
        return G, B, inv

    def load_geometry(self, G: np.ndarray, B: np.ndarray, stream=None):
        """Replace the geometric factors G[6, n_local] and mass B[n_local] (host arrays)."""
        G = np.ascontiguousarray(G, dtype=np.float64)
        B = np.ascontiguousarray(B, dtype=np.float64)
        if G.shape != (6, self.n_local) or B.shape != (self.n_local,):
            raise ValueError("load_geometry: expected G[6, n_local] and B[n_local]")
        L.check(self._lib.sem_load_geometry(self._h, G.ctypes.data, B.ctypes.data, _stream_handle(stream)),
                "sem_load_geometry")

    def export_coords(self):
        xyz = np.zeros((3, self.n_local))
        L.check(self._lib.sem_export_coords(self._h, xyz.ctypes.data), "sem_export_coords")
        return xyz


def _opts(lib, tol=1e-10, max_iter=5000, precision="fp64", inner_tol=1e-4, inner_max_iter=0,
          poll_every=16, use_graph=True):
    o = L.SolveOpts()
    lib.sem_solve_opts_default(C.byref(o))
    o.tol, o.max_iter = float(tol), int(max_iter)
    o.precision = SEM_PREC_MIXED if precision == "mixed" else SEM_PREC_FP64
    o.inner_tol, o.inner_max_iter = float(inner_tol), int(inner_max_iter)
    o.poll_every, o.use_graph = int(poll_every), int(bool(use_graph))
    return o


def _result(st) -> SolveResult:
    return SolveResult(st.status, st.iterations, st.outer_iterations, st.rel_residual, st.bnorm, st.seconds,
                       st.ms_operator, st.ms_gather_scatter, st.ms_update, st.operator_launches)


class Batch:
    """Many concurrent solves advanced by persistent batched kernels (C ABI
    sem_batch_*).  Meshes, right-hand sides and solutions passed in are kept
    referenced here until their slot is retired."""

    def __init__(self, max_slots: int = 64, budget_bytes: int = 0, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("paper_2109_03592_amd needs a ROCm GPU (gfx950); none is visible")
        self._lib = L.load()
        h = C.c_void_p()
        L.check(self._lib.sem_batch_create(int(max_slots), C.c_size_t(int(budget_bytes)), _stream_handle(stream),
                                           C.byref(h)), "sem_batch_create")
        self._h = h
        self.max_slots = int(max_slots)
        self._held = {}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sem_batch_free(self._h)
            self._h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tune(self, meshes, stream=None):
        """Autotune elements per workgroup per order and precision on these meshes."""
        arr = (C.c_void_p * len(meshes))(*[m._h.value for m in meshes])
        L.check(self._lib.sem_batch_tune(self._h, arr, len(meshes), _stream_handle(stream)), "sem_batch_tune")

    def set_epw(self, N: int, epw: int):
        L.check(self._lib.sem_batch_set_epw(self._h, int(N), int(epw)), "sem_batch_set_epw")

    def epw(self, N: int, precision: str = "fp64") -> int:
        """Elements per operator workgroup in use for order N and precision ('fp64' or 'fp32')."""
        e = C.c_int()
        p = SEM_FP32 if precision == "fp32" else SEM_FP64
        L.check(self._lib.sem_batch_get_epw(self._h, int(N), p, C.byref(e)), "sem_batch_get_epw")
        return e.value

    def set_grid(self, ax_grid: int = 0, vec_grid: int = 0):
        """Workgroups of the batched operator and vector launches (0 = default)."""
        L.check(self._lib.sem_batch_set_grid(self._h, int(ax_grid), int(vec_grid)), "sem_batch_set_grid")

    def grid(self):
        a, v = C.c_int(), C.c_int()
        L.check(self._lib.sem_batch_get_grid(self._h, C.byref(a), C.byref(v)), "sem_batch_get_grid")
        return a.value, v.value

    def solve(self, meshes, bs, xs=None, stream=None, raise_on_error: bool = True, **kw):
        """Solve A_i x_i = b_i together; returns (xs, [SolveResult])."""
        n = len(meshes)
        xs = [m.zeros() for m in meshes] if xs is None else list(xs)
        for m, b, x in zip(meshes, bs, xs):
            m._vec(b, "b", torch.float64)
            m._vec(x, "x", torch.float64)
        o = _opts(self._lib, **kw)
        harr = (C.c_void_p * n)(*[m._h.value for m in meshes])
        barr = (C.c_void_p * n)(*[b.data_ptr() for b in bs])
        xarr = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
        stats = (L.SolveStats * n)()
        status = self._lib.sem_batch_solve(self._h, harr, n, barr, xarr, C.byref(o), stats, _stream_handle(stream))
        res = [_result(stats[i]) for i in range(n)]
        if raise_on_error and status != L.SEM_OK:
            raise SemError(status, "sem_batch_solve")
        return xs, res

    def admit(self, mesh, b, x=None, stream=None, **kw) -> int:
        """Admit one solve (x: solution, zero initial guess); returns its slot."""
        x = mesh.zeros() if x is None else x
        mesh._vec(b, "b", torch.float64)
        mesh._vec(x, "x", torch.float64)
        o = _opts(self._lib, **kw)
        slot = C.c_int()
        L.check(self._lib.sem_batch_admit(self._h, mesh._h, b.data_ptr(), x.data_ptr(), C.byref(o), C.byref(slot),
                                          _stream_handle(stream)), "sem_batch_admit")
        self._held[slot.value] = (mesh, b, x)
        return slot.value

    def step(self, iterations: int = 16, use_graph: bool = True, stream=None) -> int:
        n = C.c_int()
        L.check(self._lib.sem_batch_step(self._h, int(iterations), int(bool(use_graph)), _stream_handle(stream),
                                         C.byref(n)), "sem_batch_step")
        return n.value

    def finished(self):
        cap = self.max_slots
        arr = (C.c_int * cap)()
        n = C.c_int()
        L.check(self._lib.sem_batch_finished(self._h, arr, cap, C.byref(n)), "sem_batch_finished")
        return [arr[i] for i in range(min(n.value, cap))]

    def retire(self, slot: int):
        """Free a slot; returns (x, SolveResult)."""
        st = L.SolveStats()
        L.check(self._lib.sem_batch_retire(self._h, int(slot), C.byref(st)), "sem_batch_retire")
        _, _, x = self._held.pop(slot, (None, None, None))
        return x, _result(st)


class Projection:
    """Projection onto previous solutions of one mesh (C ABI sem_proj_*):
    successive solves start from the A-norm best approximation in the span of
    earlier solutions."""

    def __init__(self, mesh: "Mesh", max_vectors: int = 8):
        self._lib = mesh._lib
        self.mesh = mesh
        h = C.c_void_p()
        L.check(self._lib.sem_proj_create(mesh._h, int(max_vectors), C.byref(h)), "sem_proj_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sem_proj_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self) -> int:
        n = C.c_int()
        L.check(self._lib.sem_proj_size(self._h, C.byref(n)), "sem_proj_size")
        return n.value

    def reset(self):
        L.check(self._lib.sem_proj_reset(self._h), "sem_proj_reset")

    def project(self, b: torch.Tensor, x: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        x = self.mesh.zeros() if x is None else x
        self.mesh._vec(b, "b", torch.float64)
        self.mesh._vec(x, "x", torch.float64)
        L.check(self._lib.sem_proj_project(self._h, b.data_ptr(), x.data_ptr(), _stream_handle(stream)),
                "sem_proj_project")
        return x

    def add(self, x: torch.Tensor, stream=None) -> bool:
        self.mesh._vec(x, "x", torch.float64)
        a = C.c_int()
        L.check(self._lib.sem_proj_add(self._h, x.data_ptr(), C.byref(a), _stream_handle(stream)), "sem_proj_add")
        return bool(a.value)

    def solve(self, b: torch.Tensor, x: Optional[torch.Tensor] = None, stream=None, raise_on_error: bool = True,
              **kw) -> Tuple[torch.Tensor, SolveResult]:
        """Projected PCG solve; the solution then joins the basis."""
        x = self.mesh.zeros() if x is None else x
        self.mesh._vec(b, "b", torch.float64)
        self.mesh._vec(x, "x", torch.float64)
        o = _opts(self._lib, **kw)
        st = L.SolveStats()
        status = self._lib.sem_proj_solve(self._h, b.data_ptr(), x.data_ptr(), C.byref(o), C.byref(st),
                                          _stream_handle(stream))
        res = _result(st)
        if raise_on_error and status != L.SEM_OK:
            raise SemError(status, "sem_proj_solve")
        return x, res


def fdm_1d(N: int, ell: float, left: int, right: int):
    """Host-only 1-D Schwarz factors (S, lam, lo): S^T B S = I, S^T A S =
    diag(lam) on the kept extended indices lo .. lo+len(lam)-1; side kinds 0
    neighbour, 1 Dirichlet, 2 free end."""
    lib = L.load()
    n = N + 3
    S = np.zeros(n * n)
    lam = np.zeros(n)
    lo, cnt = C.c_int(0), C.c_int(0)
    L.check(lib.sem_host_fdm_1d(int(N), float(ell), int(left), int(right), S.ctypes.data, lam.ctypes.data,
                                C.byref(lo), C.byref(cnt)), "sem_host_fdm_1d")
    c = cnt.value
    return S[:c * c].reshape(c, c).copy(), lam[:c].copy(), lo.value


def box_mesh(N: int, nel: Sequence[int], vertices=None, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
             periodic=(0, 0, 0), **kw) -> Mesh:
    return Mesh(N, nel, periodic=periodic, lo=lo, hi=hi, mapping=SEM_MAP_BOX, vertices=vertices, **kw)


def pipe_mesh(nx: int = 48, ny: int = 48, nz: int = 96, N: int = 7, length: float = 10.0, **kw) -> Mesh:
    """Square [-1,1]^2 x [0,length] mapped to a circular pipe; periodic in z,
    Dirichlet on the wall."""
    return Mesh(N, (nx, ny, nz), periodic=(0, 0, 1), lo=(-1.0, -1.0, 0.0), hi=(1.0, 1.0, length),
                mapping=SEM_MAP_PIPE_SQ2DISK, **kw)
