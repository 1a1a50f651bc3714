"""ctypes front-end of the plain FP64 CPU oracle (``sem_oracle.c``).

Test infrastructure only: the test-suite, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg are its only users.  The product package never
imports it, and it imports nothing from the product package.

Every function follows the paper's definitions (arXiv 2109.03592): the GLL
tensor-product basis and the global/local split of section 2, and the local
operator (the element stiffness that Algorithm 1 evaluates, here as staged
tensor contractions).  See ``sem_oracle.c`` for the formulas.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "sem_oracle.c")

MAP_BOX, MAP_PIPE = 0, 1
ALL_FACES = 0x3F


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, FMA contraction allowed, no
    fast-math) into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
               "-std=c99", "-o", _SO + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Mesh(C.Structure):
    _fields_ = [("N", C.c_int), ("nel", C.c_int * 3), ("periodic", C.c_int * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("mapping", C.c_int),
                ("vertices", C.POINTER(C.c_double)), ("dirichlet", C.c_int)]


class _Problem(C.Structure):
    _fields_ = [("N", C.c_int), ("ne", C.c_long), ("nloc", C.c_long), ("nglob", C.c_long),
                ("D", C.c_void_p), ("G", C.c_void_p), ("h1", C.c_void_p), ("h2", C.c_void_p),
                ("B", C.c_void_p), ("gid", C.c_void_p), ("gmask", C.c_void_p),
                ("invdiag", C.c_void_p)]


class _Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int),
                ("rel_residual", C.c_double), ("bnorm", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        vp, lg, i = C.c_void_p, C.c_long, C.c_int
        L.orc_gll.argtypes = [i, vp, vp]
        L.orc_deriv.argtypes = [i, vp, vp]
        for f in ("orc_num_elements", "orc_num_local", "orc_num_global"):
            getattr(L, f).argtypes = [C.POINTER(_Mesh)]
            getattr(L, f).restype = lg
        L.orc_coords.argtypes = [C.POINTER(_Mesh), vp, vp, lg, vp, vp, vp]
        L.orc_geom.argtypes = [C.POINTER(_Mesh), vp, vp, vp, lg, vp, vp, vp, vp, vp]
        L.orc_numbering.argtypes = [C.POINTER(_Mesh), vp, lg, vp]
        L.orc_global_mask.argtypes = [C.POINTER(_Mesh), vp]
        L.orc_multiplicity.argtypes = [lg, vp, lg, vp]
        L.orc_ax.argtypes = [i, lg, vp, vp, vp, vp, vp, vp, vp]
        L.orc_gs.argtypes = [lg, vp, lg, vp, vp]
        L.orc_jacobi.argtypes = [i, lg, vp, vp, vp, vp, vp, vp, lg, vp, vp]
        L.orc_apply.argtypes = [C.POINTER(_Problem), vp, vp]
        L.orc_pcg.argtypes = [C.POINTER(_Problem), vp, vp, C.c_double, i, C.POINTER(_Stats)]
        L.orc_pcg.restype = i
        L.orc_threads.argtypes = [i]
        L.orc_threads.restype = i
        _lib = L
    return _lib


def threads(n: int = 0) -> int:
    """Set the oracle's OpenMP thread count (n > 0); returns the count in use."""
    return int(lib().orc_threads(int(n)))


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def gll(N: int):
    """GLL nodes and weights of order N (N+1 points)."""
    xi = np.zeros(N + 1)
    w = np.zeros(N + 1)
    lib().orc_gll(N, _p(xi), _p(w))
    return xi, w


def deriv(N: int, xi: np.ndarray):
    """Derivative matrix D[i, l] = l_l'(xi_i)."""
    D = np.zeros((N + 1, N + 1))
    lib().orc_deriv(N, _p(np.ascontiguousarray(xi, dtype=np.float64)), _p(D))
    return D


@dataclass
class PCGResult:
    status: int
    iterations: int
    restarts: int
    rel_residual: float
    bnorm: float


class OracleMesh:
    """A structured hexahedral SEM mesh evaluated by the oracle.

    ``elems`` restricts geometry, numbering and the operator to a list of
    elements (used for sampled checks on meshes too large to evaluate whole).
    """

    def __init__(self, N: int, nel: Sequence[int], periodic=(0, 0, 0), lo=(0.0, 0.0, 0.0),
                 hi=(1.0, 1.0, 1.0), mapping: int = MAP_BOX,
                 vertices: Optional[np.ndarray] = None, dirichlet: Optional[int] = None):
        self.N = int(N)
        self.P = self.N + 1
        self.nel = tuple(int(v) for v in nel)
        self.periodic = tuple(int(v) for v in periodic)
        self.lo, self.hi = tuple(map(float, lo)), tuple(map(float, hi))
        self.mapping = int(mapping)
        self._vert = None if vertices is None else np.ascontiguousarray(vertices, dtype=np.float64)
        if dirichlet is None:
            dirichlet = 0
            for d in range(3):
                if not self.periodic[d]:
                    dirichlet |= 3 << (2 * d)
        self.dirichlet = int(dirichlet)
        m = _Mesh()
        m.N = self.N
        m.nel[:] = list(self.nel)
        m.periodic[:] = list(self.periodic)
        m.lo[:] = list(self.lo)
        m.hi[:] = list(self.hi)
        m.mapping = self.mapping
        m.vertices = (self._vert.ctypes.data_as(C.POINTER(C.c_double))
                      if self._vert is not None else None)
        m.dirichlet = self.dirichlet
        self._m = m
        L = lib()
        self.E = int(L.orc_num_elements(C.byref(m)))
        self.nloc = int(L.orc_num_local(C.byref(m)))
        self.nglob = int(L.orc_num_global(C.byref(m)))
        self.xi, self.w = gll(self.N)
        self.D = deriv(self.N, self.xi)
        self._cache = {}

    # -- setup -------------------------------------------------------------
    def _elems(self, elems):
        if elems is None:
            return None, self.E
        el = np.ascontiguousarray(elems, dtype=np.int64)
        return el, len(el)

    def coords(self, elems=None):
        key = ("coords", None if elems is None else tuple(elems))
        if elems is None and key in self._cache:
            return self._cache[key]
        el, ne = self._elems(elems)
        n = ne * self.P ** 3
        x, y, z = np.zeros(n), np.zeros(n), np.zeros(n)
        lib().orc_coords(C.byref(self._m), _p(self.xi), _p(el), ne, _p(x), _p(y), _p(z))
        if elems is None:
            self._cache[key] = (x, y, z)
        return x, y, z

    def geom(self, elems=None):
        """(G[6, n], B[n]): g1..g6 = G_rr, G_ss, G_tt, G_rs, G_rt, G_st."""
        key = ("geom", None)
        if elems is None and key in self._cache:
            return self._cache[key]
        el, ne = self._elems(elems)
        x, y, z = self.coords(elems)
        n = ne * self.P ** 3
        G = np.zeros((6, n))
        B = np.zeros(n)
        lib().orc_geom(C.byref(self._m), _p(self.w), _p(self.D), _p(el), ne,
                       _p(x), _p(y), _p(z), _p(G), _p(B))
        if elems is None:
            self._cache[key] = (G, B)
        return G, B

    def numbering(self, elems=None):
        if elems is None and "gid" in self._cache:
            return self._cache["gid"]
        el, ne = self._elems(elems)
        gid = np.zeros(ne * self.P ** 3, dtype=np.int64)
        lib().orc_numbering(C.byref(self._m), _p(el), ne, _p(gid))
        if elems is None:
            self._cache["gid"] = gid
        return gid

    def global_mask(self):
        if "gmask" not in self._cache:
            gm = np.zeros(self.nglob, dtype=np.uint8)
            lib().orc_global_mask(C.byref(self._m), _p(gm))
            self._cache["gmask"] = gm
        return self._cache["gmask"]

    def global_mult(self):
        if "gmult" not in self._cache:
            gid = self.numbering()
            gm = np.zeros(self.nglob, dtype=np.int32)
            lib().orc_multiplicity(self.nloc, _p(gid), self.nglob, _p(gm))
            self._cache["gmult"] = gm
        return self._cache["gmult"]

    def local_mult(self):
        return self.global_mult()[self.numbering()]

    def local_mask(self):
        return self.global_mask()[self.numbering()]

    # -- operators ---------------------------------------------------------
    def ax(self, u, h1=None, h2=None, elems=None):
        """Local operator A_L u (the operator of Algorithm 1; no gather-scatter)."""
        G, B = self.geom(elems)
        ne = self.E if elems is None else len(elems)
        u = np.ascontiguousarray(u, dtype=np.float64)
        assert u.size == ne * self.P ** 3
        w = np.zeros_like(u)
        h1 = None if h1 is None else np.ascontiguousarray(h1, dtype=np.float64)
        h2 = None if h2 is None else np.ascontiguousarray(h2, dtype=np.float64)
        lib().orc_ax(self.N, ne, _p(self.D), _p(G), _p(h1), _p(h2), _p(B if h2 is not None else None),
                     _p(u), _p(w))
        return w

    def gs(self, v, masked: bool = True):
        """Q Q^T v followed by the Dirichlet mask (returns a new array)."""
        v = np.array(v, dtype=np.float64, copy=True)
        gm = self.global_mask() if masked else None
        lib().orc_gs(self.nloc, _p(self.numbering()), self.nglob, _p(gm), _p(v))
        return v

    def apply(self, u, h1=None, h2=None, masked: bool = True):
        """mask(Q Q^T A_L u): the assembled operator on the E-vector u."""
        return self.gs(self.ax(u, h1, h2), masked=masked)

    def mass(self, f):
        """mask(Q Q^T (B f)): the right-hand side of the weak form for forcing f."""
        _, B = self.geom()
        return self.gs(B * f)

    def jacobi(self, h1=None, h2=None):
        """Inverse of the assembled diagonal on unmasked nodes, 0 on masked."""
        key = ("jacobi", h1 is None, h2 is None)
        if h1 is None and h2 is None and key in self._cache:
            return self._cache[key]
        G, B = self.geom()
        inv = np.zeros(self.nloc)
        h1c = None if h1 is None else np.ascontiguousarray(h1, dtype=np.float64)
        h2c = None if h2 is None else np.ascontiguousarray(h2, dtype=np.float64)
        lib().orc_jacobi(self.N, self.E, _p(self.D), _p(G), _p(h1c), _p(h2c),
                         _p(B if h2 is not None else None), _p(self.numbering()), self.nglob,
                         _p(self.global_mask()), _p(inv))
        if h1 is None and h2 is None:
            self._cache[key] = inv
        return inv

    def _problem(self, h1=None, h2=None):
        G, B = self.geom()
        inv = self.jacobi(h1, h2)
        pb = _Problem()
        pb.N, pb.ne, pb.nloc, pb.nglob = self.N, self.E, self.nloc, self.nglob
        keep = [self.D, G, h1, h2, B, self.numbering(), self.global_mask(), inv]
        pb.D, pb.G = _p(self.D).value, _p(G).value
        pb.h1 = None if h1 is None else _p(h1).value
        pb.h2 = None if h2 is None else _p(h2).value
        pb.B = _p(B).value if h2 is not None else None
        pb.gid, pb.gmask, pb.invdiag = (_p(self.numbering()).value, _p(self.global_mask()).value,
                                        _p(inv).value)
        return pb, keep

    def pcg(self, b, x0=None, tol: float = 1e-10, max_iter: int = 5000, h1=None, h2=None):
        """Jacobi-PCG on the masked assembled system; returns (x, PCGResult)."""
        pb, keep = self._problem(h1, h2)
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.nloc) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        st = _Stats()
        status = lib().orc_pcg(C.byref(pb), _p(b), _p(x), tol, max_iter, C.byref(st))
        del keep
        return x, PCGResult(status, st.iterations, st.restarts, st.rel_residual, st.bnorm)

    # -- helpers -----------------------------------------------------------
    def dot(self, a, b):
        """Unique-dof inner product sum_local a b / mult."""
        return float(np.sum(a * b / self.local_mult()))

    def true_residual(self, b, x, h1=None, h2=None):
        r = b - self.apply(x, h1, h2)
        return np.sqrt(self.dot(r, r)) / np.sqrt(self.dot(b, b))


def pipe_mesh(nx: int = 48, ny: int = 48, nz: int = 96, N: int = 7, length: float = 10.0):
    """Square [-1,1]^2 x [0,length] mapped to a circular pipe, periodic in z,
    Dirichlet on the wall (the four sides of the square)."""
    return OracleMesh(N, (nx, ny, nz), periodic=(0, 0, 1), lo=(-1.0, -1.0, 0.0),
                      hi=(1.0, 1.0, length), mapping=MAP_PIPE)
