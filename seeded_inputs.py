"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method: it only draws random numbers and
evaluates the manufactured solution and forcing at points it is given.  Both the
CPU oracle and the GPU library receive the same arrays from here.

Workloads (the paper's pipe meshes are not available, so these stand in):
  * jittered box: interior vertices of a regular lattice moved by
    U(-amp, amp) times the element width, independently per coordinate;
  * pipe right-hand side: one U[-1, 1) value per global node, mean removed;
  * manufactured solution u = sin(pi x) sin(pi y) sin(pi z), forcing 3 pi^2 u;
  * batched meshes: E* log-uniform, element counts nx, ny, nz rounded from it,
    order N drawn from a set;
  * serving: Poisson arrivals of such meshes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np


def jittered_box_vertices(nel: Sequence[int], lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                          amp: float = 0.05, seed: int = 1) -> np.ndarray:
    """Vertex lattice (nx+1)(ny+1)(nz+1) x 3, x fastest.  Strictly interior
    vertices get U(-amp, amp) * h_d added to coordinate d (h_d element width)."""
    nx, ny, nz = (int(v) for v in nel)
    rng = np.random.default_rng(seed)
    h = [(hi[d] - lo[d]) / nel[d] for d in range(3)]
    iz, iy, ix = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    V = np.stack([lo[0] + ix * h[0], lo[1] + iy * h[1], lo[2] + iz * h[2]], axis=-1).reshape(-1, 3)
    jit = rng.uniform(-amp, amp, size=V.shape) * np.asarray(h)
    interior = ((ix > 0) & (ix < nx) & (iy > 0) & (iy < ny) & (iz > 0) & (iz < nz)).reshape(-1)
    V[interior] += jit[interior]
    return np.ascontiguousarray(V)


def uniform_global_values(nglob: int, seed: int = 2) -> np.ndarray:
    """One U[-1, 1) value per global node with the arithmetic mean removed."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1.0, 1.0, size=int(nglob))
    v -= v.mean()
    return v


def sin3(x, y, z):
    """Manufactured solution sin(pi x) sin(pi y) sin(pi z)."""
    return np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


def sin3_forcing(x, y, z):
    """-Laplacian of sin3: 3 pi^2 sin(pi x) sin(pi y) sin(pi z)."""
    return 3.0 * np.pi ** 2 * sin3(x, y, z)


def random_local(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """U[-1, 1) values for an E-vector (not continuous across elements)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=int(n)).astype(dtype)


def uniform_local(n: int, seed: int, lo: float, hi: float) -> np.ndarray:
    """U[lo, hi) values for an E-vector (e.g. positive coefficients)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=int(n))


def travelling_forcing(x, y, z, t: float, speed: float = 0.02):
    """sin(pi (x + speed t)) sin(pi y) sin(pi z): a smoothly moving forcing
    whose successive right-hand sides resemble those of a time-stepping run."""
    return np.sin(np.pi * (x + speed * t)) * np.sin(np.pi * y) * np.sin(np.pi * z)


def elements_from_target(e_star: float) -> Tuple[int, int, int]:
    """Box element counts from a target element count E*:
    nx = round(cbrt E*), ny = round(sqrt(E*/nx)), nz = max(1, round(E*/(nx ny)))."""
    nx = max(1, int(round(e_star ** (1.0 / 3.0))))
    ny = max(1, int(round(math.sqrt(e_star / nx))))
    nz = max(1, int(round(e_star / (nx * ny))))
    return nx, ny, nz


@dataclass
class BoxCase:
    seed: int
    N: int
    nel: Tuple[int, int, int]

    @property
    def E(self) -> int:
        return self.nel[0] * self.nel[1] * self.nel[2]


def batched_box_cases(count: int = 64, emin: float = 8, emax: float = 4096,
                      orders=(5, 7, 9), seed0: int = 100) -> List[BoxCase]:
    """Mesh i uses seed seed0+i: E* log-uniform in [emin, emax], N uniform in orders."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        e_star = math.exp(rng.uniform(math.log(emin), math.log(emax)))
        N = int(orders[int(rng.integers(len(orders)))])
        out.append(BoxCase(seed0 + i, N, elements_from_target(e_star)))
    return out


@dataclass
class Request:
    rid: int
    t_arrival: float
    N: int
    nel: Tuple[int, int, int]
    mixed: bool

    @property
    def E(self) -> int:
        return self.nel[0] * self.nel[1] * self.nel[2]


def poisson_requests(rate: float, duration: float, max_requests: int, emin: float = 64,
                     emax: float = 32768, orders=(5, 7), seed: int = 7,
                     catalog: int = 0) -> List[Request]:
    """Poisson arrivals at `rate` per second for `duration` seconds (at most
    `max_requests`).  Per request: E* log-uniform in [emin, emax] (or one of
    `catalog` pre-drawn sizes when catalog > 0), N uniform in `orders`,
    precision FP64 or mixed with equal probability."""
    rng = np.random.default_rng(seed)
    cat = None
    if catalog > 0:
        cat = [elements_from_target(math.exp(rng.uniform(math.log(emin), math.log(emax))))
               for _ in range(catalog)]
    t, out = 0.0, []
    while len(out) < max_requests:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        if cat is None:
            nel = elements_from_target(math.exp(rng.uniform(math.log(emin), math.log(emax))))
        else:
            nel = cat[int(rng.integers(len(cat)))]
        N = int(orders[int(rng.integers(len(orders)))])
        mixed = bool(rng.integers(2))
        out.append(Request(len(out), t, N, nel, mixed))
    return out
