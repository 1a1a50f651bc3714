"""Continuous-batching solve server.

Requests (a mesh from a resident catalog, a right-hand side, a precision)
arrive over time.  The scheduler admits pending requests into free batch slots
while the device-memory budget allows, advances every admitted solve by a few
CG iterations per step (one set of persistent batched launches, see
``Batch``), retires finished solves and records arrival-to-result latency.
Requests that arrive while others are on the GPU join at the next step
boundary, so their work overlaps on the device.

The scheduling policy (``Scheduler``) is plain host logic over an engine
interface; ``GpuEngine`` is the only engine of the product and drives the HIP
library.  Meshes live in a catalog with least-recently-used eviction under the
same budget.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple


@dataclass
class Job:
    rid: int
    t_arrival: float
    key: Tuple            # catalog key of the mesh: (N, nel)
    mixed: bool
    t_admit: float = -1.0
    t_done: float = -1.0
    slot: int = -1
    status: int = -1
    iterations: int = 0
    rel_residual: float = float("nan")


@dataclass
class ServeStats:
    completed: int = 0
    unfinished: int = 0
    refused: int = 0
    elapsed: float = 0.0
    latencies: List[float] = field(default_factory=list)
    # requests without a result when the run ends: their wait so far, a lower
    # bound of their latency (right-censored)
    censored: List[float] = field(default_factory=list)
    steps: int = 0
    max_active: int = 0

    @staticmethod
    def _pct(lat: List[float], p: float) -> float:
        if not lat:
            return float("nan")
        k = min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))
        return lat[k]

    def summary(self) -> Dict:
        """p50/p99 over every request that arrived: completed ones at their
        latency, unfinished ones at their wait so far.  With unfinished
        requests the percentiles are lower bounds (``censored`` > 0); the
        completed-only figures are reported beside them."""
        done = sorted(self.latencies)
        every = sorted(self.latencies + self.censored)
        return {"completed": self.completed, "unfinished": self.unfinished, "refused": self.refused,
                "solves_per_s": self.completed / self.elapsed if self.elapsed > 0 else 0.0,
                "p50_ms": self._pct(every, 50) * 1e3, "p99_ms": self._pct(every, 99) * 1e3,
                "max_ms": (every[-1] * 1e3 if every else float("nan")),
                "censored": len(self.censored), "percentiles_are_lower_bounds": bool(self.censored),
                "p50_completed_ms": self._pct(done, 50) * 1e3, "p99_completed_ms": self._pct(done, 99) * 1e3,
                "elapsed_s": self.elapsed, "steps": self.steps, "max_active": self.max_active}


class Scheduler:
    """FIFO admission into batch slots under a device-memory budget.

    engine must provide: max_slots, slot_bytes(key, mixed), mesh_bytes(key),
    resident(key), load(key), evict(key), admit(job) -> slot, step(k) -> None,
    finished() -> [slot], retire(slot) -> (status, iterations, rel_residual).
    clock() returns seconds since the start of the run.
    """

    def __init__(self, engine, budget_bytes: int, clock: Callable[[], float], iterations_per_step: int = 8):
        self.e = engine
        self.budget = int(budget_bytes)
        self.clock = clock
        self.k = int(iterations_per_step)
        self.pending: deque = deque()
        self.active: Dict[int, Job] = {}
        self.mesh_lru: "OrderedDict[Tuple, int]" = OrderedDict()  # key -> bytes
        self.pinned: Dict[Tuple, int] = {}                         # key -> active jobs using it
        self.slot_mem = 0

    # -- memory accounting --------------------------------------------------
    def used(self) -> int:
        return self.slot_mem + sum(self.mesh_lru.values())

    def _make_room(self, need: int, keep: Optional[Tuple] = None) -> bool:
        """Evict idle meshes (least recently used first, never `keep`) until `need` bytes fit."""
        while self.used() + need > self.budget:
            victim = next((k for k in self.mesh_lru if self.pinned.get(k, 0) == 0 and k != keep), None)
            if victim is None:
                return False
            self.e.evict(victim)
            del self.mesh_lru[victim]
        return True

    def _try_admit(self, job: Job) -> bool:
        if len(self.active) >= self.e.max_slots:
            return False
        need = self.e.slot_bytes(job.key, job.mixed)
        if job.key not in self.mesh_lru:
            need += self.e.mesh_bytes(job.key)
        if need > self.budget:
            return False
        if not self._make_room(need, keep=job.key):
            return False
        if job.key not in self.mesh_lru:
            self.e.load(job.key)
            self.mesh_lru[job.key] = self.e.mesh_bytes(job.key)
            if not self._make_room(self.e.slot_bytes(job.key, job.mixed), keep=job.key):
                return False
        self.mesh_lru.move_to_end(job.key)
        job.slot = self.e.admit(job)
        job.t_admit = self.clock()
        self.slot_mem += self.e.slot_bytes(job.key, job.mixed)
        self.pinned[job.key] = self.pinned.get(job.key, 0) + 1
        self.active[job.slot] = job
        return True

    def _retire(self, slot: int, stats: ServeStats):
        job = self.active.pop(slot)
        job.status, job.iterations, job.rel_residual = self.e.retire(slot)
        job.t_done = self.clock()
        self.slot_mem -= self.e.slot_bytes(job.key, job.mixed)
        self.pinned[job.key] -= 1
        stats.completed += 1
        stats.latencies.append(job.t_done - job.t_arrival)
        return job

    # -- main loop ------------------------------------------------------------
    def run(self, jobs: Sequence[Job], horizon: float, drain_limit: float,
            on_done: Optional[Callable[[Job], None]] = None) -> ServeStats:
        """Serve `jobs` (sorted by arrival) arriving until `horizon` seconds,
        then keep serving admitted and pending work for at most `drain_limit`
        more seconds."""
        stats = ServeStats()
        arrivals = deque(j for j in jobs if j.t_arrival <= horizon)
        stats.refused = sum(1 for j in jobs if j.t_arrival > horizon)
        t_end = horizon + drain_limit
        while True:
            now = self.clock()
            while arrivals and arrivals[0].t_arrival <= now:
                self.pending.append(arrivals.popleft())
            while self.pending and self._try_admit(self.pending[0]):
                self.pending.popleft()
            if not self.active:
                if self.pending:
                    # nothing runs and the head still does not fit: it never will
                    self.pending.popleft()
                    stats.refused += 1
                    continue
                if not arrivals:
                    break
                self.e.idle(max(0.0, min(arrivals[0].t_arrival - now, 0.002)))
                continue
            stats.max_active = max(stats.max_active, len(self.active))
            self.e.step(self.k)
            stats.steps += 1
            for slot in self.e.finished():
                job = self._retire(slot, stats)
                if on_done:
                    on_done(job)
            if self.clock() > t_end:
                break
        stats.unfinished += len(self.active) + len(self.pending) + len(arrivals)
        now = self.clock()
        for job in list(self.active.values()) + list(self.pending) + list(arrivals):
            stats.censored.append(max(0.0, now - job.t_arrival))
        for slot in list(self.active):
            job = self.active.pop(slot)
            self.e.retire(slot)
            self.slot_mem -= self.e.slot_bytes(job.key, job.mixed)
            self.pinned[job.key] -= 1
        self.pending.clear()
        stats.elapsed = self.clock()
        return stats


class GpuEngine:
    """Engine of the scheduler on the HIP library: a resident mesh catalog
    (each mesh with a base right-hand side) and one Batch."""

    def __init__(self, max_slots: int, budget_bytes: int, tol: float = 1e-10, inner_tol: float = 1e-4,
                 max_iter: int = 20000, seed0: int = 1000, tune_keys: Sequence[Tuple] = (),
                 coarse_min_elems: int = 0, coarse_steps: int = 4, coarse_fraction: float = 0.05):
        import torch
        import paper_2109_03592_amd as sem
        self.torch, self.sem = torch, sem
        self.max_slots = int(max_slots)
        self.batch = sem.Batch(max_slots=max_slots, budget_bytes=budget_bytes)
        self.tol, self.inner_tol, self.max_iter = tol, inner_tol, max_iter
        self.seed0 = seed0
        # meshes of at least coarse_min_elems elements (0: none) carry the
        # coarse term of Eq. 6; their requests (FP64 and mixed) take it in the batch
        self.coarse_min_elems = int(coarse_min_elems)
        self.coarse_steps, self.coarse_fraction = int(coarse_steps), float(coarse_fraction)
        self.meshes: Dict[Tuple, object] = {}
        self.base_rhs: Dict[Tuple, object] = {}
        self.jobs: Dict[int, Tuple] = {}
        self._bytes: Dict[Tuple, int] = {}
        if tune_keys:
            ms = [self._build(k) for k in tune_keys]
            self.batch.tune(ms)
            for m in ms:
                m.close()

    # catalog ------------------------------------------------------------------
    def _build(self, key):
        import seeded_inputs as SI
        N, nel = key
        V = SI.jittered_box_vertices(nel, seed=hash((N,) + tuple(nel)) % (2 ** 31))
        return self.sem.box_mesh(N, nel, vertices=V, with_fp32=True)

    def mesh_bytes(self, key) -> int:
        if key not in self._bytes:
            N, nel = key
            nl = (N + 1) ** 3 * nel[0] * nel[1] * nel[2]
            # G (FP64 + FP32), B, inverse diagonal (FP64 + FP32), mult, gid, plan, base rhs
            self._bytes[key] = int(nl * (48 + 24 + 8 + 8 + 4 + 1 + 4 + 4 + 8))
        return self._bytes[key]

    def _coarse(self, key) -> bool:
        N, nel = key
        return self.coarse_min_elems > 0 and nel[0] * nel[1] * nel[2] >= self.coarse_min_elems

    def slot_bytes(self, key, mixed: bool) -> int:
        N, nel = key
        E = nel[0] * nel[1] * nel[2]
        nl = (N + 1) ** 3 * E
        extra = 0
        if self._coarse(key):
            extra = nl * (4 if mixed else 8) + E * 8 * 14   # P z0 and the slot's coarse vectors
        return int(nl * (8 * 3 + (16 if mixed else 0) + 8 + 8) + extra)   # slot vectors + b + x

    def resident(self, key) -> bool:
        return key in self.meshes

    def load(self, key):
        m = self._build(key)
        if self._coarse(key):
            m.set_coarse(self.coarse_steps, self.coarse_fraction)
        xyz = self.torch.from_numpy(m.export_coords()).cuda()
        f = self._forcing(xyz)
        self.base_rhs[key] = m.mass(f)
        del xyz, f
        self.meshes[key] = m
        self._bytes[key] = int(m.info.device_bytes) + 8 * m.n_local

    def _forcing(self, xyz):
        """3 pi^2 sin(pi x) sin(pi y) sin(pi z): the manufactured forcing (input data)."""
        t = self.torch
        return 3.0 * math.pi ** 2 * t.sin(math.pi * xyz[0]) * t.sin(math.pi * xyz[1]) * t.sin(math.pi * xyz[2])

    def evict(self, key):
        m = self.meshes.pop(key)
        self.base_rhs.pop(key, None)
        m.close()

    # slots --------------------------------------------------------------------
    def admit(self, job: Job) -> int:
        import numpy as np
        m = self.meshes[job.key]
        scale = 0.5 + np.random.default_rng(self.seed0 + job.rid).uniform()
        b = self.base_rhs[job.key] * scale
        slot = self.batch.admit(m, b, tol=self.tol, max_iter=self.max_iter,
                                precision="mixed" if job.mixed else "fp64", inner_tol=self.inner_tol)
        self.jobs[slot] = (b, job)
        return slot

    def step(self, k: int):
        self.batch.step(k)

    def finished(self):
        return self.batch.finished()

    def retire(self, slot: int):
        x, r = self.batch.retire(slot)
        self.jobs.pop(slot, None)
        return r.status, r.iterations, r.rel_residual

    def idle(self, seconds: float):
        time.sleep(seconds)

    def close(self):
        for k in list(self.meshes):
            self.evict(k)
        self.batch.close()


def serve_rates(rates: Sequence[float], duration: float = 10.0, max_requests: int = 2000,
                drain_limit: float = 20.0, max_slots: int = 64, budget_gb: float = 200.0,
                catalog: int = 24, emin: float = 64, emax: float = 32768, orders=(5, 7),
                iterations_per_step: int = 8, seed: int = 7, tune: bool = True,
                coarse_min_elems: int = 0) -> List[Dict]:
    """Serve Poisson arrival streams at each rate; returns one summary per rate
    (coarse_min_elems > 0: meshes of that many elements or more carry the
    coarse term of Eq. 6, taken by their requests)."""
    import seeded_inputs as SI
    budget = int(budget_gb * 2 ** 30)
    # catalog keys = every (N, nel) the streams can draw
    keys = set()
    streams = {}
    for lam in rates:
        reqs = SI.poisson_requests(lam, duration, max_requests, emin=emin, emax=emax, orders=orders,
                                   seed=seed, catalog=catalog)
        streams[lam] = reqs
        keys.update((r.N, r.nel) for r in reqs)
    tune_keys = []
    if tune:
        # one mid-sized catalog mesh per order
        for N in sorted({k[0] for k in keys}):
            ks = sorted((k for k in keys if k[0] == N), key=lambda k: k[1][0] * k[1][1] * k[1][2])
            tune_keys.append(ks[len(ks) // 2])
    eng = GpuEngine(max_slots, budget, tune_keys=tune_keys, coarse_min_elems=coarse_min_elems)
    base = [time.perf_counter()]
    sched = Scheduler(eng, budget, clock=lambda: time.perf_counter() - base[0],
                      iterations_per_step=iterations_per_step)
    out = []
    try:
        for lam in rates:
            jobs = [Job(r.rid, r.t_arrival, (r.N, r.nel), r.mixed) for r in streams[lam]]
            # make this stream's meshes resident before its clock starts (catalog, LRU)
            for key in sorted({j.key for j in jobs}):
                if key not in sched.mesh_lru and sched._make_room(eng.mesh_bytes(key)):
                    eng.load(key)
                    sched.mesh_lru[key] = eng.mesh_bytes(key)
            eng.torch.cuda.synchronize()
            bad = []
            base[0] = time.perf_counter()
            st = sched.run(jobs, horizon=duration, drain_limit=drain_limit,
                           on_done=lambda j: bad.append(j) if (j.status != 0 or j.rel_residual > 1e-10) else None)
            sm = st.summary()
            sm.update({"rate": lam, "requests": len(jobs), "failed": len(bad),
                       "coarse_min_elems": coarse_min_elems})
            out.append(sm)
            print(json.dumps(sm), file=sys.stderr, flush=True)
    finally:
        eng.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--rates", default="50,100,200,500,1000,2000")
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--max-requests", type=int, default=2000)
    ap.add_argument("--drain", type=float, default=20.0)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--coarse-min-elems", type=int, default=0,
                    help="meshes of at least this many elements carry the coarse term (0: Jacobi only)")
    a = ap.parse_args(argv)
    res = serve_rates([float(v) for v in a.rates.split(",")], duration=a.duration, max_requests=a.max_requests,
                      drain_limit=a.drain, max_slots=a.slots, budget_gb=a.budget_gb,
                      coarse_min_elems=a.coarse_min_elems)
    print(json.dumps({"serving": res}))


if __name__ == "__main__":
    main()
