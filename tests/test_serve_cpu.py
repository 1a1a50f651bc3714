"""CPU tests of the serving scheduler's policy: admission order, slot limit,
device-memory budget, least-recently-used mesh eviction, refusal of requests
that cannot fit, latency bookkeeping and the drain limit.  The engine here is
a test double with a fake clock and a cost model (steps per solve); the
product's only engine runs the HIP library."""
import math

import pytest

from paper_2109_03592_amd.serve import Job, Scheduler, ServeStats

import seeded_inputs as SI


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeEngine:
    def __init__(self, clock, max_slots=4, dt=0.01, mesh_b=100, slot_b=10):
        self.clock, self.max_slots, self.dt = clock, max_slots, dt
        self.mesh_b, self.slot_b = mesh_b, slot_b
        self.resident_set = set()
        self.left = {}
        self.key_of = {}
        self.next_slot = 0
        self.log = []
        self.sched = None

    def mesh_bytes(self, key):
        return self.mesh_b * key[1]

    def slot_bytes(self, key, mixed):
        return self.slot_b * key[1] * (2 if mixed else 1)

    def resident(self, key):
        return key in self.resident_set

    def load(self, key):
        assert key not in self.resident_set
        self.resident_set.add(key)
        self.log.append(("load", key))

    def evict(self, key):
        assert key in self.resident_set
        assert key not in self.key_of.values(), "evicted a mesh in use"
        self.resident_set.remove(key)
        self.log.append(("evict", key))

    def admit(self, job):
        assert job.key in self.resident_set
        assert len(self.left) < self.max_slots
        slot = self.next_slot
        self.next_slot += 1
        self.left[slot] = 1 + job.key[1] // 2       # cost model: steps grow with size
        self.key_of[slot] = job.key
        self.log.append(("admit", job.rid))
        return slot

    def step(self, k):
        self.clock.t += self.dt
        for s in self.left:
            self.left[s] -= 1
        if self.sched is not None:
            assert self.sched.used() <= self.sched.budget

    def finished(self):
        return [s for s, v in self.left.items() if v <= 0]

    def retire(self, slot):
        del self.left[slot]
        del self.key_of[slot]
        return 0, 10, 1e-11

    def idle(self, seconds):
        self.clock.t += max(seconds, 1e-4)


def _jobs(spec):
    return [Job(i, t, key, mixed) for i, (t, key, mixed) in enumerate(spec)]


def test_all_complete_fifo_and_slot_limit():
    clock = Clock()
    eng = FakeEngine(clock, max_slots=3)
    sched = Scheduler(eng, budget_bytes=10 ** 9, clock=clock)
    eng.sched = sched
    jobs = _jobs([(0.001 * i, (7, 1 + i % 5), bool(i % 2)) for i in range(40)])
    st = sched.run(jobs, horizon=10.0, drain_limit=10.0)
    assert st.completed == 40 and st.unfinished == 0 and st.refused == 0
    admits = [e[1] for e in eng.log if e[0] == "admit"]
    assert admits == sorted(admits)                  # FIFO
    assert st.max_active <= 3
    assert all(j.t_done >= j.t_admit >= j.t_arrival for j in jobs)
    assert len(st.latencies) == 40 and min(st.latencies) > 0


def test_budget_and_lru_eviction():
    clock = Clock()
    eng = FakeEngine(clock, max_slots=8, mesh_b=100, slot_b=10)
    # room for about two meshes of size 3 plus their slots
    sched = Scheduler(eng, budget_bytes=700, clock=clock)
    eng.sched = sched
    keys = [(5, 3), (7, 3), (5, 2), (7, 3), (5, 3)]
    jobs = _jobs([(0.05 * i, keys[i % len(keys)], False) for i in range(25)])
    st = sched.run(jobs, horizon=10.0, drain_limit=10.0)
    assert st.completed == 25
    evictions = [e for e in eng.log if e[0] == "evict"]
    assert evictions, "a tight budget must evict idle meshes"
    assert sched.used() <= 700


def test_request_that_cannot_fit_is_refused_not_blocking():
    clock = Clock()
    eng = FakeEngine(clock, max_slots=2)
    sched = Scheduler(eng, budget_bytes=500, clock=clock)
    eng.sched = sched
    jobs = _jobs([(0.0, (7, 100), False), (0.0, (5, 1), False), (0.01, (5, 2), True)])
    st = sched.run(jobs, horizon=1.0, drain_limit=1.0)
    assert st.refused == 1 and st.completed == 2


def test_drain_limit_counts_unfinished():
    clock = Clock()
    eng = FakeEngine(clock, max_slots=1, dt=0.5)
    sched = Scheduler(eng, budget_bytes=10 ** 9, clock=clock)
    jobs = _jobs([(0.0, (7, 40), False), (0.0, (7, 40), False)])
    st = sched.run(jobs, horizon=0.1, drain_limit=1.0)
    assert st.completed == 0 and st.unfinished == 2
    assert not sched.active and sched.slot_mem == 0
    # both enter the percentiles at their wait so far (lower bounds)
    assert len(st.censored) == 2 and min(st.censored) >= 1.0
    s = st.summary()
    assert s["censored"] == 2 and s["percentiles_are_lower_bounds"]
    assert s["p50_ms"] >= 1000.0 and s["p99_ms"] >= 1000.0


def test_censored_requests_raise_the_percentiles():
    """Unfinished requests count at their wait so far: a saturated run's p99
    can only rise over the completed-only figure."""
    st = ServeStats(completed=90, elapsed=2.0, latencies=[i / 1000 for i in range(1, 91)],
                    censored=[5.0] * 10)
    s = st.summary()
    assert s["p50_completed_ms"] == pytest.approx(45.0)
    assert s["p50_ms"] == pytest.approx(50.0)
    assert s["p99_ms"] == pytest.approx(5000.0) and s["max_ms"] == pytest.approx(5000.0)
    assert s["censored"] == 10 and s["percentiles_are_lower_bounds"]


def test_percentiles():
    st = ServeStats(completed=100, elapsed=2.0, latencies=[i / 1000 for i in range(1, 101)])
    s = st.summary()
    assert s["p50_ms"] == pytest.approx(50.0) and s["p99_ms"] == pytest.approx(99.0)
    assert s["solves_per_s"] == pytest.approx(50.0)


def test_poisson_arrivals_and_catalog():
    reqs = SI.poisson_requests(200.0, 5.0, 2000, seed=7, catalog=12)
    assert 800 < len(reqs) < 1200                       # ~ rate * duration
    gaps = [b.t_arrival - a.t_arrival for a, b in zip(reqs, reqs[1:])]
    assert all(g > 0 for g in gaps)
    assert abs(sum(gaps) / len(gaps) - 1 / 200.0) < 0.25 / 200.0
    assert len({r.nel for r in reqs}) <= 12
    assert {r.N for r in reqs} <= {5, 7}
    for r in reqs:
        assert 64 / 2 <= r.E <= 32768 * 2
    mixed = sum(r.mixed for r in reqs) / len(reqs)
    assert 0.4 < mixed < 0.6


def test_batched_case_rule():
    cases = SI.batched_box_cases(64)
    assert len(cases) == 64 and {c.N for c in cases} <= {5, 7, 9}
    for c in cases:
        nx, ny, nz = c.nel
        assert c.E == nx * ny * nz and 1 <= c.E <= 8192
    Es = sorted(c.E for c in cases)
    assert Es[0] <= 32 and Es[-1] >= 1000            # spans the log-uniform range
