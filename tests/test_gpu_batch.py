"""Batched and continuous solves (sem_batch_*) against the oracle.

Many independent jittered box meshes of different orders and sizes are solved
in one set of persistent launches; every solution must reach a true relative
residual <= 1e-10 measured by the oracle, and a system's result must be
bit-identical whether it is solved alone or among others.
"""
import numpy as np
import pytest
import torch

import seeded_inputs as SI

pytestmark = pytest.mark.gpu


def _case(semlib, oracle_mod, N, nel, seed, fp32=True):
    V = SI.jittered_box_vertices(nel, seed=seed)
    m = semlib.box_mesh(N, nel, vertices=V, with_fp32=fp32)
    om = oracle_mod.OracleMesh(N, nel, vertices=V)
    x, y, z = om.coords()
    b = om.mass(SI.sin3_forcing(x, y, z))
    return m, om, b


CASES = [(3, (2, 3, 2), 11), (5, (3, 3, 3), 12), (7, (4, 4, 4), 13), (9, (2, 2, 3), 14),
         (5, (5, 4, 3), 15), (7, (2, 1, 1), 16), (4, (3, 2, 2), 17), (6, (2, 2, 2), 18)]


@pytest.fixture(scope="module")
def cases(semlib, oracle_mod):
    out = [_case(semlib, oracle_mod, N, nel, seed) for N, nel, seed in CASES]
    yield out
    for m, _, _ in out:
        m.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_solve_matches_oracle(semlib, cases, prec):
    print(f"case: batch solve {prec} over {len(cases)} meshes", flush=True)
    B = semlib.Batch(max_slots=16)
    meshes = [c[0] for c in cases]
    bs = [torch.from_numpy(c[2]).cuda() for c in cases]
    xs, res = B.solve(meshes, bs, tol=1e-10, precision=prec, poll_every=8)
    for (m, om, b), x, r in zip(cases, xs, res):
        rel = om.true_residual(b, x.cpu().numpy())
        assert r.ok and rel <= 1e-10, (m.N, m.E, prec, r, rel)
        if prec == "fp64":
            # the single-mesh solver takes the same number of iterations up to rounding drift
            _, r1 = m.solve(torch.from_numpy(b).cuda(), tol=1e-10)
            assert abs(r1.iterations - r.iterations) <= max(2, 0.03 * r1.iterations)
    B.close()


def test_batch_alone_vs_mixed_bitwise(semlib, cases):
    """A system's iterates do not depend on its co-residents."""
    print("case: batch alone vs in the mix", flush=True)
    B = semlib.Batch(max_slots=16)
    m, om, b = cases[2]
    bd = torch.from_numpy(b).cuda()
    (x_alone,), (r_alone,) = B.solve([m], [bd], tol=1e-10)
    meshes = [c[0] for c in cases]
    bs = [torch.from_numpy(c[2]).cuda() for c in cases]
    xs, res = B.solve(meshes, bs, tol=1e-10)
    assert torch.equal(xs[2], x_alone) and res[2].iterations == r_alone.iterations
    # graph replay and plain launches give the same bits
    xs2, res2 = B.solve(meshes, bs, tol=1e-10, use_graph=False)
    for a, c in zip(xs, xs2):
        assert torch.equal(a, c)
    B.close()


@pytest.mark.parametrize("grid", [1, 3, 7])
def test_batch_multi_item_walks(semlib, cases, grid):
    """With 1, 3 or 7 persistent workgroups every workgroup walks many
    (slot, tile) items of several slots and orders in turn (the path of every
    launch on large batches): each slot still meets the oracle's true
    residual and keeps the bits of its alone-solve at the default grid."""
    print(f"case: batch multi-item walks, grid {grid}", flush=True)
    B = semlib.Batch(max_slots=16)
    meshes = [c[0] for c in cases]
    bs = [torch.from_numpy(c[2]).cuda() for c in cases]
    alone = {}
    for prec in ("fp64", "mixed"):
        for k in (0, 2, 3):
            (xa,), (ra,) = B.solve([meshes[k]], [bs[k]], tol=1e-10, precision=prec)
            alone[(prec, k)] = (xa.clone(), ra.iterations)
    B.set_grid(grid, grid)
    assert B.grid() == (grid, grid)
    for prec in ("fp64", "mixed"):
        xs, res = B.solve(meshes, bs, tol=1e-10, precision=prec, poll_every=8)
        for (m, om, b), x, r in zip(cases, xs, res):
            rel = om.true_residual(b, x.cpu().numpy())
            assert r.ok and rel <= 1e-10, (grid, prec, m.N, m.E, rel)
        for k in (0, 2, 3):
            xa, ia = alone[(prec, k)]
            assert torch.equal(xs[k], xa) and res[k].iterations == ia, (grid, prec, k)
    B.set_grid(0, 0)
    B.close()


@pytest.mark.timeout(900)
def test_batch_64_meshes(semlib, oracle_mod):
    """The batched workload at its real size: 64 jittered boxes (seeds
    100..163, E log-uniform in [8, 4096], N in {5, 7, 9}), after the autotuner,
    FP64 and mixed.  Every slot's solution meets the oracle's true residual,
    and the largest slots of each order keep the bits of their alone-solves."""
    cases64 = SI.batched_box_cases(64)
    print(f"case: batch 64 meshes, {sum(c.E for c in cases64)} elements", flush=True)
    meshes, oms, bh, bs = [], [], [], []
    for c in cases64:
        V = SI.jittered_box_vertices(c.nel, seed=c.seed)
        meshes.append(semlib.box_mesh(c.N, c.nel, vertices=V, with_fp32=True))
        om = oracle_mod.OracleMesh(c.N, c.nel, vertices=V)
        x, y, z = om.coords()
        b = om.mass(SI.sin3_forcing(x, y, z))
        oms.append(om)
        bh.append(b)
        bs.append(torch.from_numpy(b).cuda())
    B = semlib.Batch(max_slots=64)
    B.tune(meshes)
    picks = []
    for N in (5, 7, 9):
        ks = [k for k, c in enumerate(cases64) if c.N == N]
        if ks:
            picks.append(max(ks, key=lambda k: cases64[k].E))
    for prec in ("fp64", "mixed"):
        print(f"case: batch 64 meshes {prec}", flush=True)
        xs, res = B.solve(meshes, bs, tol=1e-10, precision=prec, poll_every=16)
        worst = 0.0
        for k, (om, b, x, r) in enumerate(zip(oms, bh, xs, res)):
            rel = om.true_residual(b, x.cpu().numpy())
            worst = max(worst, rel)
            assert r.ok and rel <= 1e-10, (prec, k, cases64[k], rel)
        print(f"  {prec}: worst oracle residual {worst:.2e}", flush=True)
        for k in picks:
            (xa,), (ra,) = B.solve([meshes[k]], [bs[k]], tol=1e-10, precision=prec, poll_every=16)
            assert torch.equal(xs[k], xa) and res[k].iterations == ra.iterations, (prec, k)
    B.close()
    for m in meshes:
        m.close()


def test_continuous_batching(semlib, cases, oracle_mod):
    """Slots admitted while others run: each result equals its alone-solve bit for bit."""
    print("case: continuous batching", flush=True)
    B = semlib.Batch(max_slots=4)
    ref = {}
    for k, (m, om, b) in enumerate(cases):
        (xa,), (ra,) = B.solve([m], [torch.from_numpy(b).cuda()], tol=1e-10,
                               precision="mixed" if k % 2 else "fp64")
        ref[k] = (xa.clone(), ra.iterations)
    queue = list(range(len(cases)))
    live = {}
    done = {}
    steps = 0
    while queue or live:
        while queue and len(live) < 4:
            k = queue.pop(0)
            m, om, b = cases[k]
            s = B.admit(m, torch.from_numpy(b).cuda(), tol=1e-10, precision="mixed" if k % 2 else "fp64")
            live[s] = k
        B.step(5)
        steps += 1
        assert steps < 10000
        for s in B.finished():
            x, r = B.retire(s)
            done[live.pop(s)] = (x, r)
    for k, (x, r) in done.items():
        m, om, b = cases[k]
        assert r.ok
        assert om.true_residual(b, x.cpu().numpy()) <= 1e-10
        assert torch.equal(x, ref[k][0]) and r.iterations == ref[k][1], k
    B.close()


def test_batch_ignores_garbage_x_without_guess(semlib, cases, oracle_mod):
    """Without an initial guess a slot starts from x = 0 whatever x holds
    (FP64 and mixed)."""
    print("case: batch x without initial guess", flush=True)
    B = semlib.Batch(max_slots=2)
    m, om, b = cases[1]
    for prec in ("fp64", "mixed"):
        x = torch.full((om.nloc,), float("nan"), dtype=torch.float64, device="cuda")
        s = B.admit(m, torch.from_numpy(b).cuda(), x, tol=1e-10, precision=prec)
        while s not in B.finished():
            B.step(8)
        xr, r = B.retire(s)
        assert r.ok, (prec, r)
        assert om.true_residual(b, xr.cpu().numpy()) <= 1e-10
    B.close()


def test_tuner_and_budget(semlib, cases):
    print("case: batch tuner and budget", flush=True)
    B = semlib.Batch(max_slots=16)
    meshes = [c[0] for c in cases]
    B.tune(meshes)
    for m in meshes:
        e = B.epw(m.N)
        assert 1 <= e and e * (m.N + 1) ** 2 <= 512
    bs = [torch.from_numpy(c[2]).cuda() for c in cases]
    xs, res = B.solve(meshes, bs, tol=1e-10)
    assert all(r.ok for r in res)
    B.close()
    # a budget too small for one slot's vectors is refused, not overrun
    small = semlib.Batch(max_slots=2, budget_bytes=1024)
    m, om, b = cases[2]
    with pytest.raises(semlib.SemError) as ei:
        small.admit(m, torch.from_numpy(b).cuda())
    assert ei.value.status == 6  # SEM_EBUDGET
    small.close()


def test_serving_loop_small(semlib):
    """Real-time continuous batching on the GPU engine: every request of a
    short Poisson stream completes with a true 1e-10 residual."""
    print("case: serving loop, small catalog", flush=True)
    from paper_2109_03592_amd.serve import serve_rates
    res = serve_rates([200.0], duration=1.5, max_requests=300, drain_limit=30.0, max_slots=32, budget_gb=8.0,
                      catalog=6, emin=8, emax=512, orders=(5, 7), iterations_per_step=8, tune=False)
    r = res[0]
    assert r["failed"] == 0 and r["unfinished"] == 0 and r["refused"] == 0, r
    assert r["completed"] == r["requests"] > 100
    assert r["p99_ms"] >= r["p50_ms"] > 0
