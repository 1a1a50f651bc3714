"""The coarse term of Eq. 6 in batched solves (sem_batch_* with meshes that
carry a coarse space), against the oracle.

* every FP64 slot of a coarse mesh reaches a true relative residual <= 1e-10
  measured by the oracle, in about the iterations of the single-mesh solve
  with the same coarse space (the two sum the prolongation in different
  orders: the same preconditioner to rounding) and far fewer than Jacobi;
* several slots on one coarse mesh (their own coarse vectors) solve
  different right-hand sides correctly, and each keeps the bits of its
  alone-solve among Jacobi and coarse co-residents, by graph replay and by
  plain launches;
* mixed-precision slots of coarse meshes take the coarse term in their FP32
  inner iterations (fewer iterations than Jacobi, the oracle's residual, and
  their alone-solve bits among co-residents);
* continuous admission: coarse slots admitted while others run keep their
  alone-solve bits.
"""
import numpy as np
import pytest
import torch

import seeded_inputs as SI

pytestmark = pytest.mark.gpu


def _case(semlib, oracle_mod, N, nel, seed, coarse=True):
    V = SI.jittered_box_vertices(nel, seed=seed)
    m = semlib.box_mesh(N, nel, vertices=V, with_fp32=True)
    om = oracle_mod.OracleMesh(N, nel, vertices=V)
    gid = om.numbering()
    b = SI.uniform_global_values(om.nglob, seed)[gid]
    b[om.local_mask() == 1] = 0.0
    if coarse:
        m.set_coarse(4, 0.05)
    return m, om, b


CASES = [(5, (6, 5, 4), 31, True), (7, (5, 5, 5), 32, True), (9, (3, 4, 3), 33, True),
         (4, (8, 6, 5), 34, True), (7, (4, 3, 2), 35, False), (6, (3, 3, 3), 36, False)]


@pytest.fixture(scope="module")
def cases(semlib, oracle_mod):
    out = [_case(semlib, oracle_mod, N, nel, seed, c) for N, nel, seed, c in CASES]
    yield out
    for m, _, _ in out:
        m.close()


def test_batch_coarse_matches_oracle(semlib, cases):
    print(f"case: batched coarse FP64 over {len(cases)} meshes", flush=True)
    B = semlib.Batch(max_slots=16)
    meshes = [c[0] for c in cases]
    bs = [torch.from_numpy(c[2]).cuda() for c in cases]
    xs, res = B.solve(meshes, bs, tol=1e-10, poll_every=8)
    for (m, om, b), x, r, case in zip(cases, xs, res, CASES):
        rel = om.true_residual(b, x.cpu().numpy())
        assert r.ok and rel <= 1e-10, (case, r, rel)
        _, r1 = m.solve(torch.from_numpy(b).cuda(), tol=1e-10)
        print(f"  N={m.N} E={m.E} coarse={case[3]}: batch {r.iterations} it, single-mesh {r1.iterations} it, "
              f"oracle residual {rel:.2e}", flush=True)
        assert abs(r1.iterations - r.iterations) <= max(2, 0.05 * r1.iterations), (case, r.iterations, r1.iterations)
    # against Jacobi on the same meshes: the coarse term cuts the iterations
    jac = {}
    for (m, om, b), case in zip(cases, CASES):
        if case[3]:
            m.set_coarse(0)
            _, rj = m.solve(torch.from_numpy(b).cuda(), tol=1e-10)
            jac[case] = rj.iterations
            m.set_coarse(4, 0.05)
    for r, case in zip(res, CASES):
        if case[3]:
            assert r.iterations < jac[case], (case, r.iterations, jac[case])
    B.close()


def test_batch_coarse_shared_mesh_and_bits(semlib, cases):
    """Three slots on one coarse mesh with different right-hand sides, among
    Jacobi and other coarse slots: each meets the oracle and keeps the bits of
    its alone-solve; graph replay and plain launches agree bit for bit."""
    print("case: batched coarse, shared mesh, alone vs mixed", flush=True)
    m, om, b = cases[1]
    gid = om.numbering()
    rhs = [b]
    for seed in (41, 42):
        v = SI.uniform_global_values(om.nglob, seed)[gid]
        v[om.local_mask() == 1] = 0.0
        rhs.append(v)
    B = semlib.Batch(max_slots=16)
    alone = []
    for v in rhs:
        (x1,), (r1,) = B.solve([m], [torch.from_numpy(v).cuda()], tol=1e-10)
        alone.append((x1, r1.iterations))
    meshes = [m, cases[0][0], m, cases[4][0], m, cases[2][0]]
    bs = [torch.from_numpy(v).cuda() for v in (rhs[0], cases[0][2], rhs[1], cases[4][2], rhs[2], cases[2][2])]
    for use_graph in (True, False):
        xs, res = B.solve(meshes, bs, tol=1e-10, use_graph=use_graph, poll_every=5)
        for q, k in ((0, 0), (2, 1), (4, 2)):
            assert res[q].iterations == alone[k][1], (use_graph, q)
            assert torch.equal(xs[q], alone[k][0]), (use_graph, q)
            assert om.true_residual(rhs[k], xs[q].cpu().numpy()) <= 1e-10
    B.close()


def test_batch_coarse_mixed_slots(semlib, cases):
    """Mixed-precision slots of coarse meshes take the coarse term in their
    FP32 inner iterations: they meet the oracle in about the inner iterations
    of the single-mesh mixed solve with the coarse term, far fewer than with
    Jacobi, and keep their alone-solve bits among co-residents."""
    print("case: batched mixed slots with the coarse term", flush=True)
    B = semlib.Batch(max_slots=16)
    try:
        for q in range(4):
            m, om, b = cases[q]
            bd = torch.from_numpy(b).cuda()
            (x,), (r,) = B.solve([m], [bd], tol=1e-10, precision="mixed")
            assert r.ok and om.true_residual(b, x.cpu().numpy()) <= 1e-10
            _, r1 = m.solve(bd, tol=1e-10, precision="mixed")
            m.set_coarse(0)
            (xj,), (rj,) = B.solve([m], [bd], tol=1e-10, precision="mixed")
            m.set_coarse(4, 0.05)
            print(f"  N={m.N} E={m.E}: batch mixed + coarse {r.iterations} inner it, single-mesh {r1.iterations}, "
                  f"batch mixed Jacobi {rj.iterations}", flush=True)
            assert r.iterations < rj.iterations, (q, r.iterations, rj.iterations)
            assert abs(r.iterations - r1.iterations) <= max(3, 0.1 * r1.iterations), (q, r.iterations, r1.iterations)
            # among co-residents (FP64 and mixed, coarse and Jacobi): the same bits
            meshes = [cases[4][0], m, cases[5][0], cases[(q + 1) % 4][0]]
            bs = [torch.from_numpy(c[2]).cuda() for c in (cases[4], cases[q], cases[5], cases[(q + 1) % 4])]
            xs, res = B.solve(meshes, bs, tol=1e-10, precision="mixed")
            assert res[1].iterations == r.iterations and torch.equal(xs[1], x), q
    finally:
        B.close()


def test_batch_coarse_continuous_admission(semlib, cases):
    """Coarse slots admitted while others run: each equals its alone-solve."""
    print("case: batched coarse, continuous admission", flush=True)
    B = semlib.Batch(max_slots=8)
    alone = {}
    for q in range(4):
        m, om, b = cases[q]
        (x1,), (r1,) = B.solve([m], [torch.from_numpy(b).cuda()], tol=1e-10)
        alone[q] = (x1, r1.iterations)
    xs = {q: torch.zeros(cases[q][0].n_local, dtype=torch.float64, device="cuda") for q in range(4)}
    bs = {q: torch.from_numpy(cases[q][2]).cuda() for q in range(4)}
    slots = {}
    slots[0] = B.admit(cases[0][0], bs[0], xs[0], tol=1e-10)
    B.step(3)
    slots[1] = B.admit(cases[1][0], bs[1], xs[1], tol=1e-10)
    slots[2] = B.admit(cases[4][0], torch.from_numpy(cases[4][2]).cuda(),
                       torch.zeros(cases[4][0].n_local, dtype=torch.float64, device="cuda"), tol=1e-10)
    B.step(5)
    slots[3] = B.admit(cases[3][0], bs[3], xs[3], tol=1e-10)
    done = {}
    for _ in range(2000):
        B.step(4)
        for sl in B.finished():
            done[sl] = B.retire(sl)[1]
        if len(done) == 4:
            break
    assert len(done) == 4
    for q in (0, 1, 3):
        assert done[slots[q]].iterations == alone[q][1], q
        assert torch.equal(xs[q], alone[q][0]), q
    B.close()


def test_serving_with_coarse_term(semlib):
    """The serving loop with the coarse term on its larger catalog meshes:
    every request of a short Poisson stream completes with a true 1e-10
    residual (those of the larger meshes through the batched coarse term)."""
    print("case: serving loop with the coarse term", flush=True)
    from paper_2109_03592_amd.serve import serve_rates
    res = serve_rates([100.0], duration=1.5, max_requests=150, drain_limit=30.0, max_slots=32, budget_gb=8.0,
                      catalog=6, emin=8, emax=512, orders=(5, 7), iterations_per_step=8, tune=False,
                      coarse_min_elems=64)
    r = res[0]
    assert r["failed"] == 0 and r["unfinished"] == 0 and r["refused"] == 0, r
    assert r["completed"] == r["requests"] > 50 and r["coarse_min_elems"] == 64


def test_batch_coarse_slot_reuse_across_meshes(semlib, oracle_mod):
    """A slot and its cached buffers reused by a later admission on another
    coarse mesh (the first mesh already closed): the later solve must not
    replay the graph captured for the earlier admission -- each solve meets
    the oracle and equals its solve in a fresh batch, FP64 and mixed."""
    print("case: batched coarse slot reuse across meshes", flush=True)
    B = semlib.Batch(max_slots=8)
    try:
        for nel_a, nel_b in (((7, 7, 6), (7, 7, 7)), ((5, 5, 4), (6, 6, 6))):
            ms = {}
            for nel in (nel_a, nel_b):
                V = SI.jittered_box_vertices(nel, seed=sum(nel))
                m = semlib.box_mesh(5, nel, vertices=V, with_fp32=True)
                om = oracle_mod.OracleMesh(5, nel, vertices=V)
                b = SI.uniform_global_values(om.nglob, 80 + sum(nel))[om.numbering()]
                b[om.local_mask() == 1] = 0.0
                m.set_coarse(4, 0.05)
                ms[nel] = (m, om, b)
            for prec in ("fp64", "mixed"):
                m, om, b = ms[nel_a]
                for sc in (0.5, 1.0):
                    (xa,), (ra,) = B.solve([m], [torch.from_numpy(b * sc).cuda()], tol=1e-10, precision=prec)
                    assert ra.ok and om.true_residual(b * sc, xa.cpu().numpy()) <= 1e-10
            ms[nel_a][0].close()
            m, om, b = ms[nel_b]
            for prec in ("fp64", "mixed"):
                (xb,), (rb,) = B.solve([m], [torch.from_numpy(b).cuda()], tol=1e-10, precision=prec)
                assert rb.ok and om.true_residual(b, xb.cpu().numpy()) <= 1e-10, (nel_b, prec)
                F = semlib.Batch(max_slots=2)
                (xf,), (rf,) = F.solve([m], [torch.from_numpy(b).cuda()], tol=1e-10, precision=prec)
                F.close()
                assert rb.iterations == rf.iterations and torch.equal(xb, xf), (nel_b, prec)
            m.close()
    finally:
        B.close()
