#!/usr/bin/env python3
"""Benchmark of the SEM Poisson hot path on one MI355X.

Workload: the pipe-like mesh at one GPU's real share -- the square
[-1,1]^2 x [0,10] with 48 x 48 x 96 = 221,184 hexahedra of order N=7 mapped to
a circular pipe, periodic in z, Dirichlet wall, seeded uniform-random
right-hand side (one U[-1,1) value per global node, mean removed).  The
paper's own pipe meshes are not available; this synthetic mesh stands in.

A step is one Jacobi-PCG iteration in FP64: the local operator with the fused
search-direction update and p.Ap partials, the gather-scatter, alpha, the x/r
update with the Jacobi-weighted dot products, beta -- every row of the hot
path, one Ax+gs apply per step.  `value` = unique global nodes x steps /
seconds (GDOF/s).  Beside it the line reports the stand-alone Ax+gs apply rate
(FP64 and FP32), full FP64 and mixed-precision solves to a 1e-10 relative
residual, the roofline of the dominant kernel (measured with HIP events on the
launch stream inside the timed region) and the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

METRIC = "SEM Ax+gs GDOF/s & HBM % (FP64 vs mixed, 1e-10) + solves/s, p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_point(N: int, kind: str, dtype_bytes: int = 8) -> float:
    """Algorithmic HBM bytes per local point of one kernel launch."""
    if kind == "ax":          # read u, 6 geometric factors; write w
        return dtype_bytes * (1 + 6 + 1)
    if kind == "ax_pcg":      # read r, invdiag, p, x, 6 factors; write p, w, x
        return dtype_bytes * (4 + 6 + 3)
    if kind == "update":      # read r, w, invdiag, mult (1 B); write r
        return dtype_bytes * 4 + 1
    if kind == "ax_helm":     # plain operator + h1, h2*B
        return dtype_bytes * (1 + 6 + 2 + 1)
    if kind == "ax_pcg_helm":  # CG operator + h1, h2*B
        return dtype_bytes * (4 + 6 + 2 + 3)
    raise ValueError(kind)


def flops_per_point(N: int) -> int:
    """Operator flops per local point: 6 contractions of length N+1 (2 flops
    each) plus the 15-flop geometric combine."""
    return 12 * (N + 1) + 15


def gs_bytes(info, dtype_bytes: int = 8) -> float:
    """Gather-scatter: per shared local copy read index + read + write value;
    per shared global id one offset."""
    return info.n_shared_local * (4 + 2 * dtype_bytes) + info.n_shared_global * 4


# Sources the operator kernel is built from; the committed counter summary
# records their hash, and its traffic figure is used only while they match.
KERNEL_SOURCES = ("paper_2109_03592_amd/csrc/operator.hpp", "paper_2109_03592_amd/csrc/kernels.hip",
                  "paper_2109_03592_amd/csrc/kernels.hpp", "paper_2109_03592_amd/csrc/axgs_impl.hpp",
                  "paper_2109_03592_amd/csrc/axgs.hpp", "paper_2109_03592_amd/csrc/axgs64.hip",
                  "paper_2109_03592_amd/csrc/lattice.hpp")
TRAFFIC_PROFILES = {((48, 48, 96), 7): "profiles/hbm_traffic_pcg_pipe48x48x96_N7.txt",
                    ((48, 48, 48), 9): "profiles/hbm_traffic_pcg_pipe48x48x48_N9.txt"}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, nel, N: int, nL: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size),
    or None when the workload differs or the kernel sources changed since."""
    rel = TRAFFIC_PROFILES.get((tuple(nel), N))
    if rel is None or not os.path.exists(os.path.join(HERE, rel)):
        return None
    path = os.path.join(HERE, rel)
    digest, row = None, None
    with open(path) as fh:
        for line in fh:
            if line.startswith("# source_sha256"):
                digest = line.split()[-1]
            elif line.startswith(kernel + " "):
                row = line[len(kernel):].split()
    if digest != kernel_source_hash() or row is None:
        return None
    return (float(row[0]) + float(row[1])) * nL


def copy_calibration():
    """A plain device copy of known size (113,246,208 doubles read and
    written, three times) to scale the hardware byte counters."""
    import torch
    n = 113246208
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: {8 * n} bytes read and {8 * n} written per dispatch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds_target: float = 10.0, solve_iterations=None):
    """The oracle, as it stands, on the host cores.  `value`: FP64 Jacobi-PCG
    iterations on a 48x48x8 slab of the pipe (the step's unit, GDOF/s) with
    every OpenMP thread; beside it the full 48x48x96 pipe's Ax+gs apply
    (median of 3 on every thread, and one apply on 1 thread).  With
    `solve_iterations` (the FP64 solve's iteration count to 1e-10 on the
    full pipe), the full-pipe FP64 solve is stated as iterations x the slab's
    time per iteration scaled by the element count (96/8): a solve the oracle
    would take hours to run."""
    from oracle import oracle as O
    import seeded_inputs as SI
    threads = O.threads(0)
    out = {"unit": "GDOF/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
           "host_cpus": os.cpu_count()}
    nz = 8
    om = O.pipe_mesh(48, 48, nz, N=7)
    gid = om.numbering()
    b = SI.uniform_global_values(om.nglob, 2)[gid]
    b[om.local_mask() == 1] = 0.0
    om.geom()
    om.jacobi()
    # probe one iteration's cost, then size the run to the target
    t0 = time.perf_counter()
    om.pcg(b, tol=1e-30, max_iter=1)
    t1 = time.perf_counter() - t0
    iters = int(max(3, min(200, seconds_target / max(t1 / 3.0, 1e-3))))
    t0 = time.perf_counter()
    _, res = om.pcg(b, tol=1e-30, max_iter=iters)
    dt = time.perf_counter() - t0
    out["value"] = om.nglob * res.iterations / dt / 1e9
    if solve_iterations:
        s_it = dt / res.iterations * (96 / nz)
        out["full_pipe_fp64_solve_estimate"] = {
            "iterations": int(solve_iterations), "s_per_iteration": s_it, "seconds": s_it * solve_iterations,
            "basis": f"slab time per iteration (2 residual applies included) x 96/{nz} elements x the FP64 "
                     f"Jacobi-PCG iteration count to 1e-10 of the full-pipe solve"}
    sample = (f"pipe 48x48x{nz} N=7 ({om.E} elements, {om.nglob} global nodes), {res.iterations} FP64 "
              f"Jacobi-PCG iterations in {dt:.2f} s (plus 2 residual applies) on {threads} threads; "
              f"OpenMP over elements, gather-scatter and dots sequential")
    del om, b, gid
    # the full pipe: Ax+gs applies
    om = O.pipe_mesh(48, 48, 96, N=7)
    om.geom()
    om.numbering()
    u = SI.random_local(om.nloc, 3)
    om.apply(u)
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        om.apply(u)
        ts.append(time.perf_counter() - t0)
    t_all = sorted(ts)[1]
    O.threads(1)
    try:
        t0 = time.perf_counter()
        om.apply(u)
        t_one = time.perf_counter() - t0
    finally:
        O.threads(threads)
    out["axgs_full_pipe"] = {"gdofs": om.nglob / t_all / 1e9, "s_per_apply": t_all, "threads": threads,
                             "gdofs_1_thread": om.nglob / t_one / 1e9, "s_per_apply_1_thread": t_one,
                             "applies": "median of 3 (all threads), 1 (1 thread)"}
    out["sample"] = sample + (f"; full 48x48x96 pipe Ax+gs apply {t_all:.2f} s on {threads} threads "
                              f"(median of 3), {t_one:.2f} s on 1 thread")
    return out


def _event_mean(evs, stride, a, b, n):
    return float(np.mean([evs[stride * q + a].elapsed_time(evs[stride * q + b]) for q in range(n)])) / 1e3


def axgs_timing(mesh, info, N, torch, SI, stream, applies: int):
    """Stand-alone Ax+gs applies in FP64 and FP32 through sem_axgs, events
    around each apply (median); the library's default runs the operator and
    the gather-scatter as two launches, timed here also launch by launch; the
    opt-in fused operator + gather-scatter is timed beside it."""
    nL, nG = mesh.n_local, mesh.n_global
    res = {}

    def applies_ms(u, w):
        for _ in range(3):
            mesh.axgs(u, w)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * applies)]
        torch.cuda.synchronize()
        for q in range(applies):
            evs[2 * q].record(stream)
            mesh.axgs(u, w)
            evs[2 * q + 1].record(stream)
        torch.cuda.synchronize()
        return sorted(evs[2 * q].elapsed_time(evs[2 * q + 1]) for q in range(applies))[applies // 2] / 1e3

    for name, dt, eb in (("fp64", torch.float64, 8), ("fp32", torch.float32, 4)):
        u = torch.from_numpy(SI.random_local(nL, 3)).to(device="cuda", dtype=dt)
        w = torch.empty_like(u)
        byt = bytes_per_point(N, "ax", eb) * nL + gs_bytes(info, eb)
        tA = time.perf_counter()
        tot = applies_ms(u, w)
        wall = time.perf_counter() - tA
        # launch by launch
        for _ in range(3):
            mesh.ax(u, w)
            mesh.gs(w)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(3 * applies)]
        torch.cuda.synchronize()
        for q in range(applies):
            evs[3 * q].record(stream)
            mesh.ax(u, w)
            evs[3 * q + 1].record(stream)
            mesh.gs(w)
            evs[3 * q + 2].record(stream)
        torch.cuda.synchronize()
        t_ax = _event_mean(evs, 3, 0, 1, applies)
        t_gs = _event_mean(evs, 3, 1, 2, applies)
        r = {"gdofs": nG / tot / 1e9, "ms_per_apply": tot * 1e3, "hbm_frac": byt / tot / 1e9 / HBM_PEAK_GBS,
             "ms_ax": t_ax * 1e3, "ms_gs": t_gs * 1e3,
             "ax_gbs": bytes_per_point(N, "ax", eb) * nL / t_ax / 1e9, "gs_gbs": gs_bytes(info, eb) / t_gs / 1e9,
             "ax_tflops": flops_per_point(N) * nL / t_ax / 1e12, "algorithmic_bytes": byt, "applies": applies,
             "wall_s": wall, "timing": "median of per-apply events"}
        r["gs_kernel"] = "lattice" if mesh.gs_kind()[1] else "plan"
        if r["gs_kernel"] == "lattice":
            # the library streams whole element rows off the z-planes at N = 7
            # once there are 2048 row walks (element rows in y x interior planes)
            nel, per = list(mesh.desc.nel), list(mesh.desc.periodic)
            walks = (nel[1] if per[1] else nel[1] + 1) * (N - 1) * nel[2]
            if N == 7 and walks >= 2048:
                r["gs_kernel"] = "lattice, row-streaming off the z-planes"
        if r["gs_kernel"] == "lattice":
            # the CSR plan's gather-scatter on the same vector, for comparison
            mesh.set_gs_kind("plan")
            for _ in range(3):
                mesh.gs(w)
            evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * applies)]
            torch.cuda.synchronize()
            for q in range(applies):
                evs[2 * q].record(stream)
                mesh.gs(w)
                evs[2 * q + 1].record(stream)
            torch.cuda.synchronize()
            r["ms_gs_plan"] = _event_mean(evs, 2, 0, 1, applies) * 1e3
            mesh.set_gs_kind("auto")
        # the opt-in fused path (lines per workgroup chosen automatically)
        mesh.set_axgs_config(True)
        fused = mesh.axgs_info(dt)
        if fused["enabled"]:
            tf = applies_ms(u, w)
            r["fused"] = {"ms_per_apply": tf * 1e3, "hbm_frac": byt / tf / 1e9 / HBM_PEAK_GBS,
                          **{k: fused[k] for k in ("epw", "lines_per_wg", "y_onchip", "residual_ids",
                                                   "residual_copies")}}
        mesh.set_axgs_config(False)
        res[name] = r
        del u, w
    return res


def n9_section(sem, torch, SI, stream, args, nel=(48, 48, 48)):
    """The same pipe at N=9 (110,592 elements, 110.6M points): Ax+gs applies
    and profiled FP64 PCG iterations."""
    mesh = sem.pipe_mesh(*nel, N=9, with_fp32=True)
    info = mesh.info
    out = {"mesh": f"pipe {nel[0]}x{nel[1]}x{nel[2]} N=9", "E": mesh.E, "n_local": mesh.n_local,
           "n_global": mesh.n_global}
    out["ax_gs"] = axgs_timing(mesh, info, 9, torch, SI, stream, max(10, args.applies // 2))
    vg = torch.from_numpy(SI.uniform_global_values(mesh.n_global, 2)).cuda()
    b = mesh.scatter(vg)
    del vg
    x = mesh.zeros()
    mesh.solve(b, x, fixed_iters=max(1, args.warmup), profile=True, initial_guess=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = max(10, args.steps // 2)
    e0.record(stream)
    _, res = mesh.solve(b, x, fixed_iters=steps, profile=True, initial_guess=False)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / steps
    ax_ms = res.ms_operator / max(1, res.operator_launches)
    out["pcg"] = {"ms_per_iteration": t * 1e3, "gdofs": mesh.n_global / t / 1e9, "ms_operator": ax_ms,
                  "operator_gbs": bytes_per_point(9, "ax_pcg") * mesh.n_local / ax_ms / 1e6}
    a64, a32 = out["ax_gs"]["fp64"], out["ax_gs"]["fp32"]
    log(f"N=9 pipe: ax+gs fp64 {a64['gdofs']:.2f} GDOF/s ({a64['hbm_frac'] * 100:.1f}% HBM, ax "
        f"{a64['ax_gbs']:.0f} GB/s), fp32 {a32['gdofs']:.2f} GDOF/s; pcg {t * 1e3:.3f} ms/iteration "
        f"({out['pcg']['gdofs']:.2f} GDOF/s), operator {out['pcg']['operator_gbs']:.0f} GB/s")
    mesh.close()
    return out


def helmholtz_section(mesh, b, args, torch, SI, stream):
    """Helmholtz form (seeded h1 in [0.5, 2), h2 in [0, 3) per local point):
    stand-alone Ax+gs applies and profiled PCG iterations; the Poisson form is
    restored afterwards."""
    nL, nG, N = mesh.n_local, mesh.n_global, mesh.N
    h1 = torch.from_numpy(SI.uniform_local(nL, 41, 0.5, 2.0)).cuda()
    h2 = torch.from_numpy(SI.uniform_local(nL, 61, 0.0, 3.0)).cuda()
    mesh.set_helmholtz(h1, h2)
    del h1, h2
    u = torch.from_numpy(SI.random_local(nL, 3)).cuda()
    w = torch.empty_like(u)
    for _ in range(3):
        mesh.ax(u, w)
        mesh.gs(w)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(3 * args.applies)]
    torch.cuda.synchronize()
    for q in range(args.applies):
        evs[3 * q].record(stream)
        mesh.ax(u, w)
        evs[3 * q + 1].record(stream)
        mesh.gs(w)
        evs[3 * q + 2].record(stream)
    torch.cuda.synchronize()
    t_ax = np.mean([evs[3 * q].elapsed_time(evs[3 * q + 1]) for q in range(args.applies)]) / 1e3
    tot = evs[0].elapsed_time(evs[-1]) / 1e3 / args.applies
    del u, w
    x = mesh.zeros()
    mesh.solve(b, x, fixed_iters=max(1, args.warmup), profile=True, initial_guess=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    _, res = mesh.solve(b, x, fixed_iters=args.steps, profile=True, initial_guess=False)
    e1.record(stream)
    torch.cuda.synchronize()
    t_it = e0.elapsed_time(e1) / 1e3 / args.steps
    ax_ms = res.ms_operator / max(1, res.operator_launches)
    mesh.set_helmholtz(None, None)
    r = {"ax_gs_gdofs": nG / tot / 1e9, "ms_per_apply": tot * 1e3, "ms_ax": t_ax * 1e3,
         "ax_gbs": bytes_per_point(N, "ax_helm") * nL / t_ax / 1e9,
         "pcg_ms_per_iteration": t_it * 1e3, "pcg_gdofs": nG / t_it / 1e9,
         "pcg_operator_ms": ax_ms, "pcg_operator_gbs": bytes_per_point(N, "ax_pcg_helm") * nL / ax_ms / 1e6}
    log(f"helmholtz: ax+gs {r['ax_gs_gdofs']:.2f} GDOF/s (ax {t_ax * 1e3:.3f} ms, {r['ax_gbs']:.0f} GB/s); "
        f"pcg {t_it * 1e3:.3f} ms/iteration ({r['pcg_gdofs']:.2f} GDOF/s), operator {ax_ms:.3f} ms "
        f"({r['pcg_operator_gbs']:.0f} GB/s)")
    return r


def coarse_section(mesh, b, args, torch, stream, jacobi_solve=None):
    """Two-level preconditioners of Eq. 6 on the same mesh and right-hand
    side.  Each setting is "k:fraction" (Jacobi + coarse term with k Chebyshev
    steps on [fraction b, b]), "s" (Schwarz local solves only) or
    "s+k:fraction" (Schwarz + coarse): set-up time, profiled PCG iterations,
    a full FP64 solve to 1e-10 and, without Schwarz, a mixed one.  The mesh is
    back on Jacobi afterwards."""
    rows = []
    for item in args.coarse.split(","):
        schwarz = item.startswith("s")
        rest = item[2:] if item.startswith("s+") else ("" if schwarz else item)
        k, frac = (int(rest.split(":")[0]), float(rest.split(":")[1])) if rest else (0, 0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mesh.set_schwarz(schwarz)
        mesh.set_coarse(k, frac)
        t_build = time.perf_counter() - t0
        info = mesh.coarse_info()
        x = mesh.zeros()
        mesh.solve(b, x, fixed_iters=max(1, args.warmup), profile=True, initial_guess=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, res = mesh.solve(b, x, fixed_iters=args.steps, profile=True, initial_guess=False)
        e1.record(stream)
        torch.cuda.synchronize()
        t_it = e0.elapsed_time(e1) / 1e3 / args.steps
        n = max(1, res.operator_launches)
        mesh.solve(b, x, fixed_iters=args.steps, use_graph=True, poll_every=25, initial_guess=False)
        torch.cuda.synchronize()
        e0.record(stream)
        mesh.solve(b, x, fixed_iters=args.steps, use_graph=True, poll_every=25, initial_guess=False)
        e1.record(stream)
        torch.cuda.synchronize()
        t_graph = e0.elapsed_time(e1) / 1e3 / args.steps
        row = {"setting": item, "schwarz": schwarz, "chebyshev_steps": k, "fraction": frac,
               "n_coarse": info["n_coarse"], "cheb_b": info["b"], "setup_s": t_build,
               "ms_per_iteration": t_it * 1e3, "ms_per_iteration_graph": t_graph * 1e3,
               "ms_operator": res.ms_operator / n, "ms_gather_scatter": res.ms_gather_scatter / n,
               "ms_update_and_preconditioner": res.ms_update / n}
        msg = (f"precond {item}: set-up {t_build:.2f} s; {t_it * 1e3:.3f} ms/iteration ({t_graph * 1e3:.3f} graph; "
               f"operator {row['ms_operator']:.3f}, update+precond {row['ms_update_and_preconditioner']:.3f})")
        if args.no_solve:
            log(msg)
            rows.append(row)
            continue
        x = mesh.zeros()
        torch.cuda.synchronize()
        tS = time.perf_counter()
        _, r = mesh.solve(b, x, tol=1e-10, max_iter=40000, poll_every=50, initial_guess=False,
                          raise_on_error=False)
        torch.cuda.synchronize()
        ts = time.perf_counter() - tS
        row = {**row, "setting": item, "schwarz": schwarz, "chebyshev_steps": k, "fraction": frac,
               "n_coarse": info["n_coarse"], "cheb_b": info["b"], "setup_s": t_build,
               "ms_per_iteration": t_it * 1e3, "ms_per_iteration_graph": t_graph * 1e3,
               "ms_operator": res.ms_operator / n, "ms_gather_scatter": res.ms_gather_scatter / n,
               "ms_update_and_preconditioner": res.ms_update / n,
               "solve": {"status": r.status, "iterations": r.iterations, "rel_residual": r.rel_residual,
                         "seconds": ts}}
        if jacobi_solve:
            row["speedup_vs_jacobi"] = jacobi_solve["seconds"] / ts
            row["iteration_ratio_vs_jacobi"] = jacobi_solve["iterations"] / max(1, r.iterations)
        msg += f"; solve status={r.status} iters={r.iterations} rel_res={r.rel_residual:.2e} {ts:.2f} s"
        if not schwarz:
            x = mesh.zeros()
            torch.cuda.synchronize()
            tS = time.perf_counter()
            _, rm = mesh.solve(b, x, tol=1e-10, max_iter=40000, precision="mixed", inner_tol=1e-4,
                               poll_every=50, initial_guess=False, raise_on_error=False)
            torch.cuda.synchronize()
            tm = time.perf_counter() - tS
            row["solve_mixed"] = {"status": rm.status, "iterations": rm.iterations, "outer": rm.outer_iterations,
                                  "rel_residual": rm.rel_residual, "seconds": tm}
            msg += f"; mixed iters={rm.iterations} outer={rm.outer_iterations} {tm:.2f} s"
        log(msg)
        rows.append(row)
    mesh.set_coarse(0)
    mesh.set_schwarz(False)
    return rows


def sweep(sem, torch, SI, orders, sizes, applies: int = 20):
    """Ax+gs apply rate against order N and element count E on jittered boxes
    (the analogue of the paper's Nekbone sweeps, section 3): FP64 and FP32,
    GDOF/s and the algorithmic HBM fraction."""
    stream = torch.cuda.current_stream()
    rows = []
    for N in orders:
        for E in sizes:
            nel = SI.elements_from_target(E)
            m = sem.box_mesh(N, nel, vertices=SI.jittered_box_vertices(nel, seed=1), with_fp32=True)
            info = m.info
            row = {"N": N, "E": m.E, "nel": list(nel), "n_local": m.n_local, "n_global": m.n_global}
            for name, dt, eb in (("fp64", torch.float64, 8), ("fp32", torch.float32, 4)):
                u = torch.from_numpy(SI.random_local(m.n_local, 3)).to(device="cuda", dtype=dt)
                w = torch.empty_like(u)
                for _ in range(3):
                    m.ax(u, w)
                    m.gs(w)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record(stream)
                for _ in range(applies):
                    m.ax(u, w)
                    m.gs(w)
                e1.record(stream)
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1) / 1e3 / applies
                byt = bytes_per_point(N, "ax", eb) * m.n_local + gs_bytes(info, eb)
                row[name] = {"ms": t * 1e3, "gdofs": m.n_global / t / 1e9, "hbm_frac": byt / t / 1e9 / HBM_PEAK_GBS}
                del u, w
            m.close()
            rows.append(row)
            log(f"sweep N={N:2d} E={row['E']:6d}: fp64 {row['fp64']['gdofs']:7.2f} GDOF/s "
                f"({row['fp64']['hbm_frac'] * 100:5.1f}% HBM), fp32 {row['fp32']['gdofs']:7.2f} GDOF/s "
                f"({row['fp32']['hbm_frac'] * 100:5.1f}% HBM)")
    return rows


def oracle_error_section(sem, torch, SI, nel=(12, 12, 8), N: int = 7):
    """Each GPU solve's error against the FP64 oracle's solve of the same
    system: a 12x12x8 slab of the pipe (the full pipe's oracle solve would take
    hours on the host) with the oracle's own factors loaded into the library,
    the same seeded noise right-hand side; FP64 and mixed GPU solves and the
    oracle's Jacobi-PCG all to a 1e-10 relative residual.  Errors in the
    unique-dof 2-norm, relative to the oracle's solution; the oracle also
    measures each GPU solution's true residual."""
    from oracle import oracle as O
    om = O.pipe_mesh(*nel, N=N)
    G, B = om.geom()
    m = sem.pipe_mesh(*nel, N=N, with_fp32=True)
    m.load_geometry(G, B)
    del G, B
    gid = om.numbering()
    b = SI.uniform_global_values(om.nglob, 2)[gid]
    b[om.local_mask() == 1] = 0.0
    t0 = time.perf_counter()
    xo, ro = om.pcg(b, tol=1e-10, max_iter=20000)
    out = {"mesh": f"pipe {nel[0]}x{nel[1]}x{nel[2]} N={N}", "n_global": om.nglob,
           "oracle": {"iterations": ro.iterations, "rel_residual": ro.rel_residual,
                      "seconds": time.perf_counter() - t0, "threads": O.threads(0)}}
    bd = torch.from_numpy(b).cuda()
    no = np.sqrt(om.dot(xo, xo))
    for prec in ("fp64", "mixed"):
        x, r = m.solve(bd, tol=1e-10, max_iter=20000, precision=prec, raise_on_error=False)
        xh = x.cpu().numpy()
        d = xh - xo
        out[prec] = {"status": r.status, "iterations": r.iterations, "outer": r.outer_iterations,
                     "rel_error_vs_oracle": float(np.sqrt(om.dot(d, d)) / no),
                     "oracle_true_residual": float(om.true_residual(b, xh))}
    m.close()
    log(f"vs oracle ({out['mesh']}): fp64 error {out['fp64']['rel_error_vs_oracle']:.2e}, mixed error "
        f"{out['mixed']['rel_error_vs_oracle']:.2e} (oracle {ro.iterations} iterations, residual "
        f"{ro.rel_residual:.2e})")
    return out


def projection_section(sem, torch, SI, nel=(24, 24, 48), N: int = 7, solves: int = 6, vectors: int = 8):
    """Successive right-hand sides b_t = mass(sin(pi (x + 0.02 t)) sin(pi y) sin(pi z)),
    t = 0..solves-1, on a smaller pipe: FP64 solves to 1e-10 with projection
    onto previous solutions against the same solves from zero."""
    mesh = sem.pipe_mesh(*nel, N=N)
    xyz = torch.from_numpy(mesh.export_coords()).cuda()
    bs = []
    for t in range(solves):
        f = (torch.sin(np.pi * (xyz[0] + 0.02 * t)) * torch.sin(np.pi * xyz[1]) * torch.sin(np.pi * xyz[2]))
        bs.append(mesh.mass(f.contiguous()))
    del xyz
    out = {"mesh": f"pipe {nel[0]}x{nel[1]}x{nel[2]} N={N}", "n_global": mesh.n_global, "solves": solves,
           "max_vectors": vectors}
    mesh.solve(bs[0], tol=1e-10)   # warm-up (graph capture)
    for name in ("plain", "projected"):
        P = sem.Projection(mesh, vectors) if name == "projected" else None
        its, t_all = [], 0.0
        for b in bs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if P is None:
                _, r = mesh.solve(b, tol=1e-10, poll_every=25)
            else:
                _, r = P.solve(b, tol=1e-10, poll_every=25)
            torch.cuda.synchronize()
            t_all += time.perf_counter() - t0
            its.append(r.iterations)
        if P is not None:
            P.close()
        out[name] = {"iterations": its, "seconds": t_all}
    out["speedup"] = out["plain"]["seconds"] / out["projected"]["seconds"]
    log(f"projection: iterations plain {out['plain']['iterations']} vs projected {out['projected']['iterations']}; "
        f"{out['plain']['seconds']:.2f} s vs {out['projected']['seconds']:.2f} s ({out['speedup']:.2f}x)")
    mesh.close()
    return out


def batched_section(sem, torch, SI):
    """64 independent jittered box meshes (seeds 100+i) solved together,
    FP64 and mixed, after the autotuner; aggregate throughput."""
    cases = SI.batched_box_cases(64)
    meshes, bs = [], []
    t0 = time.perf_counter()
    for c in cases:
        m = sem.box_mesh(c.N, c.nel, vertices=SI.jittered_box_vertices(c.nel, seed=c.seed), with_fp32=True)
        xyz = torch.from_numpy(m.export_coords()).cuda()
        f = 3.0 * np.pi ** 2 * torch.sin(np.pi * xyz[0]) * torch.sin(np.pi * xyz[1]) * torch.sin(np.pi * xyz[2])
        meshes.append(m)
        bs.append(m.mass(f))
    t_setup = time.perf_counter() - t0
    B = sem.Batch(max_slots=64)
    t0 = time.perf_counter()
    B.tune(meshes)
    t_tune = time.perf_counter() - t0
    res = {"meshes": len(meshes), "elements": int(sum(m.E for m in meshes)),
           "local_nodes": int(sum(m.n_local for m in meshes)), "global_nodes": int(sum(m.n_global for m in meshes)),
           "orders": sorted({m.N for m in meshes}), "setup_s": t_setup, "tune_s": t_tune,
           "epw": {int(N): B.epw(N) for N in sorted({m.N for m in meshes})},
           "epw_fp32": {int(N): B.epw(N, "fp32") for N in sorted({m.N for m in meshes})}}
    for prec in ("fp64", "mixed"):
        B.solve(meshes, bs, tol=1e-10, precision=prec, poll_every=16)   # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, rs = B.solve(meshes, bs, tol=1e-10, precision=prec, poll_every=16, raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = sum(r.ok and r.rel_residual <= 1e-10 for r in rs)
        dof_iters = sum(m.n_global * r.iterations for m, r in zip(meshes, rs))
        res[prec] = {"seconds": dt, "solves_per_s": len(meshes) / dt, "converged": ok,
                     "iterations_max": max(r.iterations for r in rs), "iterations_sum": sum(r.iterations for r in rs),
                     "gdofs_aggregate": dof_iters / dt / 1e9}
        log(f"batched {prec}: {len(meshes)} solves in {dt:.3f} s ({len(meshes) / dt:.1f} solves/s), "
            f"{ok} converged, aggregate {res[prec]['gdofs_aggregate']:.2f} GDOF/s")
    # FP64 and mixed with the coarse term of Eq. 6 on the meshes of 512 elements or more
    big = [m for m in meshes if m.E >= 512]
    t0 = time.perf_counter()
    for m in big:
        m.set_coarse(4, 0.05)
    t_coarse = time.perf_counter() - t0
    for prec in ("fp64", "mixed"):
        B.solve(meshes, bs, tol=1e-10, precision=prec, poll_every=16)   # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, rs = B.solve(meshes, bs, tol=1e-10, precision=prec, poll_every=16, raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = sum(r.ok and r.rel_residual <= 1e-10 for r in rs)
        key = f"{prec}_coarse"
        res[key] = {"seconds": dt, "solves_per_s": len(meshes) / dt, "converged": ok,
                    "coarse_meshes": len(big), "coarse_setup_s": t_coarse,
                    "iterations_max": max(r.iterations for r in rs),
                    "iterations_sum": sum(r.iterations for r in rs)}
        log(f"batched {prec} + coarse term on {len(big)} meshes: {dt:.3f} s ({len(meshes) / dt:.1f} solves/s), "
            f"{ok} converged, iterations max {res[key]['iterations_max']}")
    for m in big:
        m.set_coarse(0)
    # steady CG iteration rate with every slot active (tolerances no run reaches)
    for prec in ("fp64", "mixed"):
        xs = [m.zeros() for m in meshes]
        slots = [B.admit(m, b, x, tol=1e-300, max_iter=10 ** 6, precision=prec, inner_tol=1e-30,
                         inner_max_iter=10 ** 6) for m, b, x in zip(meshes, bs, xs)]
        B.step(16)
        B.step(16)
        torch.cuda.synchronize()
        reps = 8
        t0 = time.perf_counter()
        for _ in range(reps):
            B.step(16)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / (16 * reps)
        live = len(slots) - len(B.finished())
        for sl in slots:
            B.retire(sl)
        key = f"steady_{prec}"
        res[key] = {"ms_per_iteration": dt * 1e3, "active": live,
                    "gdofs": res["global_nodes"] / dt / 1e9,
                    "local_points_per_s": res["local_nodes"] / dt}
        log(f"batched steady {prec}: {dt * 1e3:.3f} ms per iteration of all {live} slots -> "
            f"{res[key]['gdofs']:.2f} GDOF/s ({res['local_nodes'] / dt / 1e9:.2f} G local points/s)")
    B.close()
    for m in meshes:
        m.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nel", type=int, nargs=3, default=(48, 48, 96))
    ap.add_argument("--order", type=int, default=7)
    ap.add_argument("--applies", type=int, default=100, help="stand-alone Ax+gs applies")
    ap.add_argument("--no-solve", action="store_true", help="skip the full FP64 / mixed solves")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-axgs", action="store_true", help="skip the stand-alone Ax+gs timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64-mesh solves")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--no-helm", action="store_true", help="skip the Helmholtz-form timing")
    ap.add_argument("--coarse-smooth", default="4:0.05",
                    help="the same preconditioner settings on a smooth right-hand side (sin forcing)")
    ap.add_argument("--coarse", default="4:0.05,s+4:0.05",
                    help="preconditioner settings: k:fraction (Jacobi + coarse), s (Schwarz), s+k:fraction "
                         "(Schwarz + coarse), comma-separated ('' skips)")
    ap.add_argument("--no-proj", action="store_true", help="skip the successive-RHS projection timing")
    ap.add_argument("--no-n9", action="store_true", help="skip the N=9 pipe (48x48x48)")
    ap.add_argument("--serve-rates", default="10,100,1000")
    ap.add_argument("--serve-duration", type=float, default=5.0)
    ap.add_argument("--serve-coarse-min-elems", type=int, default=512,
                    help="serving: meshes of at least this many elements carry the coarse term (0: Jacobi only)")
    ap.add_argument("--serve-drain", type=float, default=20.0)
    ap.add_argument("--sweep", action="store_true",
                    help="only run the Ax+gs sweep over orders and element counts (one JSON line)")
    ap.add_argument("--sweep-orders", default="2,3,4,5,6,7,8,9,10,11,12,13,14,15,16,17")
    ap.add_argument("--sweep-sizes", default="32,256,2048,16384")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain copy of known size (for scaling byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this engine has no multi-GPU path (one GPU's share of the "
              "pipe is the workload); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2109_03592_amd as sem
    import seeded_inputs as SI

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.sweep:
        import paper_2109_03592_amd as sem
        import seeded_inputs as SI
        rows = sweep(sem, torch, SI, [int(v) for v in args.sweep_orders.split(",")],
                     [int(v) for v in args.sweep_sizes.split(",")])
        print(json.dumps({"sweep": rows}), flush=True)
        return
    stream = torch.cuda.current_stream()
    nx, ny, nz = args.nel
    N = args.order
    t0 = time.perf_counter()
    mesh = sem.pipe_mesh(nx, ny, nz, N=N, with_fp32=True)
    info = mesh.info
    log(f"setup: E={mesh.E} N={N} n_local={mesh.n_local} n_global={mesh.n_global} "
        f"({time.perf_counter() - t0:.1f} s, {info.device_bytes / 2**30:.1f} GiB on device)")
    vg = torch.from_numpy(SI.uniform_global_values(mesh.n_global, 2)).cuda()
    b = mesh.scatter(vg)
    del vg
    nL, nG = mesh.n_local, mesh.n_global

    # ---- K timed PCG iterations (the steps) --------------------------------
    x = mesh.zeros()
    mesh.solve(b, x, fixed_iters=max(1, args.warmup), profile=True, initial_guess=False)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    _, res = mesh.solve(b, x, fixed_iters=args.steps, profile=True, initial_guess=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_steps = ev0.elapsed_time(ev1) / 1e3
    value = nG * args.steps / t_steps / 1e9
    ax_ms = res.ms_operator / max(1, res.operator_launches)
    gs_ms = res.ms_gather_scatter / max(1, res.operator_launches)
    up_ms = res.ms_update / max(1, res.operator_launches)
    log(f"pcg steps: {args.steps} in {t_steps * 1e3:.1f} ms -> {value:.2f} GDOF/s; per iteration "
        f"operator {ax_ms:.3f} ms, gs {gs_ms:.3f} ms, update {up_ms:.3f} ms")
    # graph-replayed iterations (no per-kernel events); the same call once
    # untimed first, so that the graph of this iteration count is captured
    # and instantiated outside the timed region
    mesh.solve(b, x, fixed_iters=args.steps, use_graph=True, poll_every=25, initial_guess=False)
    torch.cuda.synchronize()
    ev0.record(stream)
    mesh.solve(b, x, fixed_iters=args.steps, use_graph=True, poll_every=25, initial_guess=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_graph = ev0.elapsed_time(ev1) / 1e3

    # the dominant kernel: the CG operator, fused with the gather-scatter of
    # the ids a workgroup holds where that path runs; achieved counts only the
    # operator's own streams (r, D^-1, p, x, 6 factors read; p, w, x written)
    fused = mesh.axgs_info()
    kname = (f"axgs_kernel<double, {N}, 2, false>" if fused["enabled"] else f"ax_kernel<double, {N}, 2, false>")
    ax_bytes = bytes_per_point(N, "ax_pcg") * nL
    roof = {"bound": "hbm", "kernel": kname,
            "achieved": ax_bytes / (ax_ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "traffic": measured_traffic(kname, (nx, ny, nz), N, nL),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "algorithmic_bytes_per_launch": ax_bytes, "ms_per_launch": ax_ms}
    roof["frac"] = roof["achieved"] / roof["peak"]
    step_bytes = ax_bytes + gs_bytes(info) + bytes_per_point(N, "update") * nL
    # as run: with the gather-scatter folded into the update there is no gs
    # pass; the iteration needs the operator's and the update's bytes only
    gs_folded = mesh.gs_kind()[1] and N >= 3 and not fused["enabled"]
    step_bytes_run = ax_bytes + bytes_per_point(N, "update") * nL + (0 if gs_folded else gs_bytes(info))
    upd_name = f"pcg_update_gs_kernel<double, {N}>" if gs_folded else f"pcg_update_elem_kernel<double, {N}>"
    upd_traffic = measured_traffic(upd_name, (nx, ny, nz), N, nL)

    out = {
        "metric": METRIC, "value": value, "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_steps / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"pipe {nx}x{ny}x{nz} N={N} FP64 Jacobi-PCG iteration (one Ax+gs apply each)",
                   "E": mesh.E, "N": N, "n_local": nL, "n_global": nG},
        "roofline": roof,
        "step": {"ms_operator": ax_ms, "ms_gather_scatter": gs_ms, "ms_update_reduce": up_ms,
                 "gather_scatter": ("summed in the update (lattice)"
                                    if mesh.gs_kind()[1] and N >= 3 and not fused["enabled"]
                                    else ("lattice" if mesh.gs_kind()[1] else "plan")),
                 "fused_operator_gs": fused,
                 "hbm_frac_step": step_bytes / (t_steps / args.steps) / 1e9 / HBM_PEAK_GBS,
                 "algorithmic_bytes_per_step": step_bytes,
                 "algorithmic_bytes_per_step_as_run": step_bytes_run,
                 "bytes_per_point_as_run": step_bytes_run / nL,
                 "hbm_frac_step_as_run": step_bytes_run / (t_steps / args.steps) / 1e9 / HBM_PEAK_GBS,
                 "measured_bytes_per_step": (roof["traffic"] + upd_traffic
                                             if roof["traffic"] is not None and upd_traffic is not None else None),
                 "ms_per_step_graph": t_graph / args.steps * 1e3,
                 "gdofs_graph": nG * args.steps / t_graph / 1e9},
    }

    # ---- stand-alone Ax+gs applies (FP64 and FP32) ---------------------------
    if not args.no_axgs:
        axgs = axgs_timing(mesh, info, N, torch, SI, stream, args.applies)
        for name in ("fp64", "fp32"):
            a = axgs[name]
            log(f"ax+gs {name}: {a['gdofs']:.2f} GDOF/s, {a['ms_per_apply']:.3f} ms/apply, "
                f"ax {a['ms_ax']:.3f} ms ({a['ax_gbs']:.0f} GB/s), gs {a['ms_gs']:.3f} ms, "
                f"HBM {a['hbm_frac'] * 100:.1f}%; fused {a.get('fused')}")
        out["ax_gs"] = axgs

    # ---- full solves to 1e-10: FP64 and mixed --------------------------------
    if not args.no_solve:
        sol = {}
        for prec in ("fp64", "mixed"):
            x = mesh.zeros()
            torch.cuda.synchronize()
            tS = time.perf_counter()
            _, r = mesh.solve(b, x, tol=1e-10, max_iter=40000, precision=prec, inner_tol=1e-4,
                              poll_every=50, initial_guess=False, raise_on_error=False)
            torch.cuda.synchronize()
            ts = time.perf_counter() - tS
            sol[prec] = {"status": r.status, "iterations": r.iterations, "outer": r.outer_iterations,
                         "rel_residual": r.rel_residual, "seconds": ts, "solves_per_s": 1.0 / ts}
            log(f"solve {prec}: status={r.status} iters={r.iterations} outer={r.outer_iterations} "
                f"rel_res={r.rel_residual:.2e} {ts:.2f} s")
            if prec == "fp64":
                x64 = x.clone()
            else:
                d = (x - x64)
                err = float(torch.linalg.norm(d) / torch.linalg.norm(x64))
                sol[prec]["rel_diff_vs_fp64"] = err
        sol["mixed_speedup"] = sol["fp64"]["seconds"] / sol["mixed"]["seconds"]
        if not args.no_cpu:
            sol["vs_fp64_oracle"] = oracle_error_section(sem, torch, SI)
        out["solve"] = sol

    # ---- the preconditioners of Eq. 6 (coarse term, Schwarz local solves) ------
    if args.coarse:
        out["coarse"] = coarse_section(mesh, b, args, torch, stream,
                                       out.get("solve", {}).get("fp64"))
    if args.coarse_smooth:
        # a smooth right-hand side: b = mask(Q Q^T B f), f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z)
        xyz = mesh.export_coords()
        f = torch.from_numpy(SI.sin3_forcing(xyz[0], xyz[1], xyz[2])).cuda()
        del xyz
        bs = mesh.empty()
        mesh.mass(f, bs)
        del f
        base = None
        if not args.no_solve:
            x = mesh.zeros()
            torch.cuda.synchronize()
            tS = time.perf_counter()
            _, r = mesh.solve(bs, x, tol=1e-10, max_iter=40000, poll_every=50, initial_guess=False,
                              raise_on_error=False)
            torch.cuda.synchronize()
            base = {"status": r.status, "iterations": r.iterations, "seconds": time.perf_counter() - tS}
            log(f"smooth rhs, Jacobi: iters={r.iterations} {base['seconds']:.2f} s")
        saved = args.coarse
        args.coarse = args.coarse_smooth
        out["coarse_smooth_rhs"] = {"jacobi": base, "settings": coarse_section(mesh, bs, args, torch, stream, base)}
        args.coarse = saved
        del bs

    # ---- Helmholtz form (h1-weighted stiffness + h2 B) on the same mesh ------
    if not args.no_helm:
        out["helmholtz"] = helmholtz_section(mesh, b, args, torch, SI, stream)

    # ---- successive right-hand sides with projection onto previous solutions ----
    if not args.no_proj:
        out["projection"] = projection_section(sem, torch, SI)

    # ---- the pipe at N=9 (48x48x48) ------------------------------------------
    if not args.no_n9:
        del b
        mesh.close()
        out["pipe_n9"] = n9_section(sem, torch, SI, stream, args)

    # ---- batched: 64 jittered boxes, E log-uniform in [8, 4096], N in {5,7,9} ----
    if not args.no_batch:
        out["batched"] = batched_section(sem, torch, SI)

    # ---- serving: Poisson arrivals of mixed-size solves -------------------------
    if not args.no_serve:
        from paper_2109_03592_amd.serve import serve_rates
        out["serving"] = serve_rates([float(v) for v in args.serve_rates.split(",")], duration=args.serve_duration,
                                     max_requests=2000, drain_limit=args.serve_drain, max_slots=64, budget_gb=200.0,
                                     coarse_min_elems=args.serve_coarse_min_elems)

    # ---- CPU oracle on a bounded sample ---------------------------------------
    if not args.no_cpu:
        log("cpu baseline: oracle on a pipe slab ...")
        its = out.get("solve", {}).get("fp64", {}).get("iterations")
        out["cpu_baseline"] = cpu_baseline(solve_iterations=its)
        cb = out["cpu_baseline"]
        if "full_pipe_fp64_solve_estimate" in cb:
            e = cb["full_pipe_fp64_solve_estimate"]
            log(f"cpu baseline: full-pipe FP64 solve ~ {e['iterations']} it x {e['s_per_iteration']:.2f} s "
                f"= {e['seconds'] / 3600:.1f} h")
        log(f"cpu baseline ({cb['cpu_model']}, {cb['cores']} threads): PCG {cb['value']:.4f} GDOF/s; "
            f"full-pipe Ax+gs {cb['axgs_full_pipe']['gdofs']:.4f} GDOF/s, 1 thread "
            f"{cb['axgs_full_pipe']['gdofs_1_thread']:.4f} GDOF/s")

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
