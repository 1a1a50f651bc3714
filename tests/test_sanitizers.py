"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (sem_oracle.c) is built with gcc and -fsanitize=address,undefined
  and runs meshes of every periodicity, the pipe map, the operator, the
  gather-scatter, Jacobi and PCG in a child process with gcc's sanitizer
  runtimes preloaded.
* The library's host side (setup.cpp: GLL rule, coordinates, geometric
  factors, numbering, gather-scatter plan, Jacobi diagonal; api.cpp's host
  entry points; batch.cpp's slot layout; axgs.cpp's residual plan) is rebuilt
  with the sanitizers on the host pass only -- hipcc takes -Xarch_host before
  each sanitizer flag, device code is the normal build's -- linked into a
  separate copy of the library, and driven through the C ABI's host-only
  entry points with clang's sanitizer runtime preloaded.  No GPU call is made.

Any sanitizer report fails the test (UBSan halts on the first error).
"""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_SOURCES = ["setup.cpp", "api.cpp", "batch.cpp", "axgs.cpp"]


def _sanitize_flags():
    flags = []
    for kind in ("address", "undefined"):
        flags += ["-Xarch_host", "-fsanitize=" + kind]
    flags += ["-Xarch_host", "-fno-sanitize-recover=undefined"]
    return flags


def _run_child(code, env_extra, tmp_path):
    script = tmp_path / "child.py"
    script.write_text(textwrap.dedent(code))
    env = dict(os.environ)
    env.update(env_extra)
    env["PYTHONPATH"] = os.pathsep.join([ROOT, os.path.join(ROOT, "tests")])
    r = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert "CHILD OK" in out, out[-4000:]


def test_oracle_under_asan_ubsan(tmp_path):
    so = tmp_path / "liboracle_san.so"
    src = os.path.join(ROOT, "oracle", "sem_oracle.c")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                    "-o", str(so), src, "-lm"], check=True)
    rt = [subprocess.run(["gcc", "-print-file-name=" + n], capture_output=True, text=True).stdout.strip()
          for n in ("libasan.so", "libubsan.so")]
    assert all(os.path.isabs(p) and os.path.exists(p) for p in rt), rt
    _run_child(f"""
        import numpy as np
        from oracle import oracle as O
        O._SO = {str(so)!r}
        import seeded_inputs as SI
        for N, nel, per in ((1, (2, 2, 2), (0, 0, 0)), (4, (3, 2, 2), (0, 0, 1)), (7, (2, 3, 2), (1, 1, 0)),
                            (3, (2, 2, 2), (1, 1, 1))):
            V = None if any(per) else SI.jittered_box_vertices(nel, seed=N)
            om = O.OracleMesh(N, nel, vertices=V, periodic=per)
            x, y, z = om.coords()
            b = om.mass(SI.sin3_forcing(x, y, z))
            u = SI.random_local(om.nloc, 3)
            om.apply(u)
            om.jacobi()
            if not all(per):  # the all-periodic operator is singular: apply only
                xs, r = om.pcg(b, tol=1e-10, max_iter=2000)
                assert r.status == 0 and om.true_residual(b, xs) <= 1e-10
        om = O.pipe_mesh(4, 4, 2, N=5)
        om.geom()
        om.apply(SI.random_local(om.nloc, 4))
        print("CHILD OK")
        """, {"LD_PRELOAD": ":".join(rt), "ASAN_OPTIONS": "detect_leaks=0",
              "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1", "OMP_NUM_THREADS": "2"}, tmp_path)


def _build_host_sanitized(out_dir):
    from paper_2109_03592_amd import build as B
    if not all(os.path.exists(os.path.join(B.BUILD, s + ".o")) for s in B.SOURCES):
        B.build()
    flags = [f for f in B.COMMON if f != "-O3"] + ["-O1", "-g", "-fno-omit-frame-pointer"] + _sanitize_flags()
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(out_dir, src + ".san.o")
        r = subprocess.run([B.HIPCC, *flags, "-x", "hip", "-c", os.path.join(B.CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        objs.append(obj)
    dev = [os.path.join(B.BUILD, s + ".o") for s in B.SOURCES if s not in HOST_SOURCES]
    lib = os.path.join(out_dir, "libsem_hostsan.so")
    r = subprocess.run([B.HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *dev, *objs, "-o", lib],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return lib


def test_library_host_side_under_asan_ubsan(tmp_path):
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rts:
        pytest.skip("no clang sanitizer runtime under /opt/rocm/llvm")
    lib = _build_host_sanitized(str(tmp_path))
    _run_child(f"""
        import ctypes as C
        import numpy as np
        from paper_2109_03592_amd import _lib as L
        L.LIB_PATH = {lib!r}
        from libhost import host_setup, make_desc
        lib = L.load()
        for N, nel, per, mp in ((1, (2, 2, 2), (0, 0, 0), 0), (5, (3, 2, 4), (0, 0, 1), 0),
                                (7, (4, 4, 3), (0, 0, 1), 1), (12, (2, 1, 2), (1, 1, 0), 0),
                                (3, (2, 2, 1), (1, 1, 1), 0)):
            kw = dict(periodic=per)
            if mp:
                kw.update(lo=(-1, -1, 0), hi=(1, 1, 1), mapping=1)
            out = host_setup(N, nel, **kw)
            assert out["mult"].min() >= 1 and np.all(out["inv"] >= 0)
            d, keep = make_desc(L, N, nel, **kw)
            for lines in (1, 2, 5):
                for yon in (0, 1):
                    a, b = C.c_int64(0), C.c_int64(0)
                    L.check(lib.sem_host_axgs_residual(C.byref(d), lines, yon, C.byref(a), C.byref(b), None, None),
                            "residual sizes")
                    off = np.zeros(a.value + 1, np.int32)
                    idx = np.zeros(max(b.value, 1), np.int32)
                    L.check(lib.sem_host_axgs_residual(C.byref(d), lines, yon, C.byref(a), C.byref(b),
                                                       off.ctypes.data, idx.ctypes.data), "residual plan")
        # rejected descriptors take the error paths
        d, keep = make_desc(L, 0, (2, 2, 2))
        info = L.MeshInfo()
        assert lib.sem_host_setup(C.byref(d), C.byref(info), None, None, None, None, None, None, None, None) != 0
        off = np.zeros(7, np.uint64)
        tot = C.c_size_t(0)
        for nl in (1, 27, 4096 * 1000):
            for prec in (0, 1):
                L.check(lib.sem_batch_slot_layout(C.c_int64(nl), prec, off.ctypes.data, C.byref(tot)), "layout")
        for N in (2, 7, 12):
            P = N + 1
            S = np.zeros((N + 3) ** 2)
            lam = np.zeros(N + 3)
            lo, cnt = C.c_int(), C.c_int()
            for left in (0, 1, 2):
                for right in (0, 1, 2):
                    L.check(lib.sem_host_fdm_1d(N, 0.3, left, right, S.ctypes.data, lam.ctypes.data,
                                                C.byref(lo), C.byref(cnt)), "fdm")
            xi, w, D = np.zeros(P), np.zeros(P), np.zeros(P * P)
            L.check(lib.sem_export_gll(N, xi.ctypes.data, w.ctypes.data, D.ctypes.data), "gll")
        print("CHILD OK")
        """, {"LD_PRELOAD": rts[-1], "ASAN_OPTIONS": "detect_leaks=0:protect_shadow_gap=0",
              "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}, tmp_path)
