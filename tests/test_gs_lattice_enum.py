"""Host check of the plan-free gather-scatter's node enumeration and copy
offsets (csrc/lattice.hpp, the functions the kernels call), CPU only: see
lattice_enum_check.cpp for what is checked."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_lattice_enumeration_covers_every_copy_once(tmp_path):
    from paper_2109_03592_amd import build as B
    exe = tmp_path / "lattice_enum_check"
    src = os.path.join(ROOT, "tests", "lattice_enum_check.cpp")
    subprocess.run([B.HIPCC, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", src, "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
