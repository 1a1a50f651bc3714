"""The committed rocprofv3 summaries against the sources and the bench (CPU).

bench.py reports the roofline's measured traffic only while the counter
summary it reads was taken on the current kernel sources (their sha256 is
recorded in the summary).  These checks keep that link: every traffic
summary names the command that made it, records the hash of today's kernel
sources, and yields the dominant kernel's bytes per launch for its workload.
"""
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("key", sorted(bench.TRAFFIC_PROFILES))
def test_traffic_summary_matches_sources(key):
    nel, N = key
    path = os.path.join(ROOT, bench.TRAFFIC_PROFILES[key])
    text = open(path).read()
    assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
    digest = [ln.split()[-1] for ln in text.splitlines() if ln.startswith("# source_sha256")]
    assert digest == [bench.kernel_source_hash()], "kernel sources changed since the counters were taken"
    nL = nel[0] * nel[1] * nel[2] * (N + 1) ** 3
    t = bench.measured_traffic(f"ax_kernel<double, {N}, 2, false>", nel, N, nL)
    assert t is not None
    # the CG operator moves at least its algorithmic bytes
    assert t >= bench.bytes_per_point(N, "ax_pcg") * nL * 0.999


def test_traffic_lookup_declines_other_workloads():
    assert bench.measured_traffic("ax_kernel<double, 7, 2, false>", (24, 24, 48), 7, 1000) is None


def test_profiles_name_their_commands():
    for f in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        text = open(os.path.join(ROOT, "profiles", f)).read()
        assert "bench.py" in text, f
