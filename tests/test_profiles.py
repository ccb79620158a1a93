"""The committed rocprofv3 summaries under profiles/ describe the kernels in
the tree: each names the hash of the kernel sources it was measured with,
and that hash must be the one of the current sources (the multiple-shooting
summaries hash mc_ms.hpp too).  bench.py reports the measured HBM traffic
only under that condition, so this also checks that the bench line's
roofline.traffic is available."""
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

import sys  # noqa: E402

sys.path.insert(0, ROOT)
import bench  # noqa: E402

HASH = re.compile(r"(?:kernel source sha256|source_sha256)( \(with mc_ms\.hpp\))? ([0-9a-f]{64})")
SUMMARIES = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt")))


def test_profiles_exist():
    names = {os.path.basename(p) for p in SUMMARIES}
    for need in ("nmpc_kernel_c1_kernel_trace.txt", "nmpc_kernel_c1_hbm_traffic.txt",
                 "nmpc_ms_kernel_c1_kernel_trace.txt", "pi_kernels_c2_trace_traffic.txt"):
        assert need in names


@pytest.mark.parametrize("path", SUMMARIES, ids=os.path.basename)
def test_summary_matches_the_kernel_sources(path):
    text = open(path).read()
    found = HASH.findall(text)
    assert found, "no source hash in " + path
    for with_ms, h in found:
        assert h == bench.kernel_source_sha256(multiple_shooting=bool(with_ms)), path
    # every summary gives the command that produced it
    assert "rocprofv3" in text


def test_bench_reads_the_committed_traffic():
    t = bench.measured_traffic()
    assert t is not None and t > 0
    text = open(os.path.join(ROOT, "profiles", "nmpc_kernel_c1_hbm_traffic.txt")).read()
    m = re.search(r"traffic_bytes_per_launch ([0-9.e+]+)", text)
    assert float(m.group(1)) == t
