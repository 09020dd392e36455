"""Host-side checks of bench.py (no GPU): the one-GPU refusal of the command line, and that the
roofline's traffic figure is taken only from a PMC record of the current kernel source and the
launch shape the run picked."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SF_SOURCES = ["sparse_filter.hip", "sparse_device.hpp", "rosar_device.hpp"]


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""   # no JSON line


def test_kernel_source_digest_is_stable_and_source_sensitive():
    d1 = bench.kernel_source_digest(SF_SOURCES)
    assert d1 == bench.kernel_source_digest(SF_SOURCES) and len(d1) == 16
    assert d1 != bench.kernel_source_digest(SF_SOURCES[:2])


def test_traffic_record_matches_digest_and_shape():
    path = os.path.join(ROOT, "profiles", "sparse_filter_rotation_traffic.json")
    with open(path) as f:
        rec = json.load(f)
    digest = bench.kernel_source_digest(SF_SOURCES)
    shape = sorted(rec["by_shape"])[0]
    want = rec["by_shape"][shape]["traffic_bytes_per_launch"]
    if rec["kernel_source_digest"] == digest:
        assert bench.load_traffic("sparse_filter", digest, "rotation", shape) == want
    # another source, a shape without counters, or another workload: no traffic figure
    assert bench.load_traffic("sparse_filter", "0" * 16, "rotation", shape) is None
    assert bench.load_traffic("sparse_filter", rec["kernel_source_digest"], "rotation", "3x3") is None
    assert bench.load_traffic("sparse_filter", rec["kernel_source_digest"], "small", shape) is None
