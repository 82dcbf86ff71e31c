"""Host-side behaviour of bench.py that needs no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_reported_only_for_matching_sources():
    assert bench.measured_traffic("fused_mixed:plain-262144x250x80", "0" * 16) is None
    assert bench.measured_traffic("no-such-kernel", bench.source_hash(bench.FUSED_SOURCES)) is None


def test_committed_traffic_entries_are_complete():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        d = json.load(f)
    for key in ("fused_mixed:plain-262144x250x80", "batch_kernel:batch-64grids"):
        e = d[key]
        assert e["bytes_per_launch"] == e["read_bytes"] + e["write_bytes"]
        assert len(e["source_hash"]) == 16 and e["kernel"]


def test_alu_peak_follows_from_unit_counts():
    # 256 CUs x 4 SIMDs x 64 lanes per 8 cycles at 2.4 GHz, two transcendentals per term
    assert abs(bench.TERM_PEAK_PER_S - 256 * 4 * 2.4e9 * 64 / 8 / 2) < 1e3


def test_host_rows_refuses_indices_outside_the_tensor():
    import numpy as np
    import pytest
    import torch
    t = torch.arange(12.0).reshape(4, 3)
    assert bench.host_rows(t, [0, 3]).tolist() == [[0.0, 1.0, 2.0], [9.0, 10.0, 11.0]]
    with pytest.raises(IndexError):
        bench.host_rows(t, np.array([1, 4]))
    with pytest.raises(IndexError):
        bench.host_rows(t, np.array([-1]))
