"""Host logic of bench.py's measurement contract (no device work): the traffic figure is reported
only for the far-field kernel source and launch count the committed counters were taken with, the
algorithmic bytes of the symmetric product follow its block count, and a request for several GPUs
ends with a message."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_traffic_record_matches_the_current_far_kernel():
    # the committed profiles/traffic.json was taken with the far kernels as they stand
    v = bench.load_traffic("k_far_rect", "crossed192", 6)
    assert v is not None and v > 1e10


def test_traffic_is_null_for_another_launch_count_or_workload():
    assert bench.load_traffic("k_far_rect", "crossed192", 5) is None
    assert bench.load_traffic("k_far_rect", "crossed96", 1) is None
    assert bench.load_traffic("k_far", "crossed192", 6) is None


def test_traffic_is_null_once_the_far_kernel_source_changes(monkeypatch):
    monkeypatch.setattr(bench, "far_kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic("k_far_rect", "crossed192", 6) is None


@pytest.mark.parametrize("N,size,ks", [(64, 4, 8), (130, 8, 4), (1000, 4, 8)])
def test_symmetric_product_bytes(N, size, ks):
    # upper block triangle of 64 x 64 blocks, plus one 64 x 16 partial per block row and super-tile
    # (and one more), written and read back
    nb = -(-N // 64)
    nst = -(-nb // ks)
    upper = sum(nb - i for i in range(nb)) * 64 * 64 * size
    partials = 2 * nb * (nst + 1) * 64 * 16 * size
    assert bench.symv_bytes(N, size, ks) == upper + partials


def test_several_gpus_are_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_is_consistent():
    # bytes per launch = (scaled FETCH + scaled WRITE per step) / launches per step, and the summary
    # the record names is committed beside it
    import json
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for kernel, per in rec.items():
        for workload, e in per.items():
            total = e["fetch_bytes_per_step"] + e["write_bytes_per_step"]
            assert abs(e["bytes_per_launch"] * e["launches_per_step"] - total) <= 1e-9 * total
            assert e["write_bytes_per_step"] > 0 and e["fetch_scale"] > 0 and e["write_scale"] > 0
            assert os.path.isfile(os.path.join(ROOT, e["summary"]))
