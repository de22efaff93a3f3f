"""Host-side checks of bench.py's reporting (no GPU): the one-GPU refusal,
the byte model behind the roofline, and that counter traffic is reported
only for the kernel sources it was taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_iteration_byte_model():
    """The method's words per node and iteration: the divergence step
    (adjoint averages and the residual) 13, five transform passes of 2 each
    (x, y forward, colour and time, y, x inverse), the update with the prox
    and the dual steps 21: 13 + 5 * 2 + 21 = 44 (176 bytes per node)."""
    w = bench.METHOD_WORDS
    passes = 2 * w["xform_x"] + 2 * w["xform_y"] + w["tc"]
    assert passes == 10
    assert w["div"] + passes + w["update"] == bench.METHOD_ITERATION_WORDS == 44
    assert bench.HBM_PEAK_GBS == 8000.0


def test_traffic_only_for_matching_sources():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        t = json.load(fh)
    name = next(iter(t["kernels"]))
    want = t["kernels"][name]["bytes_per_launch"]
    # the committed summary, read against the hash it records
    assert bench.measured_traffic(name, sources=t["sources"]) == pytest.approx(want)
    # any other source hash: no traffic
    assert bench.measured_traffic(name, sources="0" * 16) is None
    # no such kernel: no traffic
    assert bench.measured_traffic("k_no_such_kernel", sources=t["sources"]) is None
