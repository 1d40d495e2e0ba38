"""Host logic of bench.py: the measured-traffic lookup and the one-GPU guard."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_summary_was_taken_on_the_committed_kernels():
    # The counter summary is only used while the kernel sources hash to the
    # value recorded in it; a stale summary would silently null `traffic`.
    with open(bench.TRAFFIC_FILE) as f:
        recorded = [line.split(":", 1)[1].strip() for line in f if line.startswith("kernel_source_sha256:")]
    assert recorded == [bench.kernel_digest()]


def _summary():
    with open(bench.TRAFFIC_FILE) as f:
        kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(("#", " ")))
    return {k.strip(): v.strip() for k, v in kv.items()}


def test_measured_traffic_bytes_scales_the_counters(monkeypatch):
    kv = _summary()
    monkeypatch.setattr(bench, "kernel_digest", lambda: kv["kernel_source_sha256"])
    ff, wf = float(kv["fetch_factor"]), float(kv["write_factor"])
    for kernel in ("pixel_walk_kernel<1>", "pixel_walk_kernel<2>"):
        want = (float(kv[kernel + ".fetch_kib"]) * ff + float(kv[kernel + ".write_kib"]) * wf) * 1024.0
        assert bench.measured_traffic_bytes(kernel) == pytest.approx(want)
        assert want > 1e10  # tens of GB per launch of the benchmark walk
    assert bench.measured_traffic_bytes("no_such_kernel") is None


def test_measured_traffic_is_none_for_other_kernel_sources(monkeypatch):
    monkeypatch.setattr(bench, "kernel_digest", lambda: "0" * 64)
    assert bench.measured_traffic_bytes("pixel_walk_kernel<1>") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
