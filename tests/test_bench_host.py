"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the bytes per
node behind the roofline, and the lookup of counter-measured traffic."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout


def test_values_per_node():
    # 9 + NG populations read and written per node and step
    assert bench.values_per_node("d2q5") == 28
    assert bench.values_per_node("d2q9t") == 36
    assert bench.values_per_node("isothermal") == 18
    assert bench.BYTES == {"f64": 8, "f32": 4, "f16": 2}


def _write(tmp_path, rec):
    d = tmp_path / "profiles"
    d.mkdir()
    (d / "sweep_traffic.json").write_text(json.dumps(rec))


def test_traffic_lookup_checks_sources_size_and_steps(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("f64", 100, 2) is None          # no file
    h = "0123456789abcdef"
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    ent = {"nodes": 100, "steps_per_launch": 2, "bytes_per_launch": 12345.0}
    _write(tmp_path, {"source_hash": h, "kernels": {"f64/2": ent}})
    assert bench.measured_traffic("f64", 100, 2) == 12345.0
    assert bench.measured_traffic("f64", 101, 2) is None          # other lattice
    assert bench.measured_traffic("f64", 100, 1) is None          # other kernel
    assert bench.measured_traffic("f32", 100, 2) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "fedcba9876543210")
    assert bench.measured_traffic("f64", 100, 2) is None          # counters taken on other sources


def test_source_hash_covers_the_library_sources():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert h == bench.kernel_source_hash()


def test_roofline_counts_the_state_once_per_launch():
    # a fused FP64 pair on 2048^2 in 172 us: the state (14 values read and
    # written per node) crosses HBM once per launch of two steps
    n = 2048 * 2048
    r = bench.roofline("f64", "d2q5", n, 2, 172e-6, 943e6)
    assert r["algorithmic_bytes_per_launch"] == 28 * 8 * n
    assert abs(r["achieved"] - 28 * 8 * n / 172e-6 / 1e9) < 0.1
    assert r["frac"] == round(r["achieved"] / 8000.0, 4) and r["frac"] < 1
    assert abs(r["effective_GBs"] - 2 * r["achieved"]) < 0.2 and r["effective_frac"] > 1
    assert abs(r["traffic_GBs"] - 943e6 / 172e-6 / 1e9) < 0.1
    assert r["state_in_last_level_cache"] is False
    # four steps per launch: the state still crosses HBM once
    r4 = bench.roofline("f64", "d2q5", n, 4, 223e-6, None)
    assert r4["algorithmic_bytes_per_launch"] == 28 * 8 * n
    assert abs(r4["effective_GBs"] - 4 * r4["achieved"]) < 0.2 and r4["frac"] < 1
    # one step per launch: effective equals achieved
    r1 = bench.roofline("f64", "d2q5", n, 1, 160e-6, None)
    assert r1["effective_GBs"] == r1["achieved"] and r1["traffic_GBs"] is None
    # the FP16 2048^2 state (235 MB for both buffers) fits the 256 MB last-level cache
    assert bench.roofline("f16", "d2q5", n, 1, 40e-6, None)["state_in_last_level_cache"] is True
    assert bench.roofline("f32", "d2q5", n, 2, 96e-6, None)["state_in_last_level_cache"] is False


def test_cpu_model_string():
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()
