"""Host logic of the benchmark: byte accounting, the one-GPU guard, and the
source-hash gate on counter-derived traffic."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_collision_bytes_per_particle():
    # FP64: 64-byte record read + x, v written (48) + id, state, flag (6);
    # FP32: 32-byte record + 24 + 6; plus 8 bytes per cell
    assert bench.algorithmic_bytes("collide", 1000, 100, 8, 0) == 1000 * 118 + 800
    assert bench.algorithmic_bytes("collide", 1000, 100, 4, 0) == 1000 * 62 + 800


def test_streaming_bytes_skip_list_particles():
    # free particles only: read x, v + flag, write x + key/rank
    assert bench.algorithmic_bytes("stream_bin", 1000, 10, 8, 100) == 900 * (9 * 8 + 9) + 80
    # a flow also writes v
    assert bench.algorithmic_bytes("stream_bin", 1000, 10, 4, 0, flow=True) == 1000 * (12 * 4 + 9) + 80


def test_method_floor_per_particle():
    # rho 10: 0.1 cells per particle
    assert bench.method_bytes_per_particle(8, 0.1) == pytest.approx(212.2)
    assert bench.method_bytes_per_particle(4, 0.1) == pytest.approx(128.2)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_is_dropped_when_kernels_changed(tmp_path, monkeypatch):
    from paper_1608_04904_amd.profiling import kernel_source_hash
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    entry = dict(kernels=dict(collide=dict(fetch_MB=2.0, write_MB=1.0)))
    (prof / "w_fp64_traffic.json").write_text(json.dumps(dict(entry, source_hash="0" * 16)))
    assert bench.traffic_table("w", 64) is None
    (prof / "w_fp64_traffic.json").write_text(json.dumps(dict(entry, source_hash=kernel_source_hash())))
    assert bench.traffic_table("w", 64) == {"collide": 3.0 * 1048576}
    assert bench.traffic_table("missing", 64) is None
