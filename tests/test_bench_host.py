"""Host logic of the benchmark script, on the CPU: it measures one GPU and
refuses anything else before touching a device, and it reports the counter
traffic only for the sweep sources the counters were taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, env=e,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2 and r.stdout == ""
    assert "one GPU" in r.stderr


def test_a_multi_rank_launch_is_refused():
    r = _run([], env={"WORLD_SIZE": "2"})
    assert r.returncode == 2 and "--gpus 1" in r.stderr


def test_counter_traffic_is_reported_only_for_the_measured_sources(monkeypatch):
    sha = bench.sweep_sources_sha1()
    assert len(sha) == 40
    monkeypatch.setattr(bench, "SWEEP_TRAFFIC", {"sweep_sha1": sha, "bytes_per_launch": 1.5e9})
    assert bench.sweep_traffic() == 1.5e9
    monkeypatch.setattr(bench, "SWEEP_TRAFFIC", {"sweep_sha1": "0" * 40, "bytes_per_launch": 1.5e9})
    assert bench.sweep_traffic() is None


def test_algorithmic_bytes_per_update():
    """19 population loads and 19 stores of the storage type plus the cell
    flag; for the 256^3 workload's 16,676,197 bulk cells one FP32 sweep is
    2,551,559,160 bytes."""
    assert bench.BYTES_PER_LUP == {"f32": 153, "f16": 77, "bf16": 77, "f64": 305}
    assert 16676197 * (bench.BYTES_PER_LUP["f32"] - 1) + 256 ** 3 == 2551559160
