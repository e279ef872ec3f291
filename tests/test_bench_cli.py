"""bench.py's command line on the host: more than one GPU is refused with a
message (the build runs on one GPU), and the helpers that shape the JSON
line behave."""
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
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_host_cores_respects_omp_num_threads(monkeypatch):
    n = len(os.sched_getaffinity(0))
    monkeypatch.setenv("OMP_NUM_THREADS", "1")
    assert bench.host_cores() == 1
    monkeypatch.setenv("OMP_NUM_THREADS", str(n + 5))
    assert bench.host_cores() == n
    monkeypatch.delenv("OMP_NUM_THREADS")
    assert bench.host_cores() == n


def test_traffic_record_is_tied_to_the_kernel_source():
    # the committed counter summary names the kernel source it was taken
    # with; it is used only while that source is unchanged
    v = bench.measured_traffic("lamina_2048", "f64", "k_stream_collide2")
    from paper_2006_13631_amd import profiling
    rec = json.load(open(os.path.join(ROOT, "profiles", "pmc_k_stream_collide2.lamina_2048.f64.json")))
    if rec["source_sha256"] == profiling.source_sha256():
        assert v == rec["bytes_per_launch"] and v > 0
    else:
        assert v is None
    assert bench.measured_traffic("lamina_2048", "f32", "k_stream_collide2") is None
