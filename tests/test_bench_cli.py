"""The benchmark's command line on the host: it runs on exactly one GPU and
says so for any other count, before touching a device; its helper that
reads the committed HBM-traffic summary is gated on the kernel sources."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_traffic_summary_is_gated_on_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    for name in ("planet", "s2cloud", "era5"):
        path = bench.traffic_file(name)
        if not os.path.exists(path):
            assert bench._measured_traffic(name) is None
            continue
        with open(path) as f:
            t = json.load(f)
        assert set(t["sources_sha256"]) and t["per_launch_bytes"]
        got = bench._measured_traffic(name)
        # either the committed figures (sources unchanged) or None, never stale numbers
        if got is not None:
            assert set(got) >= {"encode_kernel", "decode_kernel", "me"}
            assert all(v > 0 for v in got.values())
