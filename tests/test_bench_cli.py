"""bench.py's command-line contract that needs no GPU (CPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    """bench.py measures one GPU: --gpus N > 1 exits with status 2 and says
    so, before touching a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_lookup_follows_the_kernel_sources():
    """Stored counter traffic is returned only for the hash of the device
    sources it was taken on; any other hash gives None."""
    sys.path.insert(0, ROOT)
    import bench
    import json
    with open(bench.TRAFFIC_FILE) as f:
        data = json.load(f)
    for key, ent in data.items():
        got = bench.measured_traffic(key)
        if ent["kernel_sha"] == bench.kernel_hash():
            assert got == ent["bytes_per_launch"]
        else:
            assert got is None
    assert bench.measured_traffic("no/such/key") is None
