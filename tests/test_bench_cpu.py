"""Host-side logic of bench.py: the stored HBM traffic of the sweep is reported only for the kernel
source and the launch tiles it was measured with."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _recorded():
    kv = {}
    for line in open(bench.TRAFFIC_FILE):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    return kv


def test_traffic_needs_the_recorded_tiles_and_source(monkeypatch):
    kv = _recorded()
    tiles = [int(t) for t in kv["tiles"].split(",")]
    monkeypatch.setattr(bench, "kernel_hash", lambda: kv["kernel_source_sha256_16"])
    assert bench.read_traffic(tiles) == float(kv["hbm_bytes_per_launch"])
    other = list(tiles)
    other[1] = tiles[1] // 2  # another z chunk: the halo re-reads differ
    assert bench.read_traffic(other) is None
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    assert bench.read_traffic(tiles) is None


def test_recorded_traffic_is_near_the_algorithmic_bytes():
    kv = _recorded()
    ratio = float(kv["hbm_bytes_per_launch"]) / float(kv["algorithmic_bytes_per_launch"])
    assert 1.0 <= ratio < 1.2, ratio
    assert abs(ratio - float(kv["traffic_over_algorithmic"])) < 1e-3


def test_more_than_one_gpu_is_refused_with_a_message():
    """The build runs on one GPU: bench.py --gpus N with N > 1 exits with status 2 and says so,
    before it touches a device."""
    import subprocess

    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2, (res.returncode, res.stderr[-500:])
    assert "one GPU only" in res.stderr
    assert res.stdout.strip() == ""
