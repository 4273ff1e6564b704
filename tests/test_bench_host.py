"""Host-side checks of bench.py (no GPU): the one-GPU guard, and the sources list whose
hash gates the recorded HBM counters."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "exactly one GPU" in res.stderr
    assert res.stdout == ""


def test_traffic_sources_exist_and_hash_is_stable():
    sys.path.insert(0, ROOT)
    import bench
    for name in bench.TRAFFIC_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_2103_17081_amd", "csrc", name)), name
    assert bench.sources_sha256() == bench.sources_sha256()
    assert len(bench.sources_sha256()) == 64
