"""Host-side contract of bench.py (no GPU): it refuses more than one GPU with a message, and
the measured pairwise traffic is looked up by a digest of the kernel sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_lookup_follows_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    digest = bench.kernel_source_digest()
    assert len(digest) == 64
    # a recorded measurement is returned only for the sources it was taken with
    saved = dict(bench.MEASURED_TRAFFIC)
    try:
        bench.MEASURED_TRAFFIC.clear()
        assert bench.measured_traffic() is None
        bench.MEASURED_TRAFFIC[digest] = 12345
        assert bench.measured_traffic() == 12345
    finally:
        bench.MEASURED_TRAFFIC.clear()
        bench.MEASURED_TRAFFIC.update(saved)
