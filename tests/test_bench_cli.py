"""Host-side behaviour of bench.py that needs no GPU: the one-GPU guard and the
counter summary lookup."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_values_follow_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    vals = bench.counter_values(1000000)
    # either a measurement of exactly these sources, or nothing (never a stale number)
    if vals:
        text = open(bench.COUNTER_SUMMARY).read()
        assert bench.kernel_source_hash() in text
        assert vals["hbm_bytes_per_launch"] > 0 and vals["hw_fp64_flops_per_launch"] > 0
    assert bench.counter_values(12345) == {}
