"""bench.py's command line on a machine without a GPU: a request for more than
one GPU stops with a message before anything is measured (there is no
multi-GPU path), and the profile lookup that feeds the roofline's traffic
figure works from the committed summaries."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_profile_lookup():
    import bench

    # the committed counter summary covers the headline workload's dominant kernel
    t = bench.profiled_traffic("varden2d_10m", "k_density")
    assert t is None or t > 0
    assert bench.profiled_traffic("no_such_workload", "k_density") is None
    assert bench.profiled_traffic("varden2d_10m", "no_such_kernel") is None
