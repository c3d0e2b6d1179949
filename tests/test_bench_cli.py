"""bench.py's command line without a GPU: more than one GPU is refused with a message before
any device is touched, and the conv layer 2 traffic figure is keyed to the profiled source."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_figure_matches_the_profiled_kernel():
    """The roofline's HBM traffic is reported only while conv layer 2's source is the one the
    byte counters were taken on; the committed source is that one."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.conv2_traffic() == bench.CONV2_TRAFFIC["bytes"]
