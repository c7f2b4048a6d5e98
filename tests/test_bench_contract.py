"""bench.py contract checks that need no GPU: the one-GPU build refuses
--gpus N > 1 before touching a device, and the committed HBM-counter summary
is found (or reported stale) by the source-hash guard."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line for an unsupported configuration


def test_traffic_guard_reads_the_committed_summary():
    sys.path.insert(0, ROOT)
    import bench

    v = bench.measured_traffic("composite_bwd")
    # either the counters match the current kernel source (a byte count) or they are stale (None)
    assert v is None or (isinstance(v, int) and v > 0)
    assert bench.measured_traffic("no_such_kernel") is None
