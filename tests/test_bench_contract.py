"""The benchmark's command-line contract that holds without a GPU: it
measures one GPU only and refuses a larger count before touching a device."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""        # no JSON line for a refused run


def test_committed_traffic_record_is_for_the_committed_tracking_kernel():
    # The bench line's roofline.traffic comes from the rocprofv3 record under
    # profiles/, keyed by a hash of the tracking kernel's sources: it must be
    # the record of this kernel (else the bench reports null), and of the
    # right size: about the state a launch reads (76 B per particle: six
    # coordinates, three spin components, the status) and writes back (68 B:
    # Pt does not change), and within what spilled registers could add.
    sys.path.insert(0, ROOT)
    import bench
    traffic = bench.recorded_traffic(1 << 20, 100)
    assert traffic is not None
    algorithmic = (76 + 68) * (1 << 20)
    assert 0.99 * algorithmic < traffic < 2.5 * algorithmic
