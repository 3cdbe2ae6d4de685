"""CPU checks of bench.py: the single-GPU contract of the command line and
the recorded solver traffic against the committed profile summary."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_solver_traffic_matches_committed_profile():
    # the bench's recorded solver bytes per step are the figure the committed
    # rocprofv3 summary derives from its FETCH_SIZE / WRITE_SIZE runs
    import os
    import re
    import bench
    text = open(os.path.join(bench.ROOT, "profiles", "slope_step_kernels.md")).read()
    m = re.search(r"\*\*([0-9.]+e\+[0-9]+) scaled HBM bytes\*\* per step for all `k_shape\*` launches", text)
    assert m, "profile summary lacks the per-step solver traffic line"
    assert float(m.group(1)) == bench.SHAPE_TRAFFIC["bytes_per_step"]
