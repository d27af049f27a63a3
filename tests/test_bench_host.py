"""Host logic of bench.py: the one-GPU contract, the log-log interpolation
used for equal-error matching, and the per-kernel relative error."""
import math
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_log_interp_is_exact_on_a_power_law():
    # time = 3 * error^-2 is a straight line in log-log coordinates
    errs = [0.04, 0.02, 0.01, 0.005]
    times = [3.0 * e ** -2 for e in errs]
    for e in (0.03, 0.011, 0.0071):
        t = bench.log_interp(errs, times, e)
        assert math.isclose(t, 3.0 * e ** -2, rel_tol=1e-12)
    assert bench.log_interp(errs, times, 0.05) is None      # outside the sweep
    assert bench.log_interp(errs, times, 0.001) is None
    assert math.isclose(bench.log_interp(errs, times, 0.02), times[1], rel_tol=1e-12)


def test_relative_error_scales_per_kernel():
    ref = np.array([2.0, -0.5, 0.0, 4.0])
    v = np.array([2.2, -0.4, 0.3, np.nan])
    pot = bench.rel_errors(v, ref, 0)
    assert np.allclose(pot[:2], [0.1, 0.2]) and np.isinf(pot[2]) and np.isinf(pot[3])
    wind = bench.rel_errors(v, ref, 1)                        # |ref| floored at 1 (winding numbers)
    assert np.allclose(wind[:3], [0.1, 0.1, 0.3]) and np.isinf(wind[3])
    sd = bench.rel_errors(v, ref, 2, alpha=10.0)              # floored at 1 / alpha
    assert np.allclose(sd[:3], [0.1, 0.2, 3.0])
