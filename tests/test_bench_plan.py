"""Host-side arithmetic of the benchmark's slice window (no GPU).

The benchmark stages every slice of the stream and times the last --steps
updates; the arguments the full test run passes (--steps 20 --warmup 5) and the
defaults must give ranges inside the staged slices.
"""

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("steps,warmup", [(20, 5), (190, 5), (1, 0), (375, 5), (380, 0)])
def test_window_inside_the_stream(steps, warmup):
    n_slices, n_init = 400, 20
    p = bench.plan_window(n_slices, n_init, steps, warmup)
    assert p["init"] == (0, n_init)
    t0, t1 = p["timed"]
    assert t1 == n_slices and t1 - t0 == steps
    w0, w1 = p["warmup"]
    assert w1 == t0 and w1 - w0 == warmup and w0 >= n_init
    u0, u1 = p["untimed"]
    assert u0 == n_init and u1 == t0
    # every slice index the run touches exists
    for a, b in p.values():
        assert 0 <= a <= b <= n_slices


@pytest.mark.parametrize("steps,warmup", [(0, 5), (20, -1), (380, 1), (400, 0)])
def test_window_rejects_impossible_arguments(steps, warmup):
    with pytest.raises(ValueError):
        bench.plan_window(400, 20, steps, warmup)


def test_workload_constants():
    w = bench.WORKLOAD
    assert w["n_slices"] - w["n_init"] == 380
    assert bench.PEAK_TFLOPS["fp32"] == 157.3 and bench.PEAK_HBM_GBS == 8000.0
