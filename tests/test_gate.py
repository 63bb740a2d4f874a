"""The error gate's report (no GPU): hand-made cases whose counts are known."""
import numpy as np

from gate import TOL, errors, report


def test_report_counts_hand_made():
    ref = np.array([1.0, 1e-5, -0.5, 2e-4, 0.0])
    rel = np.array([1e-14, 5e-9, 0.0, 1e-11, 0.0])
    x = ref * (1 + rel)
    x[4] = 1e-20  # zero reference: strict error is huge, floored error tiny
    r = report(x, ref)
    # floor = 1e-3 * 1.0: components 1, 3 and 4 sit below it
    assert r["components"] == 5 and r["floored_components"] == 3
    # strict: component 1 (5e-9) and 4 (1e-20 / DBL_MIN) exceed 1e-10
    assert r["strict_over_tol"] == 2 and r["floored_over_tol"] == 0
    assert (r["strict"], r["floored"]) == errors(x, ref)
    assert r["floored"] <= TOL < r["strict"]


def test_report_flags_nonfinite_and_empty():
    r = report(np.array([np.nan, 1.0]), np.array([1.0, 1.0]))
    assert r["floored_over_tol"] == 1 and r["strict_over_tol"] == 1 and r["floored"] == float("inf")
    assert report(np.zeros(0), np.zeros(0))["components"] == 0
