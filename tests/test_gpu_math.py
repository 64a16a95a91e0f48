"""The FP64 device arithmetic of the refinement residual and of the kriging
of validation points (e^{-t} and sqrt(x), written with a Taylor polynomial
and the hardware reciprocal square root) against numpy's exp and sqrt, in
units in the last place, over the argument ranges the covariance uses."""
import sys

import numpy as np
import pytest

from paper_1912_13132_amd import pcv

pytestmark = pytest.mark.gpu


def _ulps(a, b):
    return np.abs(a - b) / np.spacing(np.abs(b))


def test_exp_neg_and_sqrt_within_ulps():
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 800]))
    k = 150000
    t = np.concatenate([[0.0, 5e-324, 1e-300, 1e-17, 0.5 * np.log(2.0), np.log(2.0), 1.0, 700.0, 708.0],
                        r.uniform(0.0, 1.0, k), r.uniform(0.0, 50.0, k), r.uniform(0.0, 708.0, k),
                        np.exp(r.uniform(-40.0, 0.0, k)),
                        # near the argument-reduction boundaries (k ln 2 / 2)
                        (np.arange(1, k + 1) % 1000 + 0.5) * np.log(2.0) * (1 + r.uniform(-1e-12, 1e-12, k))])
    x = np.concatenate([[1e-300, 1e-200, 1e-20, 1.0, 2.0, 3.0, 4.0, 1e100, 1e300],
                        r.uniform(0.0, 1.0, k), r.uniform(0.0, 1e4, k), np.exp(r.uniform(-690.0, 690.0, k)),
                        r.uniform(0.0, 1e-10, k), np.arange(1, k + 1, dtype=np.float64) ** 2])
    assert t.shape == x.shape
    print(f"[case] exp_neg / sqrt_pos on {t.size} values", file=sys.stderr, flush=True)
    e, s = pcv.selftest_math(t, x)
    ue = _ulps(e, np.exp(-t))
    us = _ulps(s, np.sqrt(x))
    print(f"   exp max {ue.max():.2f} ulp mean {ue.mean():.3f}; sqrt max {us.max():.2f} ulp",
          file=sys.stderr, flush=True)
    assert ue.max() <= 2.0
    assert us.max() <= 1.0


def test_exp_neg_tail_and_zero_distance():
    """Arguments beyond 708 give denormal or clamped results within 1e-320
    absolutely; sqrt(0) is 1e-150, where e^{-d/theta} is exactly 1."""
    t = np.array([708.5, 720.0, 739.0, 740.0, 745.0, 800.0, 1e6])
    x = np.zeros_like(t)
    e, s = pcv.selftest_math(t, x)
    assert np.all(np.abs(e - np.exp(-t)) <= 1e-320)
    assert np.all(s == 1e-150)
    e1, _ = pcv.selftest_math(s * 1e-3, x)
    assert np.all(e1 == 1.0)
