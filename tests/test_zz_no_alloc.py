"""pcv_predict_noalloc (the prediction entry point that allocates no device
memory: its buffers live in the library's fixed per-device scratch array)
against pcv_predict, bit for bit, through the C ABI: two calls in a row, the
second smaller, so the second runs on what the first left in the array; a
request whose variance panels need several consecutive launches; and the
size limit."""
import sys

import numpy as np
import pytest

from paper_1912_13132_amd import pcv
from paper_1912_13132_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def _queries(w, n, seed):
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 1300 + seed]))
    lo, hi = w.locs.min(0), w.locs.max(0)
    return r.uniform(lo - 0.01, hi + 0.01, (n, 2))


def _same(a, b):
    for x, y in zip(a, b):
        if x is None:
            assert y is None
        else:
            np.testing.assert_array_equal(x, y)


def test_noalloc_matches_predict_twice_in_a_row():
    w = W.plain_fp64()
    th = pcv.theta(0.1, 0.05, sigma2=1.3)
    with pcv.Problem.from_workload(w, prec="mixed") as P:
        P.factor(th)
        for k, (nq, want_var, obs) in enumerate(((5000, True, False), (700, True, True), (300, False, False))):
            q = _queries(w, nq, k)
            say(f"[case] predict_noalloc call {k}: {nq} queries var={want_var} obs_noise={obs}")
            ref = P.predict(q, want_var=want_var, obs_noise=obs)
            got = P.predict(q, want_var=want_var, obs_noise=obs, noalloc=True)
            _same(got, ref)


def test_noalloc_several_launches_and_limits():
    """100,000 queries over 4 subsets of about 550 points: 6,250 items whose
    variance panels (about 70 KB each) exceed the scratch array together, so
    they run in consecutive launches reusing it."""
    w = W.plain_fp64()
    th = pcv.theta(0.1, 0.05)
    q = _queries(w, 100_000, 7)
    say("[case] predict_noalloc 100,000 queries (several launches)")
    with pcv.Problem.from_workload(w, prec="mixed") as P:
        with pytest.raises(pcv.PcvError) as e:
            P.predict(q[:10], noalloc=True)
        assert e.value.status == 5  # before pcv_factor
        P.factor(th)
        ref = P.predict(q)
        got = P.predict(q, noalloc=True)
        _same(got, ref)
        small = P.predict(q[:33], noalloc=True)
        _same(small, P.predict(q[:33]))
        big = np.zeros((262_145, 2)) + 0.5
        with pytest.raises(pcv.PcvError) as e:
            P.predict(big, noalloc=True)
        assert e.value.status == 1
        # the rejected call launched nothing: the next one is still right
        _same(P.predict(q[:50], noalloc=True), P.predict(q[:50]))
