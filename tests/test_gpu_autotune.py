"""The autotuner (pcv_autotune): launch shapes and schedule picked by timing
pcv_eval, with a cache file of choices.

Three problems are tuned in one process (a tune, a reuse of the cache by an
identical problem, a new problem shape), in both precisions.  After tuning:
the loss matches the FP64 oracle within the path's tolerance (1e-6 mixed,
1e-10 FP64, every subset's SSPE too), pcv_eval_batch equals pcv_eval bit
for bit, a served evaluation equals pcv_eval bit for bit, and the cached
choice reproduces the tuned one.  The host side of the same cycle runs
under AddressSanitizer on the CPU (tests/test_host_harness.py)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1912_13132_amd import pcv
from parity_util import check_sspe

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-6}


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def _synthetic(seed, S=300):
    """S independent subsets: three large ones (shared in the first launch),
    a band around the 4-wave / 8-wave shape threshold, many small ones;
    more subsets than compute units, so two schedule groups apply."""
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 1400 + seed]))
    sizes_T = [3000, 2500, 2100] + list(r.integers(1200, 1700, size=40)) + list(r.integers(60, 400, size=S - 43))
    sizes_V = [60, 50, 40] + list(r.integers(5, 30, size=40)) + list(r.integers(1, 10, size=S - 43))
    locs, y, tl, vl = [], [], [], []
    off = 0
    for nt, nv in zip(sizes_T, sizes_V):
        spread = 3.0 * np.sqrt(nt / 2000.0)
        locs.append(r.uniform(0, spread, (nt + nv, 2)))
        y.append(r.standard_normal(nt + nv))
        tl.append(np.arange(off, off + nt))
        vl.append(np.arange(off + nt, off + nt + nv))
        off += nt + nv
    return (np.concatenate(locs), np.concatenate(y), np.r_[0, np.cumsum(sizes_T)],
            np.concatenate(tl).astype(np.int32), np.r_[0, np.cumsum(sizes_V)],
            np.concatenate(vl).astype(np.int32))


@pytest.fixture(scope="module")
def datas():
    return [_synthetic(1), _synthetic(2, S=290)]


@pytest.fixture(scope="module")
def refs(datas):
    return [oracle.cv_loss(*d, 0, 0.4, 0.1) for d in datas]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_tune_three_problems_cache_and_parity(datas, refs, prec, tmp_path):
    cache = str(tmp_path / "tune.txt")
    th = pcv.theta(0.4, 0.1)
    ths = [pcv.theta(0.4 * f, 0.1 * g) for f, g in ((1, 1), (0.8, 1.3), (1.2, 0.7))]
    chosen = []
    for k, (di, expect_cache) in enumerate(((0, 0), (0, 1), (1, 0))):
        say(f"[case] autotune prec={prec} problem {k} (data {di}), cache expected {expect_cache}")
        with pcv.Problem(*datas[di], prec=prec) as P:
            rep = P.autotune(th, cache=cache, reps=2)
            say(f"   {rep}")
            assert rep["from_cache"] == expect_cache
            assert rep["small_npad"] in (0, 1024, 1536, 2048, 3072, 4096)
            assert 1 <= rep["max_wg_per_subset"] <= 8 and rep["two_groups"] in (0, 1)
            if not expect_cache:
                assert rep["n_timed"] >= 2 and 0 < rep["best_s"] <= rep["default_s"]
            chosen.append((rep["small_npad"], rep["max_wg_per_subset"], rep["two_groups"]))
            loss, er = P.eval(th, report=True)
            ref = refs[di]
            assert abs(loss - ref["sspe"]) <= TOL[prec] * ref["sspe"]
            check_sspe(er["per_subset_sspe"], ref["per_subset_sspe"], prec, say)
            single = [P.eval(t) for t in ths]
            np.testing.assert_array_equal(P.eval_batch(ths), single)
            P.factor(th)
            with pcv.Server(P) as srv:
                served = [srv.wait(srv.submit_eval(t)) for t in ths]
            assert served == single
            assert P.eval(ths[1]) == single[1]
    assert chosen[1] == chosen[0]


def test_tune_refused_while_served(datas):
    th = pcv.theta(0.4, 0.1)
    with pcv.Problem(*datas[1], prec="mixed") as P:
        P.factor(th)
        with pcv.Server(P):
            with pytest.raises(pcv.PcvError) as e:
                P.autotune(th)
            assert e.value.status == 5
        assert P.autotune(th, reps=1)["from_cache"] == 0


def test_default_shapes_follow_schedule_groups(datas):
    """Without tuning: the first schedule group (256 largest subsets) takes
    8-wave work-groups, the remainder (all below the shape threshold) 4-wave
    ones.  The multi-theta launches and a served evaluation (launches of one
    work-group per compute unit) factor every subset with its group's shape,
    so all three agree bit for bit."""
    ths = [pcv.theta(0.4, 0.1), pcv.theta(0.3, 0.15)]
    say("[case] default shapes per schedule group: eval, eval_batch, served")
    with pcv.Problem(*datas[0], prec="mixed") as P:
        single = [P.eval(t) for t in ths]
        np.testing.assert_array_equal(P.eval_batch(ths), single)
        P.factor(ths[0])
        with pcv.Server(P) as srv:
            served = [srv.wait(srv.submit_eval(t)) for t in ths]
    assert served == single
