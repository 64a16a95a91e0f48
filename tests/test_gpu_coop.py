"""Large subsets factored by several work-groups together (the
max_wg_per_subset option): the cooperative launch must give the same bits
as one work-group per subset, in every replay, for both precisions, and
match the FP64 oracle.

Each shared subset's row chunks are dealt out over its work-groups, panel by
panel; the chunk arithmetic is unchanged, so the comparison is exact."""
import sys

import numpy as np
import pytest

import oracle
from paper_1912_13132_amd import pcv
from parity_util import check_logdet, check_sspe

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-6}


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def _synthetic(sizes_T, sizes_V, seed, spread=3.0):
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 900 + seed]))
    locs, y, tl, vl = [], [], [], []
    off = 0
    for nt, nv in zip(sizes_T, sizes_V):
        locs.append(r.uniform(0, spread, (nt + nv, 2)))
        y.append(r.standard_normal(nt + nv))
        tl.append(np.arange(off, off + nt))
        vl.append(np.arange(off + nt, off + nt + nv))
        off += nt + nv
    return (np.concatenate(locs), np.concatenate(y), np.r_[0, np.cumsum(sizes_T)],
            np.concatenate(tl).astype(np.int32), np.r_[0, np.cumsum(sizes_V)],
            np.concatenate(vl).astype(np.int32))


def _run(data, prec, max_wg, graph=True, reps=2, cov=0):
    th = pcv.theta(0.4, 0.1, cov=cov)
    with pcv.Problem(*data, prec=prec, max_wg_per_subset=max_wg, graph=graph) as P:
        out = [P.eval(th, report=True) for _ in range(reps)]
    for loss, rep in out[1:]:  # the counters are cleared before every launch
        assert loss == out[0][0]
        np.testing.assert_array_equal(rep["per_subset_logdet"], out[0][1]["per_subset_logdet"])
    return out[0]


# sizes: padded 3,008 / 2,560 / 2,112 (shared), 960 and 320 (alone), a
# ragged 1-point subset and one without validation points
SIZES_T = [3000, 2500, 2100, 900, 300, 1, 2200]
SIZES_V = [60, 50, 40, 30, 20, 3, 0]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_shared_factorisation_same_bits(prec):
    data = _synthetic(SIZES_T, SIZES_V, 1)
    say(f"[case] shared factorisation prec={prec} sizes={SIZES_T} max_wg=1")
    loss1, rep1 = _run(data, prec, 1)
    assert rep1["n_coop_subsets"] == 0
    for max_wg, graph in ((2, True), (3, False), (8, True), (0, True)):
        say(f"[case] shared factorisation prec={prec} max_wg={max_wg} graph={graph}")
        loss, rep = _run(data, prec, max_wg, graph=graph)
        # the three active subsets of at least 2,048 padded rows are shared
        assert rep["n_coop_subsets"] == 3, rep["n_coop_subsets"]
        assert loss == loss1
        for k in ("per_subset_sspe", "per_subset_logdet", "per_subset_neg2loglik"):
            np.testing.assert_array_equal(rep[k], rep1[k], err_msg=k)
        assert rep["n_fallback_fp64"] == rep1["n_fallback_fp64"] == 0


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("cov", [pcv.COV_EXP, pcv.COV_MATERN32])
def test_shared_factorisation_matches_oracle(prec, cov):
    data = _synthetic(SIZES_T, SIZES_V, 2)
    say(f"[case] shared factorisation vs oracle prec={prec} cov={cov}")
    ref = oracle.cv_loss(*data, cov, 0.4, 0.1)
    loss, rep = _run(data, prec, 8, reps=1, cov=cov)
    assert rep["n_coop_subsets"] == 3
    assert abs(loss - ref["sspe"]) <= TOL[prec] * abs(ref["sspe"])
    check_sspe(rep["per_subset_sspe"], ref["per_subset_sspe"], prec, say)
    act = ref["per_subset_nval"] > 0
    check_logdet(rep["per_subset_logdet"][act], ref["per_subset_logdet"][act], np.array(SIZES_T)[act], 0.1,
                 prec, say)


def test_only_the_largest_are_shared():
    """Many small subsets and two large ones: only the two are shared (the
    small ones are below the size floor and the average load)."""
    sizes_T = [2600, 2300] + [150] * 300
    sizes_V = [40, 40] + [5] * 300
    data = _synthetic(sizes_T, sizes_V, 3, spread=1.0)
    say("[case] shared factorisation: 2 large + 300 small")
    loss1, rep1 = _run(data, "mixed", 1, reps=1)
    loss, rep = _run(data, "mixed", 0)
    assert rep["n_coop_subsets"] == 2
    assert loss == loss1
    np.testing.assert_array_equal(rep["per_subset_sspe"], rep1["per_subset_sspe"])


def test_served_evaluation_same_bits_as_shared_launch():
    """A problem held by a server evaluates launch by launch with one
    work-group per subset (no shared launch); its losses carry the same bits
    as pcv_eval with the largest subsets shared."""
    data = _synthetic(SIZES_T, SIZES_V, 4)
    th = [pcv.theta(0.4, 0.1), pcv.theta(0.3, 0.2)]
    say("[case] served evaluation vs shared launch")
    with pcv.Problem(*data, prec="mixed") as P:
        direct = []
        for t in th:
            loss, rep = P.eval(t, report=True)
            assert rep["n_coop_subsets"] == 3
            direct.append(loss)
        P.factor(th[0])
        with pcv.Server(P) as srv:
            losses = [srv.wait(srv.submit_eval(t)) for t in th]
        # after the server: the shared launch again, same bits
        after = P.eval(th[0], report=True)
    assert losses == direct
    assert after[0] == direct[0] and after[1]["n_coop_subsets"] == 3


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_shared_launch_busy_device_falls_back_to_one_workgroup(prec):
    """An evaluation that finds another shared launch in flight on its device
    (forced by debug bit 1) factors with one work-group per subset: the same
    bits, n_coop_subsets = 0, in graph replays and eager launches; the next
    evaluation without the flag shares again."""
    data = _synthetic(SIZES_T, SIZES_V, 5)
    th = pcv.theta(0.4, 0.1)
    say(f"[case] shared launch with the device flag taken prec={prec}")
    loss1, rep1 = _run(data, prec, 1)
    for graph in (True, False):
        with pcv.Problem(*data, prec=prec, debug_flags=2, graph=graph) as P:
            out = [P.eval(th, report=True) for _ in range(2)]
        for loss, rep in out:
            assert rep["n_coop_subsets"] == 0
            assert loss == loss1
            np.testing.assert_array_equal(rep["per_subset_logdet"], rep1["per_subset_logdet"])
    loss8, rep8 = _run(data, prec, 8)
    assert rep8["n_coop_subsets"] == 3 and loss8 == loss1


def test_concurrent_evaluations_from_two_threads():
    """Two problems with shared launches evaluated at the same time from two
    threads on their own streams: every result equals the one-work-group
    factorisation bit for bit, and the shared launches never overlap (each
    evaluation either shares or, while the other holds the device, does
    not)."""
    import threading
    datas = [_synthetic(SIZES_T, SIZES_V, 6 + k) for k in range(2)]
    th = pcv.theta(0.4, 0.1)
    say("[case] two threads, two problems with shared launches")
    ref = [_run(d, "mixed", 1, reps=1)[0] for d in datas]
    probs = [pcv.Problem(*d, prec="mixed") for d in datas]
    out = [[], []]
    errs = []

    def worker(k):
        try:
            for _ in range(6):
                out[k].append(probs[k].eval(th, report=True))
        except Exception as e:  # pragma: no cover - reported below
            errs.append(e)

    ts = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    for P in probs:
        P.close()
    assert not errs, errs
    for k in range(2):
        for loss, rep in out[k]:
            assert loss == ref[k]
            assert rep["n_coop_subsets"] in (0, 3)
            assert rep["n_fallback_fp64"] == 0
    say(f"   shared launches: {[sum(r['n_coop_subsets'] > 0 for _, r in o) for o in out]} of 6 each")
