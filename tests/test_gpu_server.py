"""Serving through the C ABI: continuous batching of kriging requests and
theta-evaluations on one device.

Each query's result must not depend on the requests it is batched with:
the server's answer for a request equals, bit for bit, pcv_predict of that
request alone (the same kernel computes each query in its own lane from the
same resident factors), and both equal the FP64 oracle within 1e-9.
Evaluations submitted to the server equal pcv_eval bit for bit.
"""
import sys
import threading

import numpy as np
import pytest

import oracle
from paper_1912_13132_amd import pcv
from paper_1912_13132_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def w_plain():
    return W.plain_fp64()


def _requests(w, k, seed, qmax=600):
    """k requests with log-uniform sizes 1..qmax over the domain (and a bit
    outside it, to exercise nearest-core routing)."""
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 700 + seed]))
    lo, hi = w.locs.min(0), w.locs.max(0)
    out = []
    for _ in range(k):
        nq = int(np.floor(10 ** r.uniform(0, np.log10(qmax))))
        out.append(r.uniform(lo - 0.02, hi + 0.02, (nq, 2)))
    return out


def _alone(P, reqs, obs):
    return [P.predict(q, want_var=True, obs_noise=o)[:2] for q, o in zip(reqs, obs)]


def test_predictions_same_alone_and_in_the_mix(w_plain):
    th = pcv.theta(0.1, 0.05, sigma2=1.3)
    reqs = _requests(w_plain, 24, 1)
    obs = [i % 3 == 0 for i in range(len(reqs))]
    wantv = [i % 4 != 1 for i in range(len(reqs))]
    say(f"[case] server mix: {len(reqs)} requests, sizes {[len(q) for q in reqs]}")
    with pcv.Problem.from_workload(w_plain, prec="mixed") as P:
        P.factor(th)
        alone = _alone(P, reqs, obs)
        loss_direct = P.eval(pcv.theta(0.08, 0.06))
        with pcv.Server(P, max_inflight=64) as srv:
            tk_eval = srv.submit_eval(pcv.theta(0.08, 0.06))
            results = [None] * len(reqs)

            def client(idx):
                tickets = [(i, srv.submit_predict(reqs[i], want_var=wantv[i], obs_noise=obs[i]))
                           for i in idx]
                for i, t in tickets:
                    results[i] = srv.wait(t)

            ths = [threading.Thread(target=client, args=(list(range(c, len(reqs), 4)),)) for c in range(4)]
            for t in ths:
                t.start()
            for t in ths:
                t.join()
            loss_srv = srv.wait(tk_eval)
            rep = srv.report()
    say(f"   batches {rep['n_batches']} mean queries/batch {rep['mean_batch_queries']:.1f} "
        f"p50 {rep['p50_s'] * 1e3:.2f} ms p99 {rep['p99_s'] * 1e3:.2f} ms")
    assert rep["n_predict"] == len(reqs) and rep["n_eval"] == 1
    assert rep["n_queries"] == sum(len(q) for q in reqs)
    assert 0 < rep["p50_s"] <= rep["p99_s"] <= rep["max_s"]
    assert loss_srv == loss_direct
    for i, ((m, v), (ma, va)) in enumerate(zip(results, alone)):
        np.testing.assert_array_equal(m, ma)
        if wantv[i]:
            np.testing.assert_array_equal(v, va)
        else:
            assert v is None
    # and the oracle agrees (routing included) on a few requests
    pt = w_plain.part
    for i in (0, 5, 11):
        q = reqs[i]
        own = oracle.route_queries(q, pt.core_rect)
        for s in np.unique(own):
            sel = own == s
            T = pt.train_idx[pt.train_ptr[s]:pt.train_ptr[s + 1]]
            mo, vo = oracle.predict(w_plain.locs[T], w_plain.y[T], q[sel], 0, 0.1, 0.05, sigma2=1.3,
                                    obs_noise=obs[i])
            np.testing.assert_allclose(results[i][0][sel], mo, rtol=1e-9, atol=1e-10)
            if wantv[i]:
                np.testing.assert_allclose(results[i][1][sel], vo, rtol=1e-9, atol=1e-10)


def test_requests_larger_than_a_batch_span_several(w_plain):
    """A budget of one or two kriging items per slot forces requests across
    many batches, and queries of different requests share batches."""
    th = pcv.theta(0.1, 0.05)
    reqs = _requests(w_plain, 6, 2, qmax=2000)
    say(f"[case] server small budget: sizes {[len(q) for q in reqs]}")
    with pcv.Problem.from_workload(w_plain, prec="fp64") as P:
        P.factor(th)
        alone = _alone(P, reqs, [False] * len(reqs))
        npad = int(np.ceil(np.diff(w_plain.part.train_ptr).max() / 64) * 64)
        per_slot = 2 * npad * pcv.KRIGE_Q * 8 + 64 * 40 * 4 + 4096
        with pcv.Server(P, mem_budget=3 * per_slot, max_inflight=8) as srv:
            tks = [srv.submit_predict(q) for q in reqs]
            res = [srv.wait(t) for t in tks]
            rep = srv.report()
    say(f"   item cap {rep['batch_item_cap']} batches {rep['n_batches']}")
    assert rep["batch_item_cap"] <= 3
    assert rep["n_batches"] > len(reqs)
    for (m, v), (ma, va) in zip(res, alone):
        np.testing.assert_array_equal(m, ma)
        np.testing.assert_array_equal(v, va)


def test_admission_waits_and_ticket_rules(w_plain):
    th = pcv.theta(0.1, 0.05)
    reqs = _requests(w_plain, 12, 3)
    say("[case] server admission / tickets")
    with pcv.Problem.from_workload(w_plain, prec="mixed") as P:
        with pcv.Server(P, max_inflight=2) as srv:
            # no factors yet
            with pytest.raises(pcv.PcvError) as e:
                srv.submit_predict(reqs[0])
            assert e.value.status == 5
        P.factor(th)
        alone = _alone(P, reqs, [False] * len(reqs))
        with pcv.Server(P, max_inflight=1) as srv:
            out = [None] * len(reqs)

            def client(c):
                for i in range(c, len(reqs), 3):
                    out[i] = srv.wait(srv.submit_predict(reqs[i]))

            ths = [threading.Thread(target=client, args=(c,)) for c in range(3)]
            for t in ths:
                t.start()
            for t in ths:
                t.join()
            rep = srv.report()
            t0 = srv.submit_predict(np.zeros((0, 2)))
            assert srv.wait(t0)[0].shape == (0,)
            with pytest.raises(pcv.PcvError) as e:
                srv.wait(t0)  # already collected
            assert e.value.status == 1
            with pytest.raises(pcv.PcvError) as e:
                srv.wait(12345)
            assert e.value.status == 1
        # the problem is usable again after the server is gone
        m, _, _ = P.predict(reqs[0])
    assert rep["admission_waits"] > 0
    for (mo, vo), (ma, va) in zip(out, alone):
        np.testing.assert_array_equal(mo, ma)
        np.testing.assert_array_equal(vo, va)
    np.testing.assert_array_equal(m, alone[0][0])


def test_evaluations_interleaved_with_kriging(w_plain):
    """Several optimisers' evaluations run beside kriging batches; every
    loss equals pcv_eval of the same theta."""
    g = W.theta_grid(w_plain.theta_true, 3)
    ths = [pcv.theta(*t) for t in g]
    reqs = _requests(w_plain, 16, 4)
    say("[case] server evals + kriging")
    with pcv.Problem.from_workload(w_plain, prec="mixed") as P:
        direct = [P.eval(t) for t in ths]
        P.factor(pcv.theta(0.1, 0.05))
        alone = _alone(P, reqs, [False] * len(reqs))
        with pcv.Server(P) as srv:
            te = [srv.submit_eval(t) for t in ths]
            tp = [srv.submit_predict(q) for q in reqs]
            losses = [srv.wait(t) for t in te]
            preds = [srv.wait(t) for t in tp]
            st = srv.stats()
    assert losses == direct
    for (m, v), (ma, va) in zip(preds, alone):
        np.testing.assert_array_equal(m, ma)
        np.testing.assert_array_equal(v, va)
    assert st["evals_per_s"] > 0 and st["qps"] > 0


def test_wait_timeout_reports_busy_and_keeps_the_ticket(w_plain):
    """pcv_server_wait with a timeout shorter than the request: PCV_ERR_BUSY,
    and the ticket stays valid; the result collected afterwards equals
    pcv_predict of the request alone."""
    th = pcv.theta(0.1, 0.05)
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 710]))
    q = r.uniform(0, 1, (100_000, 2))
    say("[case] server wait timeout -> BUSY")
    with pcv.Problem.from_workload(w_plain, prec="mixed") as P:
        P.factor(th)
        alone = P.predict(q)[:2]
        with pcv.Server(P) as srv:
            te = [srv.submit_eval(pcv.theta(0.1 * (1 + 0.1 * k), 0.05)) for k in range(3)]
            tk = srv.submit_predict(q)
            with pytest.raises(pcv.PcvError) as e:
                srv.wait(tk, timeout=1e-6)
            assert e.value.status == 6
            m, v = srv.wait(tk)
            for t in te:
                srv.wait(t)
    np.testing.assert_array_equal(m, alone[0])
    np.testing.assert_array_equal(v, alone[1])


def test_batching_window_with_evaluations(w_plain):
    """With a batching window and evaluations active, kriging batches wait
    for the window (fewer, larger batches); every result still equals
    pcv_predict alone bit for bit, and every loss equals pcv_eval.  A
    window outside [0, 10] s is rejected."""
    th = pcv.theta(0.1, 0.05)
    reqs = _requests(w_plain, 20, 9)
    ths = [pcv.theta(0.1 * (1 + 0.05 * k), 0.05) for k in range(4)]
    say("[case] server batching window 0.05 s with evaluations")
    with pcv.Problem.from_workload(w_plain, prec="mixed") as P:
        direct = [P.eval(t) for t in ths]
        P.factor(th)
        alone = _alone(P, reqs, [False] * len(reqs))
        with pytest.raises(pcv.PcvError) as e:
            pcv.Server(P, window=-1.0)
        assert e.value.status == 1
        with pcv.Server(P, window=0.05) as srv:
            te = [srv.submit_eval(t) for t in ths]
            tp = [srv.submit_predict(q) for q in reqs]
            preds = [srv.wait(t) for t in tp]
            losses = [srv.wait(t) for t in te]
            rep = srv.report()
    assert losses == direct
    for (m, v), (ma, va) in zip(preds, alone):
        np.testing.assert_array_equal(m, ma)
        np.testing.assert_array_equal(v, va)
    say(f"   batches {rep['n_batches']} for {len(reqs)} requests")


def test_server_budget_errors_leave_the_problem_usable(w_plain):
    """A workspace budget below one kriging item per slot is rejected
    (PCV_ERR_INVALID), one that no device holds fails with PCV_ERR_OOM; the
    problem serves normally afterwards, with the same bits as pcv_predict."""
    th = pcv.theta(0.1, 0.05)
    reqs = _requests(w_plain, 6, 13)
    say("[case] server budget errors")
    with pcv.Problem.from_workload(w_plain, prec="mixed") as P:
        P.factor(th)
        alone = _alone(P, reqs, [False] * len(reqs))
        with pytest.raises(pcv.PcvError) as e:
            pcv.Server(P, mem_budget=1024)
        assert e.value.status == 1
        with pytest.raises(pcv.PcvError) as e:
            pcv.Server(P, mem_budget=1 << 50)
        assert e.value.status == 2
        with pcv.Server(P) as srv:
            preds = [srv.wait(srv.submit_predict(q)) for q in reqs]
    for (m, v), (ma, va) in zip(preds, alone):
        np.testing.assert_array_equal(m, ma)
        np.testing.assert_array_equal(v, va)
