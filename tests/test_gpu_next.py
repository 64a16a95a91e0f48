"""GPU checks of the per-subset likelihood, the local-theta grid evaluation
and the local-theta factorisation against the FP64 oracle.

Tolerances: -2 log-likelihood per subset (eq. (2)) within the log det bound
of tests/parity_util.py plus the loss tolerance (1e-10 FP64, 1e-6 mixed)
relative to |-2 l_i| for the quadratic term; local losses per subset and
theta within the loss tolerance.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1912_13132_amd import pcv
from paper_1912_13132_amd import workloads as W
from parity_util import TOL_SSPE, check_sspe, logdet_bound

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def w_small():
    return W.scaled("batched", 0.05)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_composite_likelihood_per_subset(w_small, prec):
    pt = w_small.part
    th = pcv.theta(0.05, 0.1, sigma2=0.7)
    say(f"[case] likelihood prec={prec}")
    with pcv.Problem.from_workload(w_small, prec=prec) as P:
        _, rep = P.eval(th, report=True)
    got = rep["per_subset_neg2loglik"]
    ref = np.zeros(pt.n_subsets)
    for i in range(pt.n_subsets):
        if pt.val_ptr[i + 1] == pt.val_ptr[i]:
            continue
        T = pt.train_idx[pt.train_ptr[i]:pt.train_ptr[i + 1]]
        ref[i] = oracle.neg2_loglik_subset(w_small.locs[T], w_small.y[T], 0, 0.05, 0.1, 0.7)
    n = np.diff(pt.train_ptr)
    act = np.diff(pt.val_ptr) > 0
    bound = logdet_bound(prec, n, 0.1) + TOL_SSPE[prec] * np.abs(ref)
    ratio = np.abs(got - ref)[act] / bound[act]
    say(f"   max |diff| {np.abs(got - ref).max():.2e}, max diff / bound {ratio.max():.3f}")
    assert ratio.max() <= 1.0
    assert np.all(got[~act] == 0.0)
    assert abs(rep["neg2loglik"] - ref.sum()) <= bound[act].sum()


def test_local_best_theta_over_a_grid(w_small):
    pt = w_small.part
    g = W.theta_grid(w_small.theta_true, 3)
    ths = [pcv.theta(*t) for t in g]
    say("[case] local best theta over a 3x3 grid")
    with pcv.Problem.from_workload(w_small, prec="mixed") as P:
        losses, z, best = P.eval_grid(ths)
    zr = np.array([oracle.cv_loss(w_small.locs, w_small.y, pt.train_ptr, pt.train_idx, pt.val_ptr,
                                  pt.val_idx, 0, r_, l_)["per_subset_sspe"] for r_, l_ in g])
    for k in range(len(g)):
        check_sspe(z[k], zr[k], "mixed", say, what=f"local SSPE at theta {k}")
    act = np.diff(pt.val_ptr) > 0
    assert np.all(best[~act] == -1)
    for i in np.nonzero(act)[0]:
        order = np.argsort(zr[:, i], kind="stable")
        k0, k1 = order[0], order[1]
        # where the two best differ by more than the tolerance the argmin is unique
        if zr[k1, i] - zr[k0, i] > 2e-6 * zr[k0, i]:
            assert best[i] == k0
        else:
            assert best[i] in (k0, k1)
    np.testing.assert_allclose(losses, zr.sum(axis=1), rtol=1e-6)


def test_local_theta_factorisation_predicts_with_each_subsets_theta(w_small):
    pt = w_small.part
    S = pt.n_subsets
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 800]))
    loc_th = [(0.05 * 2 ** r.uniform(-1, 1), 0.1 * 2 ** r.uniform(-1, 1)) for _ in range(S)]
    ths = [pcv.theta(a, b, sigma2=1.2) for a, b in loc_th]
    lo, hi = w_small.locs.min(0), w_small.locs.max(0)
    q = r.uniform(lo, hi, (400, 2))
    say("[case] local theta factorisation")
    with pcv.Problem.from_workload(w_small, prec="mixed") as P:
        P.factor_local(ths)
        mean, var, owner = P.predict(q)
        # the same theta everywhere gives exactly pcv_factor's predictions
        P.factor_local([pcv.theta(0.05, 0.1, sigma2=1.2)] * S)
        m1, v1, _ = P.predict(q)
        P.factor(pcv.theta(0.05, 0.1, sigma2=1.2))
        m2, v2, _ = P.predict(q)
    np.testing.assert_array_equal(m1, m2)
    np.testing.assert_array_equal(v1, v2)
    for s in np.unique(owner):
        sel = owner == s
        T = pt.train_idx[pt.train_ptr[s]:pt.train_ptr[s + 1]]
        mo, vo = oracle.predict(w_small.locs[T], w_small.y[T], q[sel], 0, loc_th[s][0], loc_th[s][1],
                                sigma2=1.2)
        np.testing.assert_allclose(mean[sel], mo, rtol=1e-9, atol=1e-10)
        np.testing.assert_allclose(var[sel], vo, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("local", [False, True])
def test_gls_coefficients_per_subset(w_small, local):
    """eq. (8) per subset with an intercept, the coordinates and their
    product as covariates, through the resident factors (global or local
    theta), against the oracle."""
    pt = w_small.part
    S = pt.n_subsets
    X = np.c_[np.ones(len(w_small.y)), w_small.locs, w_small.locs[:, 0] * w_small.locs[:, 1]]
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 801]))
    loc_th = [(0.05 * 2 ** r.uniform(-1, 1), 0.1 * 2 ** r.uniform(-1, 1)) for _ in range(S)]
    say(f"[case] GLS local={local}")
    with pcv.Problem.from_workload(w_small, prec="mixed") as P:
        if local:
            P.factor_local([pcv.theta(a, b) for a, b in loc_th])
        else:
            P.factor(pcv.theta(0.05, 0.1))
        beta, st = P.gls(X)
    for i in range(S):
        T = pt.train_idx[pt.train_ptr[i]:pt.train_ptr[i + 1]]
        th, lam = loc_th[i] if local else (0.05, 0.1)
        ref = oracle.gls_beta_subset(w_small.locs[T], w_small.y[T], X[T], 0, th, lam)
        assert st[i] == 0
        np.testing.assert_allclose(beta[i], ref, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_grid_batched_equals_single_evaluations(w_small, prec):
    """pcv_eval_grid runs the multi-theta launches: its losses and local
    losses equal one pcv_eval per theta bit for bit (70 values: a group of
    64 theta slots and a remainder of 6)."""
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 802]))
    ths = [pcv.theta(0.05 * 2 ** r.uniform(-1, 1), 0.1 * 2 ** r.uniform(-1, 1)) for _ in range(70)]
    say(f"[case] eval_grid batched vs single prec={prec}")
    with pcv.Problem.from_workload(w_small, prec=prec) as P:
        losses, z, best = P.eval_grid(ths)
        for k in (0, 37, 63, 64, 69):
            loss, rep = P.eval(ths[k], report=True)
            assert losses[k] == loss
            np.testing.assert_array_equal(z[k], rep["per_subset_sspe"])
