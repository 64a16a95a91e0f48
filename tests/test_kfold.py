"""Parallel k-fold CV (the remark closing Sec. 2.2): k rounds of the hold-out
division of Sec. 2.3, round j holding out the points of fold j; the loss
sums the rounds.

Pins of the oracle's k-fold construction:
  * leave-one-out (one core, k = N, one point per fold) against the closed
    form of the leave-one-out residual, y_i - yhat_i = [K^-1 y]_i / [K^-1]_ii
    with K = Sigma + lambda I (the cross-covariances carry no nugget);
  * all-covering shells with several cores equal one core with the same
    folds (every round trains each subset on all points outside the fold);
  * every point is validated in exactly one round, and no round trains on
    its own fold.
The package's host k-fold partition is checked against the oracle, and its
fold draw for balance.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import division as D
from paper_1912_13132_amd import partition as part


def _rng(k):
    return np.random.default_rng(np.random.SeedSequence([1912, 13132, 1300 + k]))


def _cov(P, kind, theta):
    d = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
    t = d / theta
    return np.exp(-t) if kind == oracle.COV_EXP else (1.0 + t) * np.exp(-t)


@pytest.mark.parametrize("kind,theta,lam", [(oracle.COV_EXP, 0.3, 0.1), (oracle.COV_MATERN32, 0.2, 0.05),
                                            (oracle.COV_EXP, 0.5, 1e-3)])
def test_leave_one_out_closed_form(kind, theta, lam):
    r = _rng(1)
    N = 40
    P = r.uniform(0.0, 1.0, (N, 2))
    y = r.standard_normal(N)
    R = np.array([[0.0, 0.0, 1.0, 1.0]])
    labels = r.permutation(N)
    tp, ti, vp, vi = D.kfold_subsets(P, R, 0.0, labels, N)
    got = oracle.cv_loss(P, y, tp, ti, vp, vi, kind, theta, lam)["sspe"]
    K = _cov(P, kind, theta) + lam * np.eye(N)
    Ki = sla.inv(K)
    e = (Ki @ y) / np.diag(Ki)
    want = float(np.sum(e * e))
    assert abs(got - want) <= 1e-10 * want, (got, want)


@pytest.mark.parametrize("k", [2, 3, 5])
def test_all_covering_shells_equal_one_core(k):
    r = _rng(2)
    N = 300
    P = r.uniform(0.0, 1.0, (N, 2))
    y = r.standard_normal(N)
    R = part.grid_cores((0.0, 0.0, 1.0, 1.0), 3, 2)
    labels = r.integers(0, k, N)
    tp, ti, vp, vi = D.kfold_subsets(P, R, 2.0, labels, k)
    many = oracle.cv_loss(P, y, tp, ti, vp, vi, oracle.COV_EXP, 0.2, 0.1)
    one = D.kfold_subsets(P, np.array([[0.0, 0.0, 1.0, 1.0]]), 0.0, labels, k)
    ref = oracle.cv_loss(P, y, *one, oracle.COV_EXP, 0.2, 0.1)
    assert abs(many["sspe"] - ref["sspe"]) <= 1e-10 * ref["sspe"]
    assert many["n_val"] == ref["n_val"] == N


def test_each_point_validated_once_and_no_round_trains_on_its_fold():
    r = _rng(3)
    N, k = 500, 4
    P = r.uniform(0.0, 1.0, (N, 2))
    R = part.grid_cores((0.0, 0.0, 1.0, 1.0), 2, 3)
    S = R.shape[0]
    labels = r.integers(0, k, N)
    tp, ti, vp, vi = D.kfold_subsets(P, R, 0.08, labels, k)
    assert tp.shape[0] == vp.shape[0] == k * S + 1
    assert np.array_equal(np.sort(vi), np.arange(N))
    for j in range(k):
        for i in range(S):
            s = j * S + i
            T = ti[tp[s]:tp[s + 1]]
            V = vi[vp[s]:vp[s + 1]]
            assert np.all(labels[T] != j) and np.all(labels[V] == j)


@pytest.mark.parametrize("k,delta", [(2, 0.0), (5, 0.05), (10, 0.1)])
def test_host_kfold_partition_matches_oracle(k, delta):
    r = _rng(4)
    P = r.uniform(0.0, 1.0, (2000, 2))
    R = part.grid_cores((0.0, 0.0, 1.0, 1.0), 3, 3)
    pt = part.build_partition_kfold(P, R, delta, k, _rng(40 + k))
    labels = pt.info["labels"]
    want = D.kfold_subsets(P, R, delta, labels, k)
    for a, b in zip((pt.train_ptr, pt.train_idx, pt.val_ptr, pt.val_idx), want):
        assert np.array_equal(a, b)
    assert pt.n_subsets == k * R.shape[0]


@pytest.mark.parametrize("k", [2, 3, 7])
def test_fold_draw_is_balanced_per_core(k):
    r = _rng(5)
    P = r.uniform(0.0, 1.0, (1000, 2))
    R = part.grid_cores((0.0, 0.0, 1.0, 1.0), 4, 2)
    owner = part.assign_cores(P, R)
    labels = part.kfold_labels(owner, R.shape[0], k, _rng(50))
    assert labels.min() >= 0 and labels.max() < k
    for i in range(R.shape[0]):
        c = np.bincount(labels[owner == i], minlength=k)
        assert c.max() - c.min() <= 1
    with pytest.raises(ValueError):
        part.kfold_labels(owner, R.shape[0], 1, _rng(51))
