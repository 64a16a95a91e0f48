"""Parallel k-fold CV on the GPU: the k rounds of hold-out subsets form one
problem of k * S subsets (round-major) evaluated by pcv_eval.

  * the device construction of the k-fold subsets equals the host's bit for
    bit (and the host's equals the division oracle, tests/test_kfold.py);
  * the k-fold loss and every subset's SSPE against the FP64 oracle, within
    1e-10 (FP64 path) and 1e-6 (mixed path);
  * leave-one-out (one core, k = N) against the closed form
    sum_i ([K^-1 y]_i / [K^-1]_ii)^2.
"""
import sys

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_1912_13132_amd import partition as part
from paper_1912_13132_amd import pcv
from parity_util import TOL_SSPE, check_sspe

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def _rng(k):
    return np.random.default_rng(np.random.SeedSequence([1912, 13132, 1400 + k]))


@pytest.fixture(scope="module")
def data():
    r = _rng(0)
    P = r.uniform(0.0, 1.0, (2000, 2))
    y = np.sin(6.0 * P[:, 0]) + np.cos(4.0 * P[:, 1]) + 0.3 * r.standard_normal(2000)
    return P, y


@pytest.mark.parametrize("k,delta", [(2, 0.05), (5, 0.08)])
def test_device_kfold_partition_matches_host(data, k, delta):
    P, _ = data
    R = part.grid_cores((0.0, 0.0, 1.0, 1.0), 2, 3)
    say(f"[case] k-fold partition device vs host k={k} delta={delta}")
    h = part.build_partition_kfold(P, R, delta, k, _rng(10 + k))
    d = part.build_partition_kfold(P, R, delta, k, _rng(10 + k), device=True)
    assert np.array_equal(h.info["labels"], d.info["labels"])
    for a, b in ((h.train_ptr, d.train_ptr), (h.train_idx, d.train_idx), (h.val_ptr, d.val_ptr),
                 (h.val_idx, d.val_idx)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_kfold_loss_against_oracle(data, prec):
    P, y = data
    k = 5
    R = part.grid_cores((0.0, 0.0, 1.0, 1.0), 2, 2)
    pt = part.build_partition_kfold(P, R, 0.08, k, _rng(20))
    say(f"[case] k-fold loss k={k} S={pt.n_subsets} prec={prec}")
    ref = oracle.cv_loss(P, y, pt.train_ptr, pt.train_idx, pt.val_ptr, pt.val_idx, 0, 0.2, 0.05)
    with pcv.Problem(P, y, pt.train_ptr, pt.train_idx, pt.val_ptr, pt.val_idx, pt.core_rect, prec=prec) as Q:
        loss, rep = Q.eval(pcv.theta(0.2, 0.05), report=True)
    assert rep["n_val"] == ref["n_val"] == P.shape[0]
    assert abs(loss - ref["sspe"]) <= TOL_SSPE[prec] * ref["sspe"]
    check_sspe(rep["per_subset_sspe"], ref["per_subset_sspe"], prec, say)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_leave_one_out_against_closed_form(prec):
    r = _rng(30)
    N = 150
    P = r.uniform(0.0, 1.0, (N, 2))
    y = r.standard_normal(N)
    R = np.array([[0.0, 0.0, 1.0, 1.0]])
    pt = part.build_partition_kfold(P, R, 0.0, N, _rng(31))
    assert pt.n_subsets == N and np.all(np.diff(pt.val_ptr) == 1)
    say(f"[case] leave-one-out N={N} prec={prec}")
    theta, lam = 0.3, 0.1
    d = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
    Ki = sla.inv(np.exp(-d / theta) + lam * np.eye(N))
    e = (Ki @ y) / np.diag(Ki)
    want = float(np.sum(e * e))
    with pcv.Problem(P, y, pt.train_ptr, pt.train_idx, pt.val_ptr, pt.val_idx, pt.core_rect, prec=prec) as Q:
        loss, rep = Q.eval(pcv.theta(theta, lam), report=True)
    say(f"   rel err {abs(loss - want) / want:.2e}")
    assert abs(loss - want) <= TOL_SSPE[prec] * want
    # subset j validates the one point val_idx[j]
    np.testing.assert_allclose(rep["per_subset_sspe"], (e * e)[pt.val_idx], rtol=TOL_SSPE[prec], atol=0)
