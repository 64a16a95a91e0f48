"""Parity at the full workload sizes, in the launch configuration bench.py
times (all subsets in one evaluation, graph replay, mixed precision with one
refinement sweep): the per-subset losses of a seeded sample of subsets are
recomputed one by one by the FP64 oracle.  Mixed path: 1e-6 relative per
subset (the loss tolerance); FP64 path: 1e-10.

The whole-problem invariants are checked too: the loss is the fixed-order
sum of the per-subset losses, every validation point is counted once, and
the mixed and FP64 GPU losses agree within 1e-6.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1912_13132_amd import pcv
from paper_1912_13132_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def _sample(w, k, seed):
    pt = w.part
    act = np.nonzero(np.diff(pt.val_ptr) > 0)[0]
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 900 + seed]))
    pick = r.choice(act, size=min(k, act.size), replace=False)
    # always include the largest and the smallest subset
    n = np.diff(pt.train_ptr)
    return np.unique(np.r_[pick, act[np.argmax(n[act])], act[np.argmin(n[act])]])


def _check(w, th, n_sample, seed, precs=("mixed", "fp64")):
    pt = w.part
    pick = _sample(w, n_sample, seed)
    say(f"[case] {w.name} full size N={len(w.y)} S={pt.n_subsets} sample={pick.tolist()}")
    ref = oracle.cv_loss(w.locs, w.y, pt.train_ptr, pt.train_idx, pt.val_ptr, pt.val_idx,
                         th.cov, th.range, th.lambda_, subsets=pick)
    losses = {}
    for prec, tol in (("mixed", 1e-6), ("fp64", 1e-10)):
        if prec not in precs:
            continue
        with pcv.Problem.from_workload(w, prec=prec) as P:
            loss, rep = P.eval(th, report=True)
        z = rep["per_subset_sspe"]
        rel = np.abs(z[pick] - ref["per_subset_sspe"]) / np.maximum(ref["per_subset_sspe"], 1e-300)
        say(f"   {prec}: loss {loss:.12g} max sampled rel err {rel.max():.2e} fallback {rep['n_fallback_fp64']}")
        assert rel.max() <= tol
        assert rep["n_val"] == int(pt.val_ptr[-1])
        assert abs(loss - math.fsum(z)) <= 1e-12 * abs(loss)
        losses[prec] = loss
    if len(losses) == 2:
        assert abs(losses["mixed"] - losses["fp64"]) <= 1e-6 * abs(losses["fp64"])


def test_batched_full_size_theta_grid_corners():
    w = W.batched()
    g = W.theta_grid(w.theta_true, 8)
    for k in (0, 63):
        _check(w, pcv.theta(*g[k], cov=w.cov), 6, k)


def test_uneven_full_size():
    w = W.uneven()
    _check(w, pcv.theta(*w.theta_true, cov=w.cov), 6, 1)


def test_large_full_size_sampled():
    w = W.large()
    _check(w, pcv.theta(*w.theta_true, cov=w.cov), 4, 2)
