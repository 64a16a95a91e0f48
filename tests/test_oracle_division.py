"""Pins of the division oracle (Sec. 2.3 shells, Sec. 2.4 recursive
division) against facts fixed by the paper and by brute force, and the
package's host partitioner against the oracle.

The brute-force checks do not reuse the oracle's recursion: every count is a
direct rectangle test over all points, each cut is re-derived from the
returned cores, and shells are checked through a different formulation (the
Chebyshev distance from a point to the core).
"""
import json
import os

import numpy as np
import pytest

from oracle import division as D
from paper_1912_13132_amd import partition as part
from paper_1912_13132_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _rng(k):
    return np.random.default_rng(np.random.SeedSequence([1912, 13132, 1100 + k]))


def _bbox(R):
    return (R[:, 0].min(), R[:, 1].min(), R[:, 2].max(), R[:, 3].max())


def _check_cuts(P, cores, dom, delta, i0, k, axis):
    """Re-derive the cut of the rectangle holding cores [i0, i0 + k) and
    check it against brute-force counts: the smallest double at which the
    balance of Sec. 2.4 holds (with shells), or a midpoint between points
    that keeps the balance (without shells)."""
    if k == 1:
        return
    kl, ku = k // 2, k - k // 2
    rect = _bbox(cores[i0:i0 + k])
    upper = cores[i0 + kl:i0 + k]
    c = upper[:, axis].min()
    assert np.all(cores[i0:i0 + kl, axis + 2] <= c)

    def f(cc):
        lo_box = list(rect)
        lo_box[axis + 2] = cc
        up_box = list(rect)
        up_box[axis] = cc
        # the rectangle's own held set bounds both parts
        nl = _held_within(P, rect, lo_box, dom, delta)
        nu = _held_within(P, rect, up_box, dom, delta)
        return ku * nl - kl * nu, nl, nu

    if delta > 0:
        assert f(c)[0] >= 0
        if c > rect[axis]:
            assert f(np.nextafter(c, -np.inf))[0] < 0
    else:
        v, nl, nu = f(c)
        assert v >= 0 and ku * (nl - 1) - kl * (nu + 1) < 0
        # the cut lies midway between the rectangle's nearest coordinates on
        # either side of it
        inside = _held_within(P, rect, rect, dom, 0.0, mask=True)
        a = P[inside, axis]
        below, above = a[a < c], a[a >= c]
        if below.size and above.size:
            assert c == 0.5 * (below.max() + above.min())
    _check_cuts(P, cores, dom, delta, i0, kl, 1 - axis)
    _check_cuts(P, cores, dom, delta, i0 + kl, ku, 1 - axis)


def _held_within(P, rect, box, dom, delta, mask=False):
    """Points held by `box` (a part of `rect`) that `rect` also holds (their
    number, or the mask)."""
    x, y = P[:, 0], P[:, 1]
    ok = np.ones(P.shape[0], dtype=bool)
    for b in (rect, box):
        if b[0] != dom[0]:
            ok &= x >= b[0] - delta
        if b[1] != dom[1]:
            ok &= y >= b[1] - delta
        if b[2] != dom[2]:
            ok &= x < b[2] + delta
        if b[3] != dom[3]:
            ok &= y < b[3] + delta
    return ok if mask else int(ok.sum())


@pytest.mark.parametrize("m,delta", [(2, 0.05), (3, 0.04), (7, 0.03), (8, 0.0), (11, 0.0), (16, 0.02)])
def test_every_cut_is_the_smallest_balanced_one(m, delta):
    r = _rng(m)
    P = r.uniform(0, 1, (700, 2)) * np.array([1.5, 1.0])
    dom = (0.0, 0.0, 1.5, 1.0)
    cores = D.divide(P, dom, m, delta)
    assert cores.shape == (m, 4)
    _check_cuts(P, cores, dom, delta, 0, m, 0)


@pytest.mark.parametrize("m", [5, 13, 32])
def test_cores_tile_the_domain(m):
    r = _rng(20 + m)
    P = W.thomas_points(3000, 12, 0.05, r)
    dom = (0.0, 0.0, 1.0, 1.0)
    cores = D.divide(P, dom, m, 0.02)
    area = (cores[:, 2] - cores[:, 0]) * (cores[:, 3] - cores[:, 1])
    assert np.all(area > 0)
    assert area.sum() == pytest.approx(1.0, rel=1e-12)
    for i in range(m):
        for j in range(i + 1, m):
            ox = min(cores[i, 2], cores[j, 2]) - max(cores[i, 0], cores[j, 0])
            oy = min(cores[i, 3], cores[j, 3]) - max(cores[i, 1], cores[j, 1])
            assert ox <= 0 or oy <= 0
    owner = D.owners(P, cores)
    assert owner.min() == 0 and owner.max() < m


def test_power_of_two_without_shells_balances_exactly():
    """Sec. 2.4: for delta = 0 the division gives subsets of similar size;
    with 2^q cores and distinct coordinates they differ by at most one."""
    r = _rng(40)
    P = r.uniform(0, 1, (10_007, 2))
    cores = D.divide(P, (0, 0, 1, 1), 64, 0.0)
    counts = np.bincount(D.owners(P, cores), minlength=64)
    assert counts.max() - counts.min() <= 1
    assert set(counts.tolist()) <= {10_007 // 64, 10_007 // 64 + 1}


def test_paper_weak_scaling_subset_counts():
    """Sec. 4.3.2: dividing 5,000,000 points into 512 subsets without shells
    gives subsets of 9,765 or 9,766 points (printed in the paper)."""
    with open(os.path.join(HERE, "golden", "weak_scaling_counts.json")) as f:
        g = json.load(f)
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 918]))
    P = r.uniform(0, 1, (g["n_points"], 2)) * np.array([2.0, 1.0])
    cores = D.divide(P, (0.0, 0.0, 2.0, 1.0), g["n_subsets"], 0.0)
    counts = np.bincount(D.owners(P, cores), minlength=g["n_subsets"])
    assert set(np.unique(counts).tolist()) <= set(g["allowed_counts"])


@pytest.mark.parametrize("delta", [0.0, 0.03, 0.11])
def test_shell_is_the_chebyshev_neighbourhood(delta):
    """A point is in the shell of core i iff it lies outside the core and at
    Chebyshev distance below delta from it (continuous random points: no
    point sits on an edge)."""
    r = _rng(50)
    P = r.uniform(0, 1, (1500, 2))
    cores = D.divide(P, (0, 0, 1, 1), 9, delta)
    owner = D.owners(P, cores)
    for i in range(9):
        R = cores[i]
        dx = np.maximum(np.maximum(R[0] - P[:, 0], 0.0), P[:, 0] - R[2])
        dy = np.maximum(np.maximum(R[1] - P[:, 1], 0.0), P[:, 1] - R[3])
        expect = np.nonzero((owner != i) & (np.maximum(dx, dy) < delta))[0]
        np.testing.assert_array_equal(D.shell(P, cores, i, delta), expect)


def test_subsets_split_and_all_covering_shells():
    """Validation points never train and are predicted once, by their own
    core; with delta larger than the domain every subset trains on every
    training point (the global CV of Sec. 3.2)."""
    r = _rng(60)
    P = r.uniform(0, 1, (900, 2))
    cores = D.divide(P, (0, 0, 1, 1), 6, 0.05)
    is_val = r.uniform(size=900) < 0.1
    owner, tp, ti, vp, vi = D.subsets(P, cores, 0.05, is_val)
    assert not np.intersect1d(ti, vi).size
    np.testing.assert_array_equal(np.sort(vi), np.nonzero(is_val)[0])
    for i in range(6):
        assert np.all(owner[vi[vp[i]:vp[i + 1]]] == i)
        t = ti[tp[i]:tp[i + 1]]
        assert np.all(np.diff(t) > 0)
    owner, tp, ti, vp, vi = D.subsets(P, cores, 2.0, is_val)
    train = np.nonzero(~is_val)[0]
    for i in range(6):
        np.testing.assert_array_equal(ti[tp[i]:tp[i + 1]], train)
    assert D.memberships(P, cores, 2.0) == 6 * 900
    assert D.memberships(P, cores, 0.0) == 900


def test_memberships_grow_with_the_shell():
    r = _rng(70)
    P = r.uniform(0, 1, (2000, 2))
    cores = D.divide(P, (0, 0, 1, 1), 16, 0.0)
    c = [D.memberships(P, cores, d) for d in (0.0, 0.01, 0.02, 0.05, 0.1)]
    assert c[0] == 2000 and all(a < b for a, b in zip(c, c[1:]))


# -------------------------------------------- host partitioner vs oracle --
def _points(kind, n, r):
    if kind == "uniform":
        return r.uniform(0, 1, (n, 2)), (0.0, 0.0, 1.0, 1.0)
    if kind == "thomas":
        return W.thomas_points(n, 50, 0.03, r), (0.0, 0.0, 1.0, 1.0)
    P, _, _ = W.jittered_lattice_with_gaps(300, 400, 300.0, 400.0, 0.15, 100_000, r)
    P[:, 0] = np.floor(P[:, 0])  # ties on the lattice
    return P, (0.0, 0.0, 300.0, 400.0)


@pytest.mark.parametrize("kind,m,delta", [("uniform", 37, 0.0), ("uniform", 64, 0.01),
                                          ("thomas", 100, 0.02), ("lattice", 250, 3.0)])
def test_host_partitioner_matches_oracle(kind, m, delta):
    r = _rng({"uniform": 1, "thomas": 2, "lattice": 3}[kind] * 100 + m)
    P, dom = _points(kind, 30_000, r)
    cores = D.divide(P, dom, m, delta)
    np.testing.assert_array_equal(part.recursive_cores(P, dom, m, delta), cores)
    assert part.count_memberships(P, cores, delta) == D.memberships(P, cores, delta)
    pt = part.build_partition(P, cores, delta, 0.1, _rng(99))
    owner, tp, ti, vp, vi = D.subsets(P, cores, delta, pt.is_val)
    np.testing.assert_array_equal(pt.owner, owner)
    np.testing.assert_array_equal(pt.train_ptr, tp)
    np.testing.assert_array_equal(pt.train_idx, ti)
    np.testing.assert_array_equal(pt.val_ptr, vp)
    np.testing.assert_array_equal(pt.val_idx, vi)
