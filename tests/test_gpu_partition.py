"""The device partitioner (pcv_part_*) against the oracle's division written
out from the definitions of Sec. 2.3 (shells) and Sec. 2.4 (recursive
balanced division): identical core rectangles, membership counts and
subset lists (bit for bit), on seeded point sets with the workloads'
structure, with and without shells and with the hold-out split.  The
oracle has no size cap (a sampling option of the workloads, not part of the
division), so the capped case is checked against the host partitioner, whose
uncapped output is itself pinned to the oracle on the CPU."""
import sys

import numpy as np
import pytest

from oracle import division as D
from paper_1912_13132_amd import partition as part
from paper_1912_13132_amd import pcv
from paper_1912_13132_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def _rng(k):
    return np.random.default_rng(np.random.SeedSequence([1912, 13132, 1000 + k]))


def _points(kind, n, r):
    if kind == "uniform":
        return r.uniform(0, 1, (n, 2)), (0.0, 0.0, 1.0, 1.0)
    if kind == "thomas":
        return W.thomas_points(n, 50, 0.03, r), (0.0, 0.0, 1.0, 1.0)
    # jittered lattice with gaps, with ties on the lattice (no jitter in x)
    P, _, _ = W.jittered_lattice_with_gaps(300, 400, 300.0, 400.0, 0.15, 100_000, r)
    P[:, 0] = np.floor(P[:, 0])
    return P, (0.0, 0.0, 300.0, 400.0)


def _same_as_oracle(pt, P, cores, delta):
    owner, tp, ti, vp, vi = D.subsets(P, cores, delta, pt.is_val)
    np.testing.assert_array_equal(pt.owner, owner)
    np.testing.assert_array_equal(pt.train_ptr, tp)
    np.testing.assert_array_equal(pt.train_idx, ti)
    np.testing.assert_array_equal(pt.val_ptr, vp)
    np.testing.assert_array_equal(pt.val_idx, vi)


def _same_partition(a, b):
    np.testing.assert_array_equal(a.owner, b.owner)
    np.testing.assert_array_equal(a.is_val, b.is_val)
    np.testing.assert_array_equal(a.train_ptr, b.train_ptr)
    np.testing.assert_array_equal(a.train_idx, b.train_idx)
    np.testing.assert_array_equal(a.val_ptr, b.val_ptr)
    np.testing.assert_array_equal(a.val_idx, b.val_idx)


@pytest.mark.parametrize("kind,m,delta", [("uniform", 37, 0.0), ("uniform", 64, 0.01),
                                          ("thomas", 100, 0.02), ("lattice", 250, 3.0)])
def test_recursive_division_matches_host(kind, m, delta):
    r = _rng({"uniform": 1, "thomas": 2, "lattice": 3}[kind] * 100 + m)
    P, dom = _points(kind, 60_000, r)
    say(f"[case] divide {kind} n={len(P)} m={m} delta={delta}")
    ref = D.divide(P, dom, m, delta)
    dev = part.recursive_cores(P, dom, m, delta, device=True)
    np.testing.assert_array_equal(dev, ref)
    assert part.count_memberships(P, ref, delta, device=True) == D.memberships(P, ref, delta)


@pytest.mark.parametrize("kind,m,delta,cap", [("uniform", 30, 0.0, None), ("thomas", 64, 0.02, None),
                                              ("thomas", 49, 0.03, 1500), ("lattice", 120, 4.0, None)])
def test_subsets_match_host(kind, m, delta, cap):
    r = _rng(7 + m)
    P, dom = _points(kind, 80_000, r)
    cores = D.divide(P, dom, m, delta)
    say(f"[case] subsets {kind} n={len(P)} m={m} delta={delta} cap={cap}")
    b = part.build_partition(P, cores, delta, 0.1, _rng(99), cap=cap, device=True)
    if cap is None:
        _same_as_oracle(b, P, cores, delta)
    a = part.build_partition(P, cores, delta, 0.1, _rng(99), cap=cap)
    _same_partition(a, b)
    assert a.info == b.info


def test_large_recipe_partition_matches_host():
    """The 5M-point workload's division (2,400 cores, 20% overlap), host vs
    device, end to end (delta search included)."""
    say("[case] large partition host vs device, device vs oracle")
    h = W.large()
    d = W.large(device=True)
    np.testing.assert_array_equal(d.part.core_rect, h.part.core_rect)
    assert d.part.delta == h.part.delta
    _same_partition(d.part, h.part)
    # the oracle's division at the delta the device search found
    P = d.locs
    dom = (0.0, 0.0, 2000.0, 2500.0)
    np.testing.assert_array_equal(D.divide(P, dom, d.part.n_subsets, d.part.delta), d.part.core_rect)
    _same_as_oracle(d.part, P, d.part.core_rect, d.part.delta)


def test_partition_rejects_points_outside_the_cores():
    P = np.array([[0.5, 0.5], [2.0, 2.0]])
    cores = np.array([[0.0, 0.0, 1.0, 1.0]])
    with pytest.raises(pcv.PcvError) as e:
        pcv.part_subsets(P, cores, 0.0)
    assert e.value.status == 1
