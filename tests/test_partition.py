"""Host-side input preparation: cores, shells, split and CSR."""
import numpy as np

from paper_1912_13132_amd import partition as part
from paper_1912_13132_amd import workloads as W


def _rng(k):
    return np.random.default_rng(np.random.SeedSequence([1912, 13132, 700 + k]))


def test_grid_partition_structure():
    r = _rng(1)
    P = r.uniform(0, 1, (3000, 2))
    cores = part.grid_cores((0, 0, 1, 1), 4, 3)
    pt = part.build_partition(P, cores, 0.05, 0.1, _rng(2))
    S = pt.n_subsets
    assert S == 12
    # every point has exactly one core; validation points never train
    assert np.bincount(pt.owner, minlength=S).sum() == 3000
    assert not np.intersect1d(pt.train_idx, pt.val_idx).size
    # each validation point is predicted once, by its own core
    assert np.array_equal(np.sort(pt.val_idx), np.nonzero(pt.is_val)[0])
    for i in range(S):
        v = pt.val_idx[pt.val_ptr[i]:pt.val_ptr[i + 1]]
        assert np.all(pt.owner[v] == i)
        core_n = int((pt.owner == i).sum())
        assert len(v) == int(round(0.1 * core_n))
        t = pt.train_idx[pt.train_ptr[i]:pt.train_ptr[i + 1]]
        x0, y0, x1, y1 = cores[i]
        Pt = P[t]
        assert np.all((Pt[:, 0] >= x0 - 0.05) & (Pt[:, 0] <= x1 + 0.05))
        assert np.all((Pt[:, 1] >= y0 - 0.05) & (Pt[:, 1] <= y1 + 0.05))
        # all core training points are present
        core_t = np.nonzero((pt.owner == i) & ~pt.is_val)[0]
        assert np.isin(core_t, t).all()


def test_zero_shell_is_core():
    r = _rng(3)
    P = r.uniform(0, 1, (1000, 2))
    cores = part.grid_cores((0, 0, 1, 1), 2, 2)
    pt = part.build_partition(P, cores, 0.0, 0.1, _rng(4))
    assert pt.train_ptr[-1] + pt.val_ptr[-1] == 1000


def test_overlap_bisection_hits_target():
    r = _rng(5)
    P = r.uniform(0, 1, (20000, 2))
    cores = part.grid_cores((0, 0, 1, 1), 8, 8)
    d, _, cnt = part.find_delta(P, lambda _d: cores, 0.1)
    assert abs(cnt - 1.1 * 20000) <= 0.005 * 1.1 * 20000
    assert part.count_memberships(P, cores, d) == cnt


def test_recursive_division_balances_with_shells():
    r = _rng(6)
    P = r.uniform(0, 1, (40000, 2))
    d = 0.01
    cores = part.recursive_cores(P, (0, 0, 1, 1), 16, d)
    assert cores.shape == (16, 4)
    # cores tile the domain
    assert np.isclose(((cores[:, 2] - cores[:, 0]) * (cores[:, 3] - cores[:, 1])).sum(), 1.0)
    pt = part.build_partition(P, cores, d, 0.0, _rng(7))
    sizes = np.diff(pt.train_ptr)
    assert sizes.max() / sizes.min() < 1.25


def test_cap_drops_shell_first():
    r = _rng(8)
    P = r.uniform(0, 1, (4000, 2))
    cores = part.grid_cores((0, 0, 1, 1), 2, 2)
    pt = part.build_partition(P, cores, 0.3, 0.1, _rng(9), cap=950)
    sizes = np.diff(pt.train_ptr)
    assert sizes.max() <= 950
    for i in range(4):
        t = pt.train_idx[pt.train_ptr[i]:pt.train_ptr[i + 1]]
        core_t = np.nonzero((pt.owner == i) & ~pt.is_val)[0]
        if len(core_t) <= 950:
            assert np.isin(core_t, t).all()


def test_workloads_are_seeded():
    a = W.plain_fp64(n=300)
    b = W.plain_fp64(n=300)
    assert np.array_equal(a.locs, b.locs) and np.array_equal(a.y, b.y)
    assert np.array_equal(a.part.train_idx, b.part.train_idx)
    g = W.theta_grid((0.05, 0.1), 8)
    assert len(g) == 64 and np.isclose(g[0][0], 0.025) and np.isclose(g[-1][1], 0.2)
