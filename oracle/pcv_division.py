"""Division of the spatial domain into cores and training / validation
subsets, written out from the definitions of Sec. 2.3 (shells) and Sec. 2.4
(recursive balanced division) of arXiv:1912.13132 (Algorithm 1, steps 2-3).

TEST INFRASTRUCTURE ONLY: the reference for the device partitioner (and for
the package's host partitioner).  Nothing in the product path imports it.
No bucket grids, no radix sorts, no precomputed tables: every membership is
a direct comparison of a point's coordinates with a rectangle's edges, and
the only library primitives are sorting and counting in a sorted array.

Readings (where the paper is silent; each is listed in the design notes):
  * A rectangle is (xlo, ylo, xhi, yhi), half-open [lo, hi) per axis, except
    that an edge on the domain's maximum is closed.  The domain is the
    bounding box of the cores.
  * Shell of a core: the core widened by delta on every side, clipped to the
    domain, minus the core.  Shells add training points only.
  * Recursive division: a rectangle holding k cores is cut across one axis
    (the x-range first, then alternating) into a lower part with floor(k/2)
    cores and an upper part with ceil(k/2).  A part "together with its
    shell" holds the points within delta of it across every cut that bounds
    it: below c + delta for the lower part, at or above c - delta for the
    upper part, among the points the rectangle itself holds that way (the
    domain boundary bounds nothing: no point lies outside the domain).  The
    cut c is the smallest double in (lo, hi] at which
    ceil(k/2) * n_lower(c) >= floor(k/2) * n_upper(c); the counts are
    monotone in c, so that double is unique, and c = hi if there is none.
  * Without shells (delta = 0) the cut is then moved to the midpoint of the
    nearest point coordinates below it and at or above it, which leaves
    both counts unchanged; the cut stays inside [lo, hi].
  * Cores are numbered depth first, the lower part before the upper part.
  * A point on no core's rectangle is an error; ties cannot occur between
    half-open cores that tile the domain (the lowest index would win).
"""
import numpy as np

_SIGN = np.int64(-0x8000000000000000)


def _key(x):
    """Order-preserving map of a double to an integer (bit pattern, with
    negative values mirrored)."""
    i = int(np.array(x, dtype=np.float64).view(np.int64))
    return i if i >= 0 else -(i & 0x7FFFFFFFFFFFFFFF)


def _unkey(k):
    bits = k if k >= 0 else (-k) | int(_SIGN)
    return float(np.array(bits, dtype=np.int64).view(np.float64))


def smallest_double(pred, lo, hi):
    """Smallest double c with lo < c <= hi and pred(c), for pred monotone
    (False below some point, True above); hi if no such double exists."""
    a, b = _key(lo), _key(hi)   # invariant: pred false at a (or a = lo), answer in (a, b]
    if not pred(hi):
        return float(hi)
    while b - a > 1:
        m = (a + b) // 2
        if pred(_unkey(m)):
            b = m
        else:
            a = m
    return _unkey(b)


def divide(locs, domain, m, delta):
    """Recursive balanced division (Sec. 2.4) of `domain` (xlo, ylo, xhi,
    yhi) into m cores; returns float64 (m, 4) in depth-first order."""
    P = np.asarray(locs, dtype=np.float64).reshape(-1, 2)
    out = []

    def rec(rect, k, axis, held):
        # held: indices of the points the rectangle holds together with its shell
        if k == 1:
            out.append(rect)
            return
        kl, ku = k // 2, k - k // 2
        a = np.sort(P[held, axis])
        tot = a.shape[0]

        def n_lower(c):
            return int(np.searchsorted(a, c + delta, side="left"))          # a < c + delta

        def n_upper(c):
            return tot - int(np.searchsorted(a, c - delta, side="left"))    # a >= c - delta

        lo, hi = float(rect[axis]), float(rect[axis + 2])
        c = smallest_double(lambda x: ku * n_lower(x) - kl * n_upper(x) >= 0, lo, hi)
        if delta <= 0:
            j = int(np.searchsorted(a, c, side="left"))                      # points below c
            if 0 < j < tot:
                c = 0.5 * (a[j - 1] + a[j])
        c = min(max(c, lo), hi)
        low = list(rect)
        low[axis + 2] = c
        up = list(rect)
        up[axis] = c
        x = P[held, axis]
        rec(tuple(low), kl, 1 - axis, held[x < c + delta])
        rec(tuple(up), ku, 1 - axis, held[x >= c - delta])

    rec(tuple(float(v) for v in domain), int(m), 0, np.arange(P.shape[0]))
    return np.array(out, dtype=np.float64).reshape(-1, 4)


def _inside(P, lo_x, lo_y, hi_x, hi_y, close_x, close_y):
    """Half-open membership of points in [lo_x, hi_x) x [lo_y, hi_y), with
    the upper edge closed where close_* is set."""
    x, y = P[:, 0], P[:, 1]
    inx = (x >= lo_x) & ((x < hi_x) | (close_x & (x == hi_x)))
    iny = (y >= lo_y) & ((y < hi_y) | (close_y & (y == hi_y)))
    return inx & iny


class _XIndex:
    """Points sorted by x, to restrict a rectangle test to an x-strip."""

    def __init__(self, P):
        self.P = P
        self.order = np.argsort(P[:, 0], kind="stable")
        self.xs = P[self.order, 0]

    def strip(self, x0, x1):
        """Indices (in no particular order) of the points with x0 <= x <= x1."""
        a = np.searchsorted(self.xs, x0, side="left")
        b = np.searchsorted(self.xs, x1, side="right")
        return self.order[a:b]


def _domain(R):
    return R[:, 0].min(), R[:, 1].min(), R[:, 2].max(), R[:, 3].max()


def owners(locs, core_rect, index=None):
    """Core of every point (half-open cores, edges on the domain maximum
    closed, lowest index first)."""
    P = np.asarray(locs, dtype=np.float64).reshape(-1, 2)
    R = np.asarray(core_rect, dtype=np.float64).reshape(-1, 4)
    xmin, ymin, xmax, ymax = _domain(R)
    ix = index or _XIndex(P)
    owner = np.full(P.shape[0], -1, dtype=np.int64)
    for i in range(R.shape[0]):
        cand = ix.strip(R[i, 0], R[i, 2])
        cand = cand[owner[cand] < 0]
        hit = _inside(P[cand], R[i, 0], R[i, 1], R[i, 2], R[i, 3], R[i, 2] >= xmax, R[i, 3] >= ymax)
        owner[cand[hit]] = i
    if (owner < 0).any():
        raise ValueError("a point lies on no core")
    return owner


def shell(locs, core_rect, i, delta, index=None):
    """Indices (increasing) of the points in the shell of core i: inside the
    core widened by delta on every side and clipped to the domain, outside
    the core."""
    P = np.asarray(locs, dtype=np.float64).reshape(-1, 2)
    R = np.asarray(core_rect, dtype=np.float64).reshape(-1, 4)
    if delta <= 0:
        return np.zeros(0, dtype=np.int64)
    xmin, ymin, xmax, ymax = _domain(R)
    ix = index or _XIndex(P)
    x0, y0 = max(R[i, 0] - delta, xmin), max(R[i, 1] - delta, ymin)
    x1, y1 = min(R[i, 2] + delta, xmax), min(R[i, 3] + delta, ymax)
    cand = ix.strip(x0, x1)
    Q = P[cand]
    wide = _inside(Q, x0, y0, x1, y1, x1 >= xmax, y1 >= ymax)
    core = _inside(Q, R[i, 0], R[i, 1], R[i, 2], R[i, 3], R[i, 2] >= xmax, R[i, 3] >= ymax)
    return np.sort(cand[wide & ~core])


def memberships(locs, core_rect, delta):
    """sum_i |core_i + shell_i| over all points (before any split)."""
    P = np.asarray(locs, dtype=np.float64).reshape(-1, 2)
    R = np.asarray(core_rect, dtype=np.float64).reshape(-1, 4)
    ix = _XIndex(P)
    owners(P, R, ix)  # every point in exactly one core
    return int(P.shape[0] + sum(shell(P, R, i, delta, ix).shape[0] for i in range(R.shape[0])))


def subsets(locs, core_rect, delta, is_val=None):
    """The subsets of Sec. 2.3: subset i trains on the points of core i and
    of its shell that are not held out, and validates on the held-out points
    of core i.  is_val: bool (N,) or None (nothing held out).
    Returns (owner, train_ptr, train_idx, val_ptr, val_idx); lists increase
    within each subset."""
    P = np.asarray(locs, dtype=np.float64).reshape(-1, 2)
    R = np.asarray(core_rect, dtype=np.float64).reshape(-1, 4)
    N, S = P.shape[0], R.shape[0]
    v = np.zeros(N, dtype=bool) if is_val is None else np.asarray(is_val, dtype=bool)
    ix = _XIndex(P)
    owner = owners(P, R, ix)
    by_core = np.argsort(owner, kind="stable")        # increasing index within a core
    start = np.searchsorted(owner[by_core], np.arange(S + 1))
    train, val = [], []
    for i in range(S):
        core = by_core[start[i]:start[i + 1]]
        sh = shell(P, R, i, delta, ix)
        train.append(np.sort(np.concatenate([core[~v[core]], sh[~v[sh]]])))
        val.append(core[v[core]])
    tptr = np.r_[0, np.cumsum([t.shape[0] for t in train])].astype(np.int64)
    vptr = np.r_[0, np.cumsum([t.shape[0] for t in val])].astype(np.int64)
    tidx = np.concatenate(train).astype(np.int32) if S else np.zeros(0, np.int32)
    vidx = np.concatenate(val).astype(np.int32) if S else np.zeros(0, np.int32)
    return owner.astype(np.int32), tptr, tidx, vptr, vidx


def kfold_subsets(locs, core_rect, delta, labels, k):
    """Parallel k-fold CV (the remark closing Sec. 2.2), read as k rounds of
    the hold-out CV of Sec. 2.3: round j holds out every point whose fold
    label is j.  Returns the subsets of all rounds concatenated round-major
    (subset j * S + i = core i in round j), as (train_ptr, train_idx,
    val_ptr, val_idx); the summed SSPE over them is the k-fold loss.
    labels: int (N,) fold of every point, an input (the draw is not part of
    the method)."""
    labels = np.asarray(labels)
    tp_all, ti_all, vp_all, vi_all = [np.zeros(1, np.int64)], [], [np.zeros(1, np.int64)], []
    for j in range(k):
        _, tp, ti, vp, vi = subsets(locs, core_rect, delta, is_val=labels == j)
        tp_all.append(tp[1:] + tp_all[-1][-1])
        vp_all.append(vp[1:] + vp_all[-1][-1])
        ti_all.append(ti)
        vi_all.append(vi)
    return (np.concatenate(tp_all), np.concatenate(ti_all).astype(np.int32),
            np.concatenate(vp_all), np.concatenate(vi_all).astype(np.int32))
