"""Division of the spatial domain into cores, shells and a hold-out split
(Sec. 2.3 shells, Sec. 2.4 recursive division, Algorithm 1 steps 2-3).

This is input preparation: it turns locations into the CSR subset lists that
the library and the oracle both consume.  It contains no part of the CV
arithmetic.

Conventions (readings where the paper is silent):
  * A core is a rectangle (xlo, ylo, xhi, yhi), half-open [lo, hi) per axis,
    except that edges on the domain's maximum are closed.  A point belongs to
    exactly one core.
  * The shell of core D_i is the core's rectangle widened by delta on every
    side (axis-aligned), minus the core.  Shells add training points only.
  * The train/validation split is drawn per core, before shells are added:
    round(val_frac * #core) points uniformly without replacement, so each
    validation point is predicted exactly once (by its own core).
  * The recursive division splits the x-range first and alternates axes;
    a rectangle holding m cores is split into floor(m/2) : ceil(m/2) cores
    at the coordinate that makes the (core + shell) point counts of the two
    halves proportional to those core counts (Sec. 2.4 balances them).
  * Optional size cap: subsets above `cap` training points are subsampled,
    shell points dropped first (Sec. 4.3.2 caps shells by random sampling).

recursive_cores, count_memberships and build_partition take device=True to
run the geometry on the GPU (the library's pcv_part_* calls), with results
identical to the host code; the random hold-out split and the cap are drawn
on the host in both cases.

Parallel k-fold CV (the remark closing Sec. 2.2): every point gets a fold
label, drawn per core (a random permutation of the core's points cut into k
folds whose sizes differ by at most one); round j holds out the points
labelled j everywhere, so that its subsets are the hold-out subsets of
Sec. 2.3 for that split (shells drop held-out points too).  The k rounds
become one problem of k * S subsets, round-major, whose summed loss is the
k-fold loss: every point is predicted once, in the round that holds it out.
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Partition:
    core_rect: np.ndarray          # (S, 4) float64: xlo, ylo, xhi, yhi
    delta: float                   # shell width
    train_ptr: np.ndarray          # (S+1,) int64
    train_idx: np.ndarray          # (nnz_T,) int32
    val_ptr: np.ndarray            # (S+1,) int64
    val_idx: np.ndarray            # (nnz_V,) int32
    owner: np.ndarray              # (N,) int32 core of every point
    is_val: np.ndarray             # (N,) bool
    info: dict = field(default_factory=dict)

    @property
    def n_subsets(self):
        return self.core_rect.shape[0]

    def train_sizes(self):
        return np.diff(self.train_ptr)

    def val_sizes(self):
        return np.diff(self.val_ptr)


def _in_rect(P, rect, xmax, ymax):
    """Half-open membership with closed edges on the domain maximum."""
    x, y = P[:, 0], P[:, 1]
    inx = (x >= rect[0]) & ((x < rect[2]) | ((x == rect[2]) & (rect[2] >= xmax)))
    iny = (y >= rect[1]) & ((y < rect[3]) | ((y == rect[3]) & (rect[3] >= ymax)))
    return inx & iny


class _Buckets:
    """Uniform bucket grid over the points for fast rectangle queries."""

    def __init__(self, P, domain, per_bucket=32):
        self.P = P
        self.x0, self.y0, x1, y1 = domain
        n = max(P.shape[0], 1)
        g = int(max(1, min(4096, np.sqrt(n / per_bucket))))
        self.gx = self.gy = g
        self.dx = (x1 - self.x0) / g
        self.dy = (y1 - self.y0) / g
        bx = np.clip(((P[:, 0] - self.x0) / self.dx).astype(np.int64), 0, g - 1)
        by = np.clip(((P[:, 1] - self.y0) / self.dy).astype(np.int64), 0, g - 1)
        key = by * g + bx
        self.order = np.argsort(key, kind="stable")
        self.start = np.searchsorted(key[self.order], np.arange(g * g + 1))

    def candidates(self, rect):
        g = self.gx
        bx0 = int(np.clip(np.floor((rect[0] - self.x0) / self.dx), 0, g - 1))
        bx1 = int(np.clip(np.floor((rect[2] - self.x0) / self.dx), 0, g - 1))
        by0 = int(np.clip(np.floor((rect[1] - self.y0) / self.dy), 0, g - 1))
        by1 = int(np.clip(np.floor((rect[3] - self.y0) / self.dy), 0, g - 1))
        parts = []
        for by in range(by0, by1 + 1):
            a = self.start[by * g + bx0]
            b = self.start[by * g + bx1 + 1]
            parts.append(self.order[a:b])
        return np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)


def grid_cores(domain, nx, ny):
    """nx * ny equal cells of the rectangle domain = (xlo, ylo, xhi, yhi),
    numbered row-major from the lower-left corner (x fastest)."""
    x0, y0, x1, y1 = domain
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)
    xs[-1], ys[-1] = x1, y1
    rects = []
    for j in range(ny):
        for i in range(nx):
            rects.append((xs[i], ys[j], xs[i + 1], ys[j + 1]))
    return np.array(rects, dtype=np.float64)


def recursive_cores(P, domain, m, delta, device=False):
    """Recursive balanced division of Sec. 2.4 into m cores.

    Splits alternate between the x-range (first) and the y-range.  Each split
    position balances the number of points in each half together with its
    shell of width delta, in proportion to the number of cores each half
    receives.  Cores are returned in depth-first (left/bottom first) order.
    """
    P = np.asarray(P, dtype=np.float64)
    if device:
        from . import pcv
        return pcv.part_divide(P, domain, m, delta)
    out = []
    stack = [(np.array(domain, dtype=np.float64), m, 0, np.arange(P.shape[0]))]
    while stack:
        rect, k, axis, cand = stack.pop()
        if k == 1:
            out.append(rect)
            continue
        kl, kr = k // 2, k - k // 2
        a = np.sort(P[cand, axis])
        lo, hi = rect[axis], rect[axis + 2]
        tot = a.shape[0]

        def balance(c):
            cl = np.searchsorted(a, c + delta, side="left")
            cr = tot - np.searchsorted(a, c - delta, side="left")
            return kr * cl - kl * cr

        b_lo, b_hi = lo, hi
        for _ in range(64):
            mid = 0.5 * (b_lo + b_hi)
            if balance(mid) < 0:
                b_lo = mid
            else:
                b_hi = mid
        # b_hi is the smallest cut found with balance >= 0; without shells
        # move it midway between the two neighbouring coordinates, which
        # keeps both counts unchanged
        c = b_hi
        if delta <= 0:
            j = np.searchsorted(a, c)
            if 0 < j < tot:
                c = 0.5 * (a[j - 1] + a[j])
        c = min(max(c, lo), hi)
        ax = P[cand, axis]
        left = rect.copy()
        left[axis + 2] = c
        right = rect.copy()
        right[axis] = c
        # push right first so that the left half is emitted first
        stack.append((right, kr, 1 - axis, cand[ax >= c - delta]))
        stack.append((left, kl, 1 - axis, cand[ax < c + delta]))
    return np.array(out, dtype=np.float64)


def assign_cores(P, core_rect):
    """Core index of every point under the half-open rule (vectorised over
    cores, which tile the domain)."""
    P = np.asarray(P, dtype=np.float64)
    R = np.asarray(core_rect, dtype=np.float64)
    xmax, ymax = R[:, 2].max(), R[:, 3].max()
    domain = (R[:, 0].min(), R[:, 1].min(), xmax, ymax)
    bk = _Buckets(P, domain)
    owner = np.full(P.shape[0], -1, dtype=np.int64)
    for i in range(R.shape[0]):
        cand = bk.candidates(R[i])
        cand = cand[owner[cand] < 0]
        hit = cand[_in_rect(P[cand], R[i], xmax, ymax)]
        owner[hit] = i
    if (owner < 0).any():
        raise ValueError("cores do not cover every point")
    return owner.astype(np.int32)


def _shell_members(P, core_rect, delta, eligible, bk):
    """For every core: indices of eligible points inside the widened
    rectangle but outside the core (its shell)."""
    R = core_rect
    xmax, ymax = R[:, 2].max(), R[:, 3].max()
    xmin, ymin = R[:, 0].min(), R[:, 1].min()
    out = []
    for i in range(R.shape[0]):
        if delta <= 0:
            out.append(np.zeros(0, dtype=np.int64))
            continue
        big = np.array([max(R[i, 0] - delta, xmin), max(R[i, 1] - delta, ymin),
                        min(R[i, 2] + delta, xmax), min(R[i, 3] + delta, ymax)])
        cand = bk.candidates(big)
        cand = cand[eligible[cand]]
        x = P[cand, 0]
        y = P[cand, 1]
        inbig = ((x >= big[0]) & ((x < big[2]) | ((x == big[2]) & (big[2] >= xmax)))
                 & (y >= big[1]) & ((y < big[3]) | ((y == big[3]) & (big[3] >= ymax))))
        incore = ((x >= R[i, 0]) & ((x < R[i, 2]) | ((x == R[i, 2]) & (R[i, 2] >= xmax)))
                  & (y >= R[i, 1]) & ((y < R[i, 3]) | ((y == R[i, 3]) & (R[i, 3] >= ymax))))
        out.append(np.sort(cand[inbig & ~incore]))
    return out


def count_memberships(P, core_rect, delta, device=False):
    """Total number of (point, subset) memberships: sum over subsets of the
    points in core + shell (all points, before any split)."""
    P = np.asarray(P, dtype=np.float64)
    R = np.asarray(core_rect, dtype=np.float64)
    if device:
        from . import pcv
        return pcv.part_count(P, R, delta)
    domain = (R[:, 0].min(), R[:, 1].min(), R[:, 2].max(), R[:, 3].max())
    bk = _Buckets(P, domain)
    shells = _shell_members(P, R, delta, np.ones(P.shape[0], dtype=bool), bk)
    return P.shape[0] + sum(s.shape[0] for s in shells)


def find_delta(P, core_fn, overlap, tol=0.005, iters=40, device=False):
    """Shell width delta such that the total memberships equal
    (1 + overlap) * N within tol (relative).  core_fn(delta) -> core
    rectangles (the recursive division depends on delta; a grid does not).

    The count is monotone in delta; the root is bracketed from a geometric
    first guess (memberships ~ N (1 + perimeter * delta / area)) and refined
    by the Illinois variant of regula falsi."""
    N = P.shape[0]
    target = (1.0 + overlap) * N
    R0 = core_fn(0.0)
    w = R0[:, 2] - R0[:, 0]
    h = R0[:, 3] - R0[:, 1]
    guess = overlap * float(np.mean(w * h)) / float(np.mean(2.0 * (w + h)))

    def g(d):
        R = core_fn(d)
        c = count_memberships(P, R, d, device=device)
        return c - target, R, c

    lo, glo, best = 0.0, N - target, (0.0, R0, N)
    hi = guess
    ghi, R, c = g(hi)
    best = (hi, R, c)
    n_eval = 1
    while ghi < 0 and n_eval < iters:
        lo, glo = hi, ghi
        hi *= 2.0
        ghi, R, c = g(hi)
        best = (hi, R, c)
        n_eval += 1
    side = 0
    while abs(best[2] - target) > tol * target and n_eval < iters:
        d = hi - ghi * (hi - lo) / (ghi - glo) if ghi != glo else 0.5 * (lo + hi)
        if not (lo < d < hi):
            d = 0.5 * (lo + hi)
        gd, R, c = g(d)
        n_eval += 1
        best = (d, R, c)
        if gd < 0:
            lo, glo = d, gd
            if side == -1:
                ghi *= 0.5
            side = -1
        else:
            hi, ghi = d, gd
            if side == 1:
                glo *= 0.5
            side = 1
    return best


def build_partition(P, core_rect, delta, val_frac, rng, cap=None, device=False):
    """CSR subsets from cores: validation split per core, then each subset's
    training set = training points of its core plus its shell (Sec. 2.3).

    rng: numpy Generator for the split and the cap subsampling."""
    P = np.asarray(P, dtype=np.float64)
    R = np.asarray(core_rect, dtype=np.float64)
    S = R.shape[0]
    if device:
        return _build_partition_device(P, R, delta, val_frac, rng, cap)
    owner = assign_cores(P, R)
    order = np.argsort(owner, kind="stable")
    starts = np.searchsorted(owner[order], np.arange(S + 1))
    is_val = np.zeros(P.shape[0], dtype=bool)
    val_lists = []
    core_train = []
    for i in range(S):
        members = order[starts[i]:starts[i + 1]]
        nv = int(round(val_frac * members.shape[0]))
        pick = rng.choice(members.shape[0], size=nv, replace=False) if nv else np.zeros(0, np.int64)
        v = np.sort(members[pick])
        is_val[v] = True
        val_lists.append(v)
    for i in range(S):
        members = order[starts[i]:starts[i + 1]]
        core_train.append(members[~is_val[members]])
    domain = (R[:, 0].min(), R[:, 1].min(), R[:, 2].max(), R[:, 3].max())
    bk = _Buckets(P, domain)
    shells = _shell_members(P, R, delta, ~is_val, bk)
    train_lists = []
    n_capped = 0
    for i in range(S):
        ct, sh = core_train[i], shells[i]
        if cap is not None and ct.shape[0] + sh.shape[0] > cap:
            n_capped += 1
            keep_shell = max(cap - ct.shape[0], 0)
            sh = sh[np.sort(rng.choice(sh.shape[0], size=keep_shell, replace=False))] if keep_shell else sh[:0]
            if ct.shape[0] > cap:
                ct = ct[np.sort(rng.choice(ct.shape[0], size=cap, replace=False))]
        train_lists.append(np.sort(np.concatenate([ct, sh])))
    tptr = np.zeros(S + 1, dtype=np.int64)
    tptr[1:] = np.cumsum([t.shape[0] for t in train_lists])
    vptr = np.zeros(S + 1, dtype=np.int64)
    vptr[1:] = np.cumsum([v.shape[0] for v in val_lists])
    tidx = np.concatenate(train_lists).astype(np.int32) if S else np.zeros(0, np.int32)
    vidx = np.concatenate(val_lists).astype(np.int32) if S else np.zeros(0, np.int32)
    info = dict(memberships=int(tptr[-1] + vptr[-1]), n_capped=n_capped,
                train_min=int(np.diff(tptr).min()), train_max=int(np.diff(tptr).max()),
                val_total=int(vptr[-1]))
    return Partition(core_rect=R, delta=float(delta), train_ptr=tptr, train_idx=tidx,
                     val_ptr=vptr, val_idx=vidx, owner=owner, is_val=is_val, info=info)


def kfold_labels(owner, S, k, rng):
    """Fold label (0..k-1) of every point: per core, in core order, a random
    permutation of its points (increasing index) cut into k consecutive
    folds of sizes differing by at most one."""
    owner = np.asarray(owner)
    if k < 2:
        raise ValueError("k-fold CV needs k >= 2")
    order = np.argsort(owner, kind="stable")
    starts = np.searchsorted(owner[order], np.arange(S + 1))
    labels = np.zeros(owner.shape[0], dtype=np.int32)
    for i in range(S):
        members = order[starts[i]:starts[i + 1]]
        perm = members[rng.permutation(members.shape[0])]
        labels[perm] = (np.arange(members.shape[0]) * k) // max(members.shape[0], 1)
    return labels


def build_partition_kfold(P, core_rect, delta, k, rng, device=False):
    """Parallel k-fold CV: the hold-out subsets of every round j (points
    labelled j held out, kfold_labels), concatenated round-major into one
    Partition of k * S subsets (subset j * S + i: core i in round j; core
    rectangles repeated).  is_val marks nothing; info["labels"] holds the
    fold of every point."""
    P = np.asarray(P, dtype=np.float64)
    R = np.asarray(core_rect, dtype=np.float64)
    S = R.shape[0]
    if device:
        from . import pcv
        owner = pcv.part_subsets(P, R, delta, lists=False)
    else:
        owner = assign_cores(P, R)
    labels = kfold_labels(owner, S, k, rng)
    rounds = []
    for j in range(k):
        held = labels == j
        if device:
            _, tp, ti, vp, vi = pcv.part_subsets(P, R, delta, is_val=held)
        else:
            tp, ti, vp, vi = _subsets_for_split(P, R, delta, owner, held)
        rounds.append((tp, ti, vp, vi))
    tptr = np.zeros(k * S + 1, dtype=np.int64)
    vptr = np.zeros(k * S + 1, dtype=np.int64)
    for j, (tp, _, vp, _) in enumerate(rounds):
        tptr[j * S + 1:(j + 1) * S + 1] = tp[1:] + tptr[j * S]
        vptr[j * S + 1:(j + 1) * S + 1] = vp[1:] + vptr[j * S]
    tidx = np.concatenate([r[1] for r in rounds]).astype(np.int32)
    vidx = np.concatenate([r[3] for r in rounds]).astype(np.int32)
    info = dict(k=int(k), labels=labels, memberships=int(tptr[-1] + vptr[-1]),
                train_min=int(np.diff(tptr).min()), train_max=int(np.diff(tptr).max()),
                val_total=int(vptr[-1]))
    return Partition(core_rect=np.tile(R, (k, 1)), delta=float(delta), train_ptr=tptr, train_idx=tidx,
                     val_ptr=vptr, val_idx=vidx, owner=owner, is_val=np.zeros(P.shape[0], dtype=bool),
                     info=info)


def _subsets_for_split(P, R, delta, owner, is_val):
    """Host CSR of the subsets for a given hold-out mask (no cap)."""
    S = R.shape[0]
    order = np.argsort(owner, kind="stable")
    starts = np.searchsorted(owner[order], np.arange(S + 1))
    domain = (R[:, 0].min(), R[:, 1].min(), R[:, 2].max(), R[:, 3].max())
    shells = _shell_members(P, R, delta, ~is_val, _Buckets(P, domain))
    train, val = [], []
    for i in range(S):
        members = order[starts[i]:starts[i + 1]]
        train.append(np.sort(np.concatenate([members[~is_val[members]], shells[i]])))
        val.append(members[is_val[members]])
    tptr = np.r_[0, np.cumsum([t.shape[0] for t in train])].astype(np.int64)
    vptr = np.r_[0, np.cumsum([v.shape[0] for v in val])].astype(np.int64)
    tidx = np.concatenate(train).astype(np.int32) if S else np.zeros(0, np.int32)
    vidx = np.concatenate(val).astype(np.int32) if S else np.zeros(0, np.int32)
    return tptr, tidx, vptr, vidx


def _split(owner, S, val_frac, rng):
    """The per-core hold-out draw (the same calls in the same order as the
    host path of build_partition)."""
    order = np.argsort(owner, kind="stable")
    starts = np.searchsorted(owner[order], np.arange(S + 1))
    is_val = np.zeros(owner.shape[0], dtype=bool)
    for i in range(S):
        members = order[starts[i]:starts[i + 1]]
        nv = int(round(val_frac * members.shape[0]))
        pick = rng.choice(members.shape[0], size=nv, replace=False) if nv else np.zeros(0, np.int64)
        is_val[members[pick]] = True
    return is_val


def _build_partition_device(P, R, delta, val_frac, rng, cap):
    from . import pcv
    S = R.shape[0]
    owner = pcv.part_subsets(P, R, delta, lists=False)
    is_val = _split(owner, S, val_frac, rng)
    _, tptr, tidx, vptr, vidx = pcv.part_subsets(P, R, delta, is_val=is_val)
    n_capped = 0
    if cap is not None:
        # the host path's cap, in the same order: shell points dropped first
        lists = []
        for i in range(S):
            t = tidx[tptr[i]:tptr[i + 1]]
            ct, sh = t[owner[t] == i], t[owner[t] != i]
            if ct.shape[0] + sh.shape[0] > cap:
                n_capped += 1
                keep_shell = max(cap - ct.shape[0], 0)
                sh = sh[np.sort(rng.choice(sh.shape[0], size=keep_shell, replace=False))] if keep_shell else sh[:0]
                if ct.shape[0] > cap:
                    ct = ct[np.sort(rng.choice(ct.shape[0], size=cap, replace=False))]
            lists.append(np.sort(np.concatenate([ct, sh])))
        tptr = np.zeros(S + 1, dtype=np.int64)
        tptr[1:] = np.cumsum([t.shape[0] for t in lists])
        tidx = np.concatenate(lists).astype(np.int32) if S else np.zeros(0, np.int32)
    info = dict(memberships=int(tptr[-1] + vptr[-1]), n_capped=n_capped,
                train_min=int(np.diff(tptr).min()), train_max=int(np.diff(tptr).max()),
                val_total=int(vptr[-1]))
    return Partition(core_rect=R, delta=float(delta), train_ptr=tptr, train_idx=tidx,
                     val_ptr=vptr, val_idx=vidx, owner=owner, is_val=is_val, info=info)
