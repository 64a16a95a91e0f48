"""Seeded synthetic workloads shaped like the paper's experiments.

Input generation only: locations, a simulated response and the subset CSR.
This module holds no part of the CV arithmetic (no kriging, no loss); both
the library's tests/benchmark and the oracle read its outputs.  It simulates
data from the model of eq. (1) with its own covariance code (data synthesis
only; nothing on the evaluation path calls it).

Workloads (sizes from the paper's experiments and the benchmark targets):
  plain_fp64   2,000 uniform points on [0,1]^2, exponential GP (range 0.1,
               nugget 0.05) by dense Cholesky; 2x2 grid, 10% overlap,
               10% of each core held out.
  batched      100,000 uniform points, exponential field (range 0.05,
               nugget 0.1) by circulant embedding; 16x16 grid, 10% overlap;
               8x8 geometric (range, nugget) grid around the truth.
  uneven       1,000,000 Thomas-process points (200 parents, sigma 0.02),
               Matern-3/2 field (range 0.03, nugget 0.02); 32x32 grid,
               10% overlap, subsets capped at 4,000 training points.
  large        5,000,000 points on a jittered 2,170 x 2,712 lattice over
               [0,2000] x [0,2500] with 15% of the nodes removed in random
               rectangular gaps (stand-in for the LiDAR strips of Sec. 4.1);
               exponential field (range 50, nugget 0.1); recursive division
               (Sec. 2.4) into 2,400 cores with 20% overlap.
Seeds: SeedSequence([1912, 13132, c]) spawned into child streams
(locations, field, split, queries, optimisers).
"""
from dataclasses import dataclass, field

import numpy as np

from . import partition as part

COV_EXP = 0
COV_MATERN32 = 1

WORKLOAD_IDS = {"plain_fp64": 1, "batched": 2, "uneven": 3, "large": 4, "serving": 5}


@dataclass
class Workload:
    name: str
    locs: np.ndarray            # (N, 2) float64
    y: np.ndarray               # (N,) float64
    part: part.Partition
    cov: int
    theta_true: tuple           # (range, lambda)
    domain: tuple
    info: dict = field(default_factory=dict)


def streams(c):
    ss = np.random.SeedSequence([1912, 13132, int(c)])
    kids = ss.spawn(5)
    return [np.random.default_rng(k) for k in kids]   # locations, field, split, queries, optimisers


# ---------------------------------------------------------------- fields ---
def _corr(kind, d, rng_):
    t = d / rng_
    if kind == COV_EXP:
        return np.exp(-t)
    return (1.0 + t) * np.exp(-t)


def lattice_field(nx, ny, hx, hy, kind, range_, rng):
    """Stationary GP on an nx x ny lattice (spacings hx, hy) by circulant
    embedding on a 2x periodic torus; negative eigenvalues are clipped to 0,
    so the field is approximate (it only needs to look realistic)."""
    mx, my = 2 * nx, 2 * ny
    ix = np.minimum(np.arange(mx), mx - np.arange(mx)) * hx
    iy = np.minimum(np.arange(my), my - np.arange(my)) * hy
    d = np.sqrt(ix[None, :] ** 2 + iy[:, None] ** 2)
    base = _corr(kind, d, range_)
    lam = np.fft.rfft2(base).real
    del base, d
    lam = np.maximum(lam, 0.0)
    z = rng.standard_normal((my, mx))
    f = np.fft.irfft2(np.fft.rfft2(z) * np.sqrt(lam), s=(my, mx))
    return f[:ny, :nx].astype(np.float64)   # unit variance up to the clipping


def _bilinear(F, x0, y0, hx, hy, P):
    ny, nx = F.shape
    gx = np.clip((P[:, 0] - x0) / hx, 0, nx - 1 - 1e-9)
    gy = np.clip((P[:, 1] - y0) / hy, 0, ny - 1 - 1e-9)
    i = np.floor(gx).astype(np.int64)
    j = np.floor(gy).astype(np.int64)
    fx, fy = gx - i, gy - j
    return ((1 - fx) * (1 - fy) * F[j, i] + fx * (1 - fy) * F[j, i + 1]
            + (1 - fx) * fy * F[j + 1, i] + fx * fy * F[j + 1, i + 1])


# ------------------------------------------------------------- workloads ---
def plain_fp64(n=2000, grid=(2, 2), overlap=0.1, val_frac=0.1, seed_id=1, device=False):
    r_loc, r_field, r_split, _, _ = streams(seed_id)
    P = r_loc.uniform(0.0, 1.0, size=(n, 2))
    dx = P[:, 0][:, None] - P[:, 0][None, :]
    dy = P[:, 1][:, None] - P[:, 1][None, :]
    C = np.exp(-np.sqrt(dx * dx + dy * dy) / 0.1) + 0.05 * np.eye(n)
    y = np.linalg.cholesky(C) @ r_field.standard_normal(n)
    dom = (0.0, 0.0, 1.0, 1.0)
    cores = part.grid_cores(dom, *grid)
    delta, _, cnt = part.find_delta(P, lambda d: cores, overlap, device=device)
    pt = part.build_partition(P, cores, delta, val_frac, r_split, device=device)
    return Workload("plain_fp64", P, y, pt, COV_EXP, (0.1, 0.05), dom,
                    dict(memberships_all=cnt))


def batched(n=100_000, grid=(16, 16), overlap=0.1, val_frac=0.1, lattice=2048, seed_id=2, device=False):
    r_loc, r_field, r_split, _, _ = streams(seed_id)
    P = r_loc.uniform(0.0, 1.0, size=(n, 2))
    h = 1.0 / (lattice - 1)
    F = lattice_field(lattice, lattice, h, h, COV_EXP, 0.05, r_field)
    y = _bilinear(F, 0.0, 0.0, h, h, P) + np.sqrt(0.1) * r_field.standard_normal(n)
    dom = (0.0, 0.0, 1.0, 1.0)
    cores = part.grid_cores(dom, *grid)
    delta, _, cnt = part.find_delta(P, lambda d: cores, overlap, device=device)
    pt = part.build_partition(P, cores, delta, val_frac, r_split, device=device)
    return Workload("batched", P, y, pt, COV_EXP, (0.05, 0.1), dom, dict(memberships_all=cnt))


def theta_grid(theta_true, k=8):
    """k x k geometric grid on [theta/2, 2 theta] x [lambda/2, 2 lambda]
    (Sec. 3.1 uses such a grid with 15 values per axis)."""
    r0, l0 = theta_true
    f = 4.0 ** (np.arange(k) / (k - 1))
    return [(r0 / 2 * a, l0 / 2 * b) for a in f for b in f]


def thomas_points(n, n_parents_mean, sigma, rng):
    npar = max(1, rng.poisson(n_parents_mean))
    parents = rng.uniform(0.0, 1.0, size=(npar, 2))
    counts = rng.multinomial(n, np.full(npar, 1.0 / npar))
    pid = np.repeat(np.arange(npar), counts)
    P = parents[pid] + sigma * rng.standard_normal((n, 2))
    bad = (P < 0).any(1) | (P > 1).any(1)
    while bad.any():
        k = int(bad.sum())
        P[bad] = parents[pid[bad]] + sigma * rng.standard_normal((k, 2))
        bad = (P < 0).any(1) | (P > 1).any(1)
    return P


def uneven(n=1_000_000, grid=(32, 32), overlap=0.1, val_frac=0.1, cap=4000,
           lattice=2048, seed_id=3, device=False):
    r_loc, r_field, r_split, _, _ = streams(seed_id)
    P = thomas_points(n, 200, 0.02, r_loc)
    h = 1.0 / (lattice - 1)
    F = lattice_field(lattice, lattice, h, h, COV_MATERN32, 0.03, r_field)
    y = _bilinear(F, 0.0, 0.0, h, h, P) + np.sqrt(0.02) * r_field.standard_normal(n)
    dom = (0.0, 0.0, 1.0, 1.0)
    cores = part.grid_cores(dom, *grid)
    delta, _, cnt = part.find_delta(P, lambda d: cores, overlap, device=device)
    pt = part.build_partition(P, cores, delta, val_frac, r_split, cap=cap, device=device)
    return Workload("uneven", P, y, pt, COV_MATERN32, (0.03, 0.02), dom, dict(memberships_all=cnt))


def jittered_lattice_with_gaps(nx, ny, W, H, frac_removed, n_keep, rng):
    hx, hy = W / nx, H / ny
    keep = np.ones((ny, nx), dtype=bool)
    target_removed = nx * ny - n_keep
    removed = 0
    while removed < target_removed:
        w, h = rng.uniform(20.0, 250.0, size=2)
        x0, y0 = rng.uniform(0.0, W - w), rng.uniform(0.0, H - h)
        i0, i1 = int(x0 / hx), int(np.ceil((x0 + w) / hx))
        j0, j1 = int(y0 / hy), int(np.ceil((y0 + h) / hy))
        blk = keep[j0:j1, i0:i1]
        newly = int(blk.sum())
        if removed + newly > target_removed:
            # trim the last rectangle: drop its first surviving nodes only
            need = target_removed - removed
            jj, ii = np.nonzero(blk)
            blk[jj[:need], ii[:need]] = False
            removed += need
        else:
            blk[:] = False
            removed += newly
    jj, ii = np.nonzero(keep)
    P = np.empty((jj.shape[0], 2))
    P[:, 0] = (ii + rng.uniform(0.0, 1.0, jj.shape[0])) * hx
    P[:, 1] = (jj + rng.uniform(0.0, 1.0, jj.shape[0])) * hy
    return P, (ii, jj), (hx, hy)


LARGE_DELTA = None   # shell width found by find_delta on the large workload


def large(n=5_000_000, nx=2170, ny=2712, W=2000.0, H=2500.0, n_cores=2400,
          overlap=0.2, val_frac=0.1, delta=None, seed_id=4, device=False):
    r_loc, r_field, r_split, _, _ = streams(seed_id)
    P, (ii, jj), (hx, hy) = jittered_lattice_with_gaps(nx, ny, W, H, 0.15, n, r_loc)
    F = lattice_field(nx, ny, hx, hy, COV_EXP, 50.0, r_field)
    y = F[jj, ii] + np.sqrt(0.1) * r_field.standard_normal(P.shape[0])
    del F
    dom = (0.0, 0.0, W, H)
    info = {}
    if delta is None:
        delta, cores, cnt = part.find_delta(
            P, lambda d: part.recursive_cores(P, dom, n_cores, d, device=device), overlap, iters=20,
            device=device)
        info["memberships_all"] = cnt
    else:
        cores = part.recursive_cores(P, dom, n_cores, delta, device=device)
    pt = part.build_partition(P, cores, delta, val_frac, r_split, device=device)
    return Workload("large", P, y, pt, COV_EXP, (50.0, 0.1), dom, info)


def scaled(name, scale, seed_id=None):
    """A smaller copy of a workload's recipe (same structure, fewer points),
    used by tests that must finish quickly."""
    if name == "plain_fp64":
        return plain_fp64(n=max(40, int(2000 * scale)))
    if name == "batched":
        g = max(2, int(round(16 * np.sqrt(scale))))
        return batched(n=max(200, int(100_000 * scale)), grid=(g, g), lattice=256)
    if name == "uneven":
        g = max(2, int(round(32 * np.sqrt(scale))))
        return uneven(n=max(400, int(1_000_000 * scale)), grid=(g, g), lattice=256,
                      cap=max(100, int(4000 * np.sqrt(scale))))
    raise ValueError(name)
