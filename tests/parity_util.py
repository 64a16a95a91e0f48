"""Per-subset parity bounds shared by the GPU tests.

Loss (eq. (4) per subset, eq. (7) summed): relative 1e-10 on the FP64 path
and 1e-6 on the mixed path, for the total and for every subset's SSPE.

Log determinant of M_i = Sigma_i + lambda I (the likelihood of eq. (2)).  A
computed factor satisfies L L^T = M + E, and to first order
    logdet(M + E) - logdet(M) = tr(M^{-1} E),
so |delta| <= ||M^{-1}||_2 ||E||_* <= ||E||_* / lambda, since Sigma_i is
positive semi-definite and the smallest eigenvalue of M is at least lambda.
The nuclear norm of the backward error of a Cholesky factorisation carried
out in unit roundoff u, of an n x n matrix with diagonal 1 + lambda (plus the
rounding of the covariance entries themselves), is modelled as
c u n (1 + lambda).  With c = 1 this matched the largest error of an FP32
LAPACK factorisation on the CPU over n = 200..2,000, lambda = 0.02..0.1 and
ranges 0.05..0.3 (ratios 0.002..1.0); the bound takes c = 8.  The mixed
path factors in FP32 (u = 2^-24) with FP64 diagonal blocks, the FP64 path
in u = 2^-53.
"""
import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53
TOL_SSPE = {"fp64": 1e-10, "mixed": 1e-6}
LOGDET_C = 8.0


def logdet_bound(prec, n, lam):
    """Absolute bound on the log det difference of one subset (n training
    points, nugget lam > 0)."""
    u = U32 if prec == "mixed" else U64
    n = np.asarray(n, dtype=np.float64)
    return LOGDET_C * u * n * (1.0 + lam) / lam


def check_sspe(got, ref, prec, say=None, what="per-subset SSPE"):
    """Every subset's SSPE within the loss tolerance (relative); subsets
    whose reference SSPE is below 1e-12 of the largest (or zero) must be
    below 1e-10 absolute."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    tol = TOL_SSPE[prec]
    big = ref > 1e-12 * max(float(ref.max(initial=0.0)), 1.0)
    rel = np.abs(got[big] - ref[big]) / ref[big]
    worst = float(rel.max()) if rel.size else 0.0
    if say:
        say(f"   {what}: max rel err {worst:.2e} (bound {tol:g})")
    assert worst <= tol, (what, worst, tol, np.nonzero(big)[0][np.argmax(rel)])
    assert np.all(np.abs(got[~big]) <= 1e-10), what
    return worst


def check_logdet(got, ref, n, lam, prec, say=None):
    """Every evaluated subset's log det within logdet_bound."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    b = logdet_bound(prec, n, lam)
    d = np.abs(got - ref)
    pos = b > 0
    assert np.all(d[~pos] == 0.0), "log det of an empty subset"
    ratio = float((d[pos] / b[pos]).max()) if pos.any() else 0.0
    if say:
        say(f"   log det: max |diff| {float(d.max(initial=0.0)):.2e}, max diff / bound {ratio:.3f}")
    assert ratio <= 1.0, ("log det", ratio)
    return ratio


def mixed_size_subsets(seed, S=300):
    """S independent subsets: three large ones (shared in the first launch),
    a band around the 4-wave / 8-wave shape threshold, many small ones;
    more subsets than compute units, so two schedule groups apply."""
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 1400 + seed]))
    sizes_T = [3000, 2500, 2100] + list(r.integers(1200, 1700, size=40)) + list(r.integers(60, 400, size=S - 43))
    sizes_V = [60, 50, 40] + list(r.integers(5, 30, size=40)) + list(r.integers(1, 10, size=S - 43))
    locs, y, tl, vl = [], [], [], []
    off = 0
    for nt, nv in zip(sizes_T, sizes_V):
        spread = 3.0 * np.sqrt(nt / 2000.0)
        locs.append(r.uniform(0, spread, (nt + nv, 2)))
        y.append(r.standard_normal(nt + nv))
        tl.append(np.arange(off, off + nt))
        vl.append(np.arange(off + nt, off + nt + nv))
        off += nt + nv
    return (np.concatenate(locs), np.concatenate(y), np.r_[0, np.cumsum(sizes_T)],
            np.concatenate(tl).astype(np.int32), np.r_[0, np.cumsum(sizes_V)],
            np.concatenate(vl).astype(np.int32))
