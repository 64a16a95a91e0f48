"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

Tolerances (relative, on the SSPE of eq. (4) / eq. (7)), for the total and
for every subset's SSPE:
  FP64 path    1e-10  (the only differences are summation order and
                       centring of coordinates; both ~1e-14 here)
  mixed path   1e-6   (FP32 factor, FP64 refinement / prediction / sums)
Log determinants per subset within the first-order bound of
tests/parity_util.py (8 u n (1 + lambda) / lambda, u the factor's unit
roundoff).  Predictions from the resident FP64 factors: mean and variance
within 1e-9.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1912_13132_amd import partition as part
from paper_1912_13132_amd import pcv
from paper_1912_13132_amd import workloads as W
from parity_util import check_logdet, check_sspe

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
TOL_MIXED = 1e-6


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def _rng(k):
    return np.random.default_rng(np.random.SeedSequence([1912, 13132, 500 + k]))


def _oracle(w, th, subsets=None):
    pt = w.part
    return oracle.cv_loss(w.locs, w.y, pt.train_ptr, pt.train_idx, pt.val_ptr, pt.val_idx,
                          th.cov, th.range, th.lambda_, subsets=subsets)


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _check_full(w, th, prec, tol, max_refine=2):
    say(f"[case] {w.name} N={len(w.y)} S={w.part.n_subsets} prec={prec} "
        f"theta=({th.range},{th.lambda_},cov={th.cov})")
    ref = _oracle(w, th)
    with pcv.Problem.from_workload(w, prec=prec, max_refine=max_refine) as P:
        loss, rep = P.eval(th, report=True)
    assert rep["n_val"] == ref["n_val"]
    assert _rel(loss, ref["sspe"]) <= tol, (loss, ref["sspe"], _rel(loss, ref["sspe"]))
    say(f"   loss rel err {_rel(loss, ref['sspe']):.2e}  fallback {rep['n_fallback_fp64']}"
        f"  max rel residual {rep['max_rel_residual']:.2e}")
    check_sspe(rep["per_subset_sspe"], ref["per_subset_sspe"], prec, say)
    act = ref["per_subset_nval"] > 0
    n = np.diff(w.part.train_ptr)
    check_logdet(rep["per_subset_logdet"][act], ref["per_subset_logdet"][act], n[act], th.lambda_, prec, say)
    return loss, rep


# ------------------------------------------------------------ workloads ---
@pytest.fixture(scope="module")
def w_plain():
    return W.plain_fp64()


@pytest.fixture(scope="module")
def w_batched_small():
    return W.scaled("batched", 0.05)


@pytest.fixture(scope="module")
def w_uneven_small():
    return W.scaled("uneven", 0.01)


def test_plain_fp64_config_fp64_path(w_plain):
    _check_full(w_plain, pcv.theta(0.1, 0.05), "fp64", TOL_FP64)


def test_plain_fp64_config_mixed_path(w_plain):
    _check_full(w_plain, pcv.theta(0.1, 0.05), "mixed", TOL_MIXED)


@pytest.mark.parametrize("k", [0, 27, 63])
def test_batched_recipe_theta_grid(w_batched_small, k):
    g = W.theta_grid(w_batched_small.theta_true, 8)
    th = pcv.theta(*g[k])
    _check_full(w_batched_small, th, "fp64", TOL_FP64)
    _check_full(w_batched_small, th, "mixed", TOL_MIXED)


def test_uneven_recipe_matern(w_uneven_small):
    th = pcv.theta(0.03, 0.02, cov=pcv.COV_MATERN32)
    _check_full(w_uneven_small, th, "fp64", TOL_FP64)
    _check_full(w_uneven_small, th, "mixed", TOL_MIXED)


# ----------------------------------------------------------- edge cases ---
def _synthetic(sizes_T, sizes_V, seed, spread=1.0):
    """Independent subsets with the given training / validation sizes."""
    r = _rng(seed)
    locs, y, tl, vl = [], [], [], []
    off = 0
    for nt, nv in zip(sizes_T, sizes_V):
        P = r.uniform(0, spread, (nt + nv, 2))
        yy = r.standard_normal(nt + nv)
        locs.append(P)
        y.append(yy)
        tl.append(np.arange(off, off + nt))
        vl.append(np.arange(off + nt, off + nt + nv))
        off += nt + nv
    locs = np.concatenate(locs)
    y = np.concatenate(y)
    tp = np.r_[0, np.cumsum(sizes_T)]
    vp = np.r_[0, np.cumsum(sizes_V)]
    ti = np.concatenate(tl).astype(np.int32)
    vi = np.concatenate(vl).astype(np.int32)
    return locs, y, tp, ti, vp, vi


@pytest.mark.parametrize("prec,tol", [("fp64", TOL_FP64), ("mixed", TOL_MIXED)])
def test_ragged_sizes_and_degenerate_subsets(prec, tol):
    """Sizes around the 64-row tile and the 256-row chunk, n = 1, n = 0 with
    validation points (prior mean), and subsets without validation points
    (skipped)."""
    sizes_T = [1, 2, 63, 64, 65, 127, 128, 255, 256, 257, 300, 513, 0, 40, 77]
    sizes_V = [3, 5, 7, 1, 9, 11, 13, 2, 4, 6, 30, 50, 4, 0, 8]
    locs, y, tp, ti, vp, vi = _synthetic(sizes_T, sizes_V, 1)
    say(f"[case] ragged prec={prec} sizes={sizes_T}")
    th = pcv.theta(0.3, 0.1)
    ref = oracle.cv_loss(locs, y, tp, ti, vp, vi, 0, 0.3, 0.1)
    with pcv.Problem(locs, y, tp, ti, vp, vi, prec=prec) as P:
        loss, rep = P.eval(th, report=True)
    assert _rel(loss, ref["sspe"]) <= tol
    check_sspe(rep["per_subset_sspe"], ref["per_subset_sspe"], prec, say)
    act = ref["per_subset_nval"] > 0
    check_logdet(rep["per_subset_logdet"][act], ref["per_subset_logdet"][act], np.array(sizes_T)[act], 0.1,
                 prec, say)
    assert rep["per_subset_sspe"][13] == 0.0
    assert rep["n_val"] == ref["n_val"]


@pytest.mark.parametrize("prec,tol", [("fp64", TOL_FP64), ("mixed", TOL_MIXED)])
def test_ragged_sizes_up_to_512_points(prec, tol):
    """Every subset pads to at most 512 rows, so the FP32 factorisation takes
    its smallest shape (2-wave work-groups, 64-row chunks, the inverse tiles
    of the triangular solves in registers): sizes around the 64-row tile,
    n = 1, n = 0 with validation points and a skipped subset."""
    sizes_T = [1, 2, 63, 64, 65, 127, 128, 129, 200, 255, 256, 257, 400, 511, 512, 0, 37]
    sizes_V = [3, 5, 7, 1, 9, 11, 13, 2, 4, 6, 30, 50, 4, 8, 10, 4, 0]
    locs, y, tp, ti, vp, vi = _synthetic(sizes_T, sizes_V, 8)
    say(f"[case] ragged up to 512 prec={prec} sizes={sizes_T}")
    ref = oracle.cv_loss(locs, y, tp, ti, vp, vi, 0, 0.3, 0.1)
    with pcv.Problem(locs, y, tp, ti, vp, vi, prec=prec) as P:
        loss, rep = P.eval(pcv.theta(0.3, 0.1), report=True)
    assert _rel(loss, ref["sspe"]) <= tol
    check_sspe(rep["per_subset_sspe"], ref["per_subset_sspe"], prec, say)
    act = ref["per_subset_nval"] > 0
    check_logdet(rep["per_subset_logdet"][act], ref["per_subset_logdet"][act], np.array(sizes_T)[act], 0.1,
                 prec, say)
    assert rep["per_subset_sspe"][16] == 0.0


@pytest.mark.parametrize("prec,tol", [("fp64", TOL_FP64), ("mixed", TOL_MIXED)])
def test_subsets_above_4096_points(prec, tol):
    """Subsets of 5,000 and 4,097 training points take the solve variants
    for more than 4,096 padded rows; a small subset rides along."""
    sizes_T = [5000, 4097, 300]
    sizes_V = [120, 40, 20]
    locs, y, tp, ti, vp, vi = _synthetic(sizes_T, sizes_V, 5, spread=3.0)
    say(f"[case] large subsets prec={prec} sizes={sizes_T}")
    ref = oracle.cv_loss(locs, y, tp, ti, vp, vi, 0, 0.4, 0.1)
    with pcv.Problem(locs, y, tp, ti, vp, vi, prec=prec) as P:
        loss, rep = P.eval(pcv.theta(0.4, 0.1), report=True)
    assert _rel(loss, ref["sspe"]) <= tol
    check_sspe(rep["per_subset_sspe"], ref["per_subset_sspe"], prec, say)
    check_logdet(rep["per_subset_logdet"], ref["per_subset_logdet"], np.array(sizes_T), 0.1, prec, say)


@pytest.mark.parametrize("prec,tol", [("fp64", TOL_FP64), ("mixed", TOL_MIXED)])
def test_subset_above_8192_points(prec, tol):
    """A subset of 9,000 training points: the solve variants for more than
    8,192 padded rows (32 row slots per thread)."""
    sizes_T = [9000, 200]
    sizes_V = [90, 10]
    locs, y, tp, ti, vp, vi = _synthetic(sizes_T, sizes_V, 6, spread=4.0)
    say(f"[case] subset above 8192 prec={prec} sizes={sizes_T}")
    ref = oracle.cv_loss(locs, y, tp, ti, vp, vi, 0, 0.4, 0.1)
    with pcv.Problem(locs, y, tp, ti, vp, vi, prec=prec) as P:
        loss, rep = P.eval(pcv.theta(0.4, 0.1), report=True)
    assert _rel(loss, ref["sspe"]) <= tol
    check_sspe(rep["per_subset_sspe"], ref["per_subset_sspe"], prec, say)
    check_logdet(rep["per_subset_logdet"], ref["per_subset_logdet"], np.array(sizes_T), 0.1, prec, say)


def test_no_nugget_fp64():
    """lambda = 0 is allowed (tau >= 0 in eq. (1)); distinct points keep M SPD."""
    locs, y, tp, ti, vp, vi = _synthetic([120, 90], [10, 10], 2)
    say("[case] lambda=0 fp64")
    ref = oracle.cv_loss(locs, y, tp, ti, vp, vi, 0, 0.05, 0.0)
    with pcv.Problem(locs, y, tp, ti, vp, vi, prec="fp64") as P:
        loss = P.eval(pcv.theta(0.05, 0.0))
    assert _rel(loss, ref["sspe"]) <= 1e-8


def test_not_positive_definite_is_reported():
    """Duplicate training locations with lambda = 0 make M singular: the FP64
    path reports PCV_ERR_NOT_PD naming the subset."""
    locs = np.array([[0.1, 0.1], [0.1, 0.1], [0.5, 0.5], [0.2, 0.3]])
    y = np.array([1.0, 1.0, 0.5, 0.2])
    say("[case] not PD")
    with pcv.Problem(locs, y, [0, 3], [0, 1, 2], [0, 1], [3], prec="fp64") as P:
        with pytest.raises(pcv.PcvError) as e:
            P.eval(pcv.theta(0.2, 0.0))
        assert e.value.status == 3
        # the same problem with a nugget is fine
        ref = oracle.cv_loss(locs, y, [0, 3], [0, 1, 2], [0, 1], [3], 0, 0.2, 0.1)
        assert _rel(P.eval(pcv.theta(0.2, 0.1)), ref["sspe"]) <= TOL_FP64


def test_mixed_fallback_path(w_plain):
    """The FP64 re-run that replaces a broken-down FP32 factorisation,
    forced for every subset from the host: identical to the FP64 path."""
    th = pcv.theta(0.1, 0.05)
    say("[case] forced mixed -> fp64 fallback")
    with pcv.Problem.from_workload(w_plain, prec="mixed", debug_flags=1) as P:
        loss, rep = P.eval(th, report=True)
    with pcv.Problem.from_workload(w_plain, prec="fp64") as P:
        ref = P.eval(th)
    assert rep["n_fallback_fp64"] == rep["n_subsets_used"] == w_plain.part.n_subsets
    assert loss == ref


def test_refinement_convergence_test_falls_back(w_plain):
    """refine_tol = 0 fails the per-subset convergence test everywhere, so
    every subset is re-run in FP64: identical to the FP64 path.  With the
    default threshold no subset of this well-conditioned problem falls back."""
    th = pcv.theta(0.1, 0.05)
    say("[case] refinement convergence test -> fp64 fallback")
    with pcv.Problem.from_workload(w_plain, prec="mixed", refine_tol=0.0) as P:
        loss, rep = P.eval(th, report=True)
    with pcv.Problem.from_workload(w_plain, prec="fp64") as P:
        ref = P.eval(th)
    assert rep["n_fallback_fp64"] == rep["n_subsets_used"] == w_plain.part.n_subsets
    assert loss == ref
    with pcv.Problem.from_workload(w_plain, prec="mixed") as P:
        loss, rep = P.eval(th, report=True)
    assert rep["n_fallback_fp64"] == 0
    assert 0.0 < rep["max_rel_residual"] <= 1e-4


@pytest.mark.parametrize("graph", [True, False])
def test_second_sweep_only_where_residual_above_tol(w_batched_small, graph):
    """A second refinement sweep runs only for the subsets whose first-sweep
    residual exceeds refine_tol.  With refine_tol just below the largest
    first-sweep residual the subset that has it takes two sweeps and the
    others (residuals of distinct subsets differ) one; none
    falls back (the second sweep's residual is far below the threshold), the
    one-sweep subsets keep the one-sweep result bit for bit, every subset's
    SSPE is within the mixed tolerance of the oracle, and pcv_eval_batch
    gates the same way (bit-identical losses)."""
    w = w_batched_small
    th = pcv.theta(*w.theta_true)
    say(f"[case] gated second sweep graph={graph}")
    ref = _oracle(w, th)
    with pcv.Problem.from_workload(w, prec="mixed", max_refine=1, refine_tol=1.0, graph=graph) as P:
        l1, r1 = P.eval(th, report=True)
    m1 = r1["max_rel_residual"]
    assert 0.0 < m1 <= 1e-4 and r1["n_fallback_fp64"] == 0
    act = ref["per_subset_nval"] > 0
    assert np.all(r1["per_subset_iters"][act] == 1)
    with pcv.Problem.from_workload(w, prec="mixed", max_refine=2, refine_tol=m1 * (1 - 1e-9), graph=graph) as P:
        l2, r2 = P.eval(th, report=True)
        g = W.theta_grid(w.theta_true, 2)
        ths = [th] + [pcv.theta(*t) for t in g]
        single = [P.eval(t) for t in ths]
        batch = P.eval_batch(ths)
    it = r2["per_subset_iters"]
    say(f"   max first-sweep residual {m1:.2e}: {int((it[act] == 2).sum())} of {int(act.sum())} subsets "
        f"took a second sweep; max residual corrected last {r2['max_rel_residual']:.2e}")
    assert r2["n_fallback_fp64"] == 0 and r2["max_refine_iters"] == 2
    assert set(np.unique(it[act])) == {1, 2}
    assert np.all(it[~act] == 0)
    one = act & (it == 1)
    np.testing.assert_array_equal(r2["per_subset_sspe"][one], r1["per_subset_sspe"][one])
    assert _rel(l2, ref["sspe"]) <= TOL_MIXED
    check_sspe(r2["per_subset_sspe"], ref["per_subset_sspe"], "mixed", say)
    assert single[0] == l2
    np.testing.assert_array_equal(batch, single)


def test_partial_fallback_matches_fp64_per_subset(w_batched_small):
    """Subsets re-run in FP64 get their factors in a buffer sized for them
    alone.  With refine_tol just below the largest first-sweep residual at
    theta and one sweep, exactly that subset is re-run: its SSPE equals the
    FP64 path's bit for bit, every other subset keeps its mixed result bit
    for bit.  At a quarter of the nugget more subsets exceed the same
    threshold on the same problem (the buffer grows; each re-run subset
    equals the FP64 path's), and theta again gives the same bits."""
    w = w_batched_small
    th = pcv.theta(*w.theta_true)
    th2 = pcv.theta(w.theta_true[0], w.theta_true[1] / 4)
    say("[case] partial FP64 fallback")
    with pcv.Problem.from_workload(w, prec="fp64") as P:
        l64, r64 = P.eval(th, report=True)
        l64b, r64b = P.eval(th2, report=True)
    with pcv.Problem.from_workload(w, prec="mixed", max_refine=1, refine_tol=1.0) as P:
        l1, r1 = P.eval(th, report=True)
    m1 = r1["max_rel_residual"]
    with pcv.Problem.from_workload(w, prec="mixed", max_refine=1, refine_tol=m1 * (1 - 1e-9)) as P:
        la, ra = P.eval(th, report=True)
        lb, rb = P.eval(th2, report=True)
        lc, rc = P.eval(th, report=True)
    act = r64["per_subset_sspe"] > 0
    fa = act & (ra["per_subset_iters"] == 0)
    assert ra["n_fallback_fp64"] == 1 and fa.sum() == 1
    np.testing.assert_array_equal(ra["per_subset_sspe"][fa], r64["per_subset_sspe"][fa])
    np.testing.assert_array_equal(ra["per_subset_sspe"][~fa], r1["per_subset_sspe"][~fa])
    fb = act & (rb["per_subset_iters"] == 0)
    say(f"   re-run subsets: {int(fa.sum())} at theta, {int(fb.sum())} at a quarter of the nugget")
    assert rb["n_fallback_fp64"] == fb.sum() > 1
    np.testing.assert_array_equal(rb["per_subset_sspe"][fb], r64b["per_subset_sspe"][fb])
    assert abs(lb - l64b) <= TOL_MIXED * l64b
    assert lc == la
    np.testing.assert_array_equal(rc["per_subset_sspe"], ra["per_subset_sspe"])


@pytest.mark.parametrize("max_refine", [0, 1, 2])
def test_error_estimate_tracks_fp64(w_batched_small, max_refine):
    """est_rel_err, the loss change one more refinement sweep makes, against
    the measured relative difference from the FP64 path.  With no sweep the
    FP32 solve's error dominates and the two agree within 25% (the
    refinement contracts the error by far more); with sweeps both are tiny
    and the estimate stays within a factor 3 of the measured difference or
    below 1e-13 (the FP64 path's own rounding).  The estimate leaves the
    result bit for bit as it is, reads -1 when not asked for and 0 for an
    FP64 problem."""
    w = w_batched_small
    th = pcv.theta(w.theta_true[0], w.theta_true[1] / 2)
    say(f"[case] error estimate max_refine={max_refine}")
    with pcv.Problem.from_workload(w, prec="fp64", est_error=True) as P:
        l64, r64 = P.eval(th, report=True)
    assert r64["est_rel_err"] == 0.0
    with pcv.Problem.from_workload(w, prec="mixed", max_refine=max_refine) as P:
        l0, r0 = P.eval(th, report=True)
    assert r0["est_rel_err"] == -1.0
    with pcv.Problem.from_workload(w, prec="mixed", max_refine=max_refine, est_error=True) as P:
        l1, r1 = P.eval(th, report=True)
        l2 = P.eval(th, report=True)[0]
    assert l1 == l0 == l2
    np.testing.assert_array_equal(r1["per_subset_sspe"], r0["per_subset_sspe"])
    est, act = r1["est_rel_err"], _rel(l1, l64)
    say(f"   estimated {est:.3e}  measured against the FP64 path {act:.3e}")
    assert est >= 0.0
    if max_refine == 0:
        assert act > 1e-9 and 0.8 * act <= est <= 1.25 * act
    else:
        assert est <= max(3 * act, 1e-13) and act <= max(3 * est, 1e-13)


@pytest.mark.parametrize("lam", [1e-3, 3e-4])
def test_small_nugget_second_sweep_avoids_fallback(w_plain, lam):
    """Small nugget: the FP32 factor is poorly conditioned, so a subset's
    first-sweep residual can exceed refine_tol.  The default two sweeps
    re-run in FP64 no more subsets than one sweep does, and the loss stays
    within the mixed tolerance of the oracle."""
    th = pcv.theta(0.3, lam)
    say(f"[case] small nugget lambda={lam}")
    ref = _oracle(w_plain, th)
    out = {}
    for mr in (1, 2):
        with pcv.Problem.from_workload(w_plain, prec="mixed", max_refine=mr) as P:
            loss, rep = P.eval(th, report=True)
        out[mr] = rep["n_fallback_fp64"]
        say(f"   max_refine={mr}: fallback {rep['n_fallback_fp64']} max rel residual "
            f"{rep['max_rel_residual']:.2e} loss rel err {_rel(loss, ref['sspe']):.2e}")
        assert _rel(loss, ref["sspe"]) <= TOL_MIXED
        check_sspe(rep["per_subset_sspe"], ref["per_subset_sspe"], "mixed", say)
    assert out[2] <= out[1]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_graph_replays_match_eager(w_batched_small, prec):
    """The captured evaluation, replayed for several theta with eager
    evaluations and host synchronisations in between, gives every replay
    bit for bit the eager result (loss, per-subset SSPE and log det)."""
    g = W.theta_grid(w_batched_small.theta_true, 3)
    ths = [pcv.theta(*t) for t in g] + [pcv.theta(*g[0])]
    say(f"[case] graph replays prec={prec}")
    with pcv.Problem.from_workload(w_batched_small, prec=prec, graph=True, profile=True) as Pg, \
            pcv.Problem.from_workload(w_batched_small, prec=prec, graph=False) as Pe:
        for th in ths:
            a, ra = Pg.eval(th, report=True)
            b, rb = Pe.eval(th, report=True)
            assert a == b
            np.testing.assert_array_equal(ra["per_subset_sspe"], rb["per_subset_sspe"])
            np.testing.assert_array_equal(ra["per_subset_logdet"], rb["per_subset_logdet"])
            assert ra["ms_factor"] > 0.0


def test_graph_with_fallback_matches_fp64(w_plain):
    th = pcv.theta(0.1, 0.05)
    say("[case] graph + forced fallback")
    with pcv.Problem.from_workload(w_plain, prec="mixed", debug_flags=1, graph=True) as P:
        a = [P.eval(th) for _ in range(3)]
    with pcv.Problem.from_workload(w_plain, prec="fp64", graph=False) as P:
        ref = P.eval(th)
    assert a == [ref] * 3


def test_repeatable_bitwise(w_batched_small):
    """Two evaluations of the same theta are bitwise equal (fixed-order sums)."""
    th = pcv.theta(0.05, 0.1)
    with pcv.Problem.from_workload(w_batched_small, prec="mixed") as P:
        a = P.eval(th)
        P.eval(pcv.theta(0.03, 0.2))
        b = P.eval(th)
    assert a == b


@pytest.mark.parametrize("prec,graph", [("mixed", True), ("mixed", False), ("fp64", True)])
def test_eval_batch_matches_single(w_batched_small, prec, graph):
    """Several theta in one launch per kernel (descriptors replicated per
    theta slot): every loss equals the single evaluation bit for bit.  70
    values = a group of 64 slots and a remainder group of 6."""
    r = _rng(30)
    t0, l0 = w_batched_small.theta_true
    ths = [pcv.theta(t0 * 2 ** r.uniform(-1, 1), l0 * 2 ** r.uniform(-1, 1)) for _ in range(70)]
    say(f"[case] eval_batch prec={prec} graph={graph} K=70")
    with pcv.Problem.from_workload(w_batched_small, prec=prec, graph=graph) as P:
        batch = P.eval_batch(ths)
        single = [P.eval(t) for t in ths]
        again = P.eval_batch(ths[:9])
    np.testing.assert_array_equal(batch, single)
    np.testing.assert_array_equal(again, single[:9])


def test_eval_batch_with_forced_fallback(w_plain):
    ths = [pcv.theta(*t) for t in W.theta_grid(w_plain.theta_true, 2)]
    say("[case] eval_batch forced fallback")
    with pcv.Problem.from_workload(w_plain, prec="mixed", debug_flags=1) as P:
        batch = P.eval_batch(ths)
    with pcv.Problem.from_workload(w_plain, prec="fp64") as P:
        ref = [P.eval(t) for t in ths]
    np.testing.assert_array_equal(batch, ref)


# ------------------------------------------------------------ prediction --
def test_predict_matches_oracle(w_plain):
    th = pcv.theta(0.1, 0.05, sigma2=1.3)
    r = _rng(4)
    q = np.concatenate([r.uniform(0, 1, (300, 2)), [[0.5, 0.5], [1.0, 1.0], [0.0, 0.0], [1.2, -0.1]]])
    pt = w_plain.part
    say("[case] predict plain_fp64")
    with pcv.Problem.from_workload(w_plain, prec="mixed") as P:
        with pytest.raises(pcv.PcvError) as e:
            P.predict(q)
        assert e.value.status == 5
        P.factor(th)
        P.eval(pcv.theta(0.2, 0.3))  # evaluations must not disturb the factors
        mean, var, owner = P.predict(q)
        m2, v2, _ = P.predict(q, obs_noise=True)
    rm, rv, ro = oracle.predict_problem(w_plain.locs, w_plain.y, pt.train_ptr, pt.train_idx,
                                        pt.core_rect, q, 0, 0.1, 0.05, sigma2=1.3)
    np.testing.assert_array_equal(owner, ro)
    np.testing.assert_allclose(mean, rm, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(var, rv, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(v2, rv + 1.3 * 0.05, rtol=1e-9, atol=1e-11)
    np.testing.assert_array_equal(m2, mean)


def test_predict_interpolates_without_nugget():
    """lambda = 0: predicting at training locations returns the data with
    zero variance (oracle pin carried to the device path)."""
    r = _rng(5)
    locs = r.uniform(0, 1, (150, 2))
    y = r.standard_normal(150)
    with pcv.Problem(locs, y, [0, 150], np.arange(150), [0, 0], [], prec="fp64",
                     core_rect=[[0, 0, 1, 1]]) as P:
        P.factor(pcv.theta(0.1, 0.0))
        mean, var, _ = P.predict(locs[::5])
    np.testing.assert_allclose(mean, y[::5], atol=1e-8)
    np.testing.assert_allclose(var, 0.0, atol=1e-8)


@pytest.mark.parametrize("prec,tol", [("fp64", TOL_FP64), ("mixed", TOL_MIXED)])
def test_two_stream_schedule(prec, tol):
    """More evaluated subsets than compute units and not a whole number of
    rounds (300 on 256): the remainder's factorisation and solves run on a
    second stream beside the first group's.  The loss and per-subset values
    carry the same bits as the single-stream phase-by-phase schedule, in
    graph replays and eager launches, and match the oracle."""
    r = _rng(41)
    sizes_T = list(r.integers(30, 200, size=300))
    sizes_V = list(r.integers(1, 12, size=300))
    sizes_V[7] = 0  # a skipped subset among them
    locs, y, tp, ti, vp, vi = _synthetic(sizes_T, sizes_V, 42)
    say(f"[case] two-stream schedule prec={prec} S=300")
    th = pcv.theta(0.3, 0.1)
    ref = oracle.cv_loss(locs, y, tp, ti, vp, vi, 0, 0.3, 0.1)
    out = {}
    for name, kw in (("graph", {}), ("eager", {"graph": False}), ("phases", {"profile": True})):
        with pcv.Problem(locs, y, tp, ti, vp, vi, prec=prec, **kw) as P:
            vals = [P.eval(th, report=True) for _ in range(3)]
        for loss, rep in vals[1:]:
            assert loss == vals[0][0]
            np.testing.assert_array_equal(rep["per_subset_sspe"], vals[0][1]["per_subset_sspe"])
        out[name] = vals[0]
    for name in ("eager", "phases"):
        assert out[name][0] == out["graph"][0], name
        np.testing.assert_array_equal(out[name][1]["per_subset_sspe"], out["graph"][1]["per_subset_sspe"])
        np.testing.assert_array_equal(out[name][1]["per_subset_logdet"], out["graph"][1]["per_subset_logdet"])
    assert _rel(out["graph"][0], ref["sspe"]) <= tol


# ----------------------------------------------------------- memory cap ---
def test_memory_cap_refuses_and_bounds_the_batch_workspace(w_plain):
    """mem_cap_bytes below what the problem needs: creation fails with
    PCV_ERR_OOM (and a later problem on the device works).  A cap that holds
    the problem and its factor but not the multi-theta workspace: the
    batched call evaluates theta by theta, bit for bit the same losses; a
    cap that also holds a small workspace gives the same bits."""
    th = pcv.theta(0.1, 0.05)
    ths = [pcv.theta(*t) for t in W.theta_grid(w_plain.theta_true, 3)]
    say("[case] memory cap")
    with pcv.Problem.from_workload(w_plain, prec="mixed") as P:
        l_ref = P.eval(th)
        need = P.info()["device_bytes"]
        b_ref = P.eval_batch(ths)
        need_batch = P.info()["device_bytes"]
    assert need_batch > need
    with pytest.raises(pcv.PcvError) as e:
        pcv.Problem.from_workload(w_plain, prec="mixed", mem_cap=need // 4)
    assert e.value.status == 2
    with pcv.Problem.from_workload(w_plain, prec="mixed", mem_cap=need + (1 << 20)) as P:
        assert P.eval(th) == l_ref
        np.testing.assert_array_equal(P.eval_batch(ths), b_ref)
        assert P.info()["device_bytes"] <= need + (1 << 20)
    slot = (need_batch - need) // len(ths)
    with pcv.Problem.from_workload(w_plain, prec="mixed", mem_cap=need + 3 * slot + (1 << 20)) as P:
        assert P.eval(th) == l_ref
        np.testing.assert_array_equal(P.eval_batch(ths), b_ref)
