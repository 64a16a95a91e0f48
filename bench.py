"""Seconds per theta-evaluation of the parallel CV loss on one MI355X.

Workload: 5,000,000 points on a jittered 2,170 x 2,712 lattice over
[0,2000] x [0,2500] with 15% of the nodes removed in random rectangular gaps,
an exponential-covariance field (range 50, nugget 0.1), the recursive
division of Sec. 2.4 into 2,400 cores with 20% overlap (shells) and 10% of
every core held out.  One step = one full theta-evaluation (covariance,
Cholesky, solves + refinement, kriging of the validation points, loss
reduction), inputs resident in HBM.  The timed steps are graph replays of
the evaluation with the library's default launch shapes and schedule
(--tune picks them with pcv_autotune first, outside the timed region).

Prints one JSON line.  Besides the timed mixed-precision path it reports the
plain FP64 GPU path, the relative difference between the two losses, the
factorisation kernel's fraction of the FP32 MFMA peak (HIP events on the
library's stream), and the FP64 oracle timed on the host's cores on a
bounded sample of subsets, extrapolated by n^3 share.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "s per θ-eval @5M pts, CV loss ≤1e-6 rel vs FP64; kriging p99 latency"
PEAK_FP32_MFMA = 157.3   # TFLOP/s, MI355X dense FP32 matrix
PEAK_FP64_MFMA = 78.6    # TFLOP/s, MI355X dense FP64 matrix


def measured_traffic(kernel_src, prec, launch_subsets):
    """HBM bytes per launch of the factorisation kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when the kernel's
    source has changed since the counters were taken or the summary covers
    launches of another size."""
    path = os.path.join(ROOT, "profiles", "k_potrf_large_5M_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
        with open(kernel_src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    entry = t.get(prec)
    if not entry or t.get("source_sha256") != sha or t.get("launch_subsets") != launch_subsets:
        return None
    return entry["fetch_bytes"] + entry["write_bytes"]


def copy_probe(torch, mib):
    """A plain device copy of known size (y = 1.0 * x, fp32), for calibrating
    HBM byte counters; returns the measured copy bandwidth in GB/s."""
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    torch.mul(x, 1.0, out=y)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * n * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    return gbs


def serve(pcv, w, seconds, rate=200.0, n_opt=4, n_lhs=30, seed=11, with_evals=True, log=print, warmup=0.0,
          window=None):
    """Kriging service on the factored problem: Poisson arrivals at `rate`
    requests/s for `seconds`, each with floor(10^U(0,4)) query locations
    uniform over the domain (gaps included), plus `n_opt` closed-loop
    optimisers each walking its own Latin-hypercube design of `n_lhs` points
    over [theta/2, 2 theta] x [lambda/2, 2 lambda] through the same server.
    With warmup > 0 the same traffic first runs for `warmup` seconds on a
    server that is then discarded (its latencies are not reported)."""
    th0, lam0 = w.theta_true
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 5, seed]))
    P = pcv.Problem.from_workload(w, prec="mixed")
    P.factor(pcv.theta(th0, lam0, cov=w.cov))
    if warmup > 0:
        out = _serve_run(pcv, w, P, warmup, rate, n_opt, n_lhs, r, with_evals, seed, window)
        log(f"[serve] warm-up ({warmup} s) done: p50 {out['p50_ms']:.1f} ms")
    out = _serve_run(pcv, w, P, seconds, rate, n_opt, n_lhs, r, with_evals, seed, window)
    P.close()
    log(f"[serve] {'with' if with_evals else 'without'} evaluations: {out}")
    return out


def _serve_run(pcv, w, P, seconds, rate, n_opt, n_lhs, r, with_evals, seed, window=None):
    import threading
    import queue
    th0, lam0 = w.theta_true
    lo, hi = w.locs.min(0), w.locs.max(0)
    srv = pcv.Server(P, max_inflight=256, window=window)
    stop = threading.Event()
    evals = []

    def optimiser(k):
        # walks its seeded Latin-hypercube design, again from the start when
        # it is done, until the arrivals stop
        rr = np.random.default_rng(np.random.SeedSequence([1912, 13132, 5, seed, 100 + k]))
        u = (rr.permuted(np.tile(np.arange(n_lhs), (2, 1)), axis=1).T + rr.uniform(size=(n_lhs, 2))) / n_lhs
        while True:
            for a, b in u:
                if stop.is_set():
                    return
                t = pcv.theta(th0 * 4.0 ** (a - 0.5), lam0 * 4.0 ** (b - 0.5), cov=w.cov)
                evals.append(srv.wait(srv.submit_eval(t)))

    tickets = queue.Queue()

    def collector():
        while True:
            t = tickets.get()
            if t is None:
                return
            srv.wait(t)

    col = threading.Thread(target=collector)
    col.start()
    opts = [threading.Thread(target=optimiser, args=(k,)) for k in range(n_opt if with_evals else 0)]
    for t in opts:
        t.start()
    t0 = time.perf_counter()
    t_next = t0
    n_req = 0
    while True:
        t_next += r.exponential(1.0 / rate)
        if t_next - t0 > seconds:
            break
        nq = int(np.floor(10 ** r.uniform(0, 4)))
        q = r.uniform(lo, hi, (nq, 2))
        d = t_next - time.perf_counter()
        if d > 0:
            time.sleep(d)
        tickets.put(srv.submit_predict(q, want_var=True))
        n_req += 1
    stop.set()
    tickets.put(None)
    col.join()
    for t in opts:
        t.join()
    rep = srv.report()
    srv.close()
    return {"requests": rep["n_predict"], "queries": rep["n_queries"],
           "p50_ms": 1e3 * rep["p50_s"], "p99_ms": 1e3 * rep["p99_s"], "max_ms": 1e3 * rep["max_s"],
           "qps": rep["qps"], "evals": rep["n_eval"], "evals_per_s": rep["evals_per_s"],
           "eval_p50_ms": 1e3 * rep["eval_p50_s"], "eval_p99_ms": 1e3 * rep["eval_p99_s"],
           "batches": rep["n_batches"], "mean_batch_queries": rep["mean_batch_queries"],
           "admission_waits": rep["admission_waits"], "workspace_bytes": rep["workspace_bytes"],
           "seconds": seconds, "rate_req_per_s": rate, "optimisers": len(opts)}


def _oracle_subset(args):
    """CPU-baseline worker: one subset through the FP64 oracle, one BLAS thread."""
    from threadpoolctl import threadpool_limits
    import oracle
    locT, yT, locV, yV, kind, rng_, lam = args
    with threadpool_limits(1):
        t0 = time.perf_counter()
        r = oracle.subset_cv(locT, yT, locV, yV, kind, rng_, lam)
        return time.perf_counter() - t0, r["sspe"]


def cpu_baseline(w, th, gpu_per_subset, sample=144, seed=7, workload="large"):
    import multiprocessing as mp
    pt = w.part
    n = np.diff(pt.train_ptr)
    m = np.diff(pt.val_ptr)
    act = np.nonzero(m > 0)[0]
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 4, seed]))
    pick = np.sort(r.choice(act, size=min(sample, act.size), replace=False))
    jobs = []
    for i in pick:
        T = pt.train_idx[pt.train_ptr[i]:pt.train_ptr[i + 1]]
        V = pt.val_idx[pt.val_ptr[i]:pt.val_ptr[i + 1]]
        jobs.append((w.locs[T], w.y[T], w.locs[V], w.y[V], w.cov, th[0], th[1]))
    # one worker per host core this process may use, at most 16: the host
    # cores a one-GPU machine grants its GPU's jobs
    cores = max(1, min(16, len(os.sched_getaffinity(0)), os.cpu_count() or 1))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_subset, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    cpu_s = np.array([x[0] for x in res])
    z = np.array([x[1] for x in res])
    n3 = n.astype(np.float64) ** 3
    share = n3[act].sum() / n3[pick].sum()
    est_single = cpu_s.sum() * share
    rel = np.abs(gpu_per_subset[pick] - z) / np.maximum(z, 1e-300)
    return dict(value=est_single / cores, unit="s", cores=cores, kind="oracle",
                sample=f"{workload}: {len(pick)} of {act.size} subsets (seeded), {cpu_s.sum():.1f} CPU-s, "
                       f"extrapolated by n^3 share to all subsets on {cores} cores (one worker process per "
                       f"core, one BLAS thread each; the box grants 16 host cores per GPU, "
                       f"os.cpu_count() = {os.cpu_count()})",
                single_core_s=est_single, sample_wall_s=wall), float(rel.max())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--max-refine", type=int, default=2)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparator")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--workload", default="large", choices=["large", "plain", "batched", "uneven"])
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the 5M workload (testing)")
    ap.add_argument("--serve-warmup", type=float, default=5.0,
                    help="seconds of the same traffic on a discarded server before the serving run with "
                         "optimisers (the kriging-only run warms up for at most 2 s)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the serving run with optimisers (0 = skip serving); the kriging-only "
                         "run lasts at most 15 s")
    ap.add_argument("--serve-window", type=float, default=None,
                    help="kriging batching window while evaluations are active (s; library default 0.03)")
    ap.add_argument("--tune", action="store_true",
                    help="pick the launch shapes and schedule with pcv_autotune first (off by default: "
                         "the tuner is not yet cleared for GPU runs)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (HBM counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(subsets would shard across GPUs with one broadcast and one scalar reduce)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1912_13132_amd import pcv
    from paper_1912_13132_amd import workloads as W

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream(0)

    t0 = time.perf_counter()
    if a.workload == "large":
        if a.scale >= 1.0:
            w = W.large(device=True)
        else:
            s = a.scale
            w = W.large(n=int(5_000_000 * s), nx=int(2170 * math.sqrt(s)) + 1,
                        ny=int(2712 * math.sqrt(s)) + 1, W=2000 * math.sqrt(s), H=2500 * math.sqrt(s),
                        n_cores=max(2, int(2400 * s)))
    else:
        w = {"plain": W.plain_fp64, "batched": W.batched, "uneven": W.uneven}[a.workload](device=True)
    pt = w.part
    nT = np.diff(pt.train_ptr)
    mV = np.diff(pt.val_ptr)
    act = mV > 0
    log(f"workload generated in {time.perf_counter() - t0:.1f}s: N={len(w.y)} S={pt.n_subsets} "
        f"train {nT.min()}..{nT.max()} val {mV.min()}..{mV.max()}")
    copy_gbs = copy_probe(torch, a.copy_probe_mib) if a.copy_probe_mib > 0 else None
    th_true = w.theta_true
    # the theta values of one step: the 8 x 8 grid for the batched workload,
    # the generating value otherwise
    if a.workload == "batched":
        thetas = [pcv.theta(r_, l_, cov=w.cov) for r_, l_ in W.theta_grid(th_true, 8)]
    else:
        thetas = [pcv.theta(th_true[0], th_true[1], cov=w.cov)]
    n3 = nT[act].astype(np.float64)
    flops_potrf = float(np.sum(n3 ** 3 / 3.0 + n3 ** 2 / 2.0 + n3 / 6.0))
    # the library factors the evaluated subsets largest padded size first
    # (stable); the first factorisation launch takes the first n_factor_first
    act_ids = np.nonzero(act)[0]
    npad = (nT + 63) // 64 * 64
    lpt = act_ids[np.argsort(-npad[act_ids], kind="stable")]

    def flops_of(ids):
        n = nT[ids].astype(np.float64)
        return float(np.sum(n ** 3 / 3.0 + n ** 2 / 2.0 + n / 6.0))

    import tempfile
    tune_cache = os.path.join(tempfile.mkdtemp(prefix="pcv_tune_"), "cache.txt")

    def run(prec, steps, warmup):
        """Timed evaluations on graph replays (after the autotuner picked the
        launch shapes and schedule), then a few evaluations of a second
        problem with the same configuration launched eagerly with HIP events
        between the phases, for the phase times and the factorisation
        kernel's time (roofline)."""
        t1 = time.perf_counter()
        P = pcv.Problem.from_workload(w, prec=prec, max_refine=a.max_refine, stream=stream)
        log(f"[{prec}] problem resident in {time.perf_counter() - t1:.1f}s: {P.info()}")
        tune = P.autotune(thetas[0], cache=tune_cache, reps=3) if a.tune else None
        if tune:
            log(f"[{prec}] autotune: {tune}")

        def step(Q, report):
            if len(thetas) > 1:
                # all theta values of the step in one batched evaluation;
                # phase times per theta are the batch's sums / K
                if not report:
                    return list(Q.eval_batch(thetas)), None
                losses, rep = Q.eval_batch(thetas, report=True)
                K = len(thetas)
                for k in ("ms_factor", "ms_solve", "ms_refine", "ms_predict", "ms_reduce", "ms_factor_all"):
                    rep[k] /= K
                rep["max_rel_residual"] = 0.0
                return list(losses), [rep]
            if not report:
                return [Q.eval(th) for th in thetas], None
            out = [Q.eval(th, report=True) for th in thetas]
            return [o[0] for o in out], [o[1] for o in out]

        for k in range(warmup):
            losses, _ = step(P, False)
            log(f"[{prec}] warmup {k}: loss {losses[0]:.12g}")
        torch.cuda.synchronize()
        tt = time.perf_counter()
        for k in range(steps):
            losses, _ = step(P, False)
        torch.cuda.synchronize()
        total = time.perf_counter() - tt
        log(f"[{prec}] {steps} timed steps (graph replays): {1e3 * total / steps:.2f} ms per step, "
            f"loss {losses[0]:.12g}")
        P.close()
        # phase times and the factorisation launch's time: eager launches with events
        Pp = pcv.Problem.from_workload(w, prec=prec, max_refine=a.max_refine, stream=stream, profile=True,
                                       est_error=True)
        if a.tune:
            Pp.autotune(thetas[0], cache=tune_cache, reps=3)  # the same choice, from the cache
        facs, facs_all = [], []
        step(Pp, True)
        for k in range(max(2, min(steps, 5))):
            lp, reps = step(Pp, True)
            facs += [r["ms_factor"] for r in reps]
            facs_all += [r["ms_factor_all"] for r in reps]
            r0 = reps[0]
            log(f"[{prec}] profiled {k}: loss {lp[0]:.12g} factor {r0['ms_factor']:.2f}ms "
                f"(all {r0['ms_factor_all']:.2f}) solve {r0['ms_solve']:.2f} refine {r0['ms_refine']:.2f} "
                f"predict {r0['ms_predict']:.2f}")
        if lp[0] != losses[0]:
            raise RuntimeError(f"graph and eager evaluations differ: {losses[0]!r} vs {lp[0]!r}")
        if len(thetas) > 1:
            # per-subset losses of the first theta for the oracle cross-check
            _, r1 = Pp.eval(thetas[0], report=True)
            reps[0]["per_subset_sspe"] = r1["per_subset_sspe"]
            reps[0]["max_rel_residual"] = r1["max_rel_residual"]
            reps[0]["est_rel_err"] = r1["est_rel_err"]
        Pp.close()
        return (losses, reps, total / (steps * len(thetas)), float(np.mean(facs)), float(np.mean(facs_all)),
                tune)

    losses, reps, s_per, ms_fac, ms_fac_all, tune = run(a.prec, a.steps, a.warmup)
    rep = reps[0]
    n_first = int(rep["n_factor_first"])
    flops_first = flops_of(lpt[:n_first])
    descr = {
        "large": "large fit: 5M jittered-lattice points with 15% in gaps, exponential covariance "
                 "range 50 nugget 0.1, 2400 recursive cores, 20% overlap",
        "plain": "plain FP64: 2,000 uniform points, exponential range 0.1 nugget 0.05, 2x2 cores, 10% overlap",
        "batched": "batched uniform: 100,000 uniform points, exponential range 0.05 nugget 0.1, "
                   "16x16 cores, 10% overlap, 8x8 theta grid per step",
        "uneven": "uneven batch: 1,000,000 Thomas-process points, Matern-3/2 range 0.03 nugget 0.02, "
                  "32x32 cores, 10% overlap, cap 4,000",
    }[a.workload]
    out = {
        "metric": METRIC, "value": s_per, "unit": "s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * s_per * len(thetas), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if a.prec == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": descr,
                   "n_points": int(len(w.y)), "subsets": int(pt.n_subsets),
                   "train_min": int(nT.min()), "train_max": int(nT.max()),
                   # evaluated subsets by training size (500-point buckets) and their total n^3
                   "size_histogram": {f"{500 * k}-{500 * k + 499}": int(c) for k, c in
                                      enumerate(np.bincount(nT[act] // 500)) if c},
                   "sum_n3": float(np.sum(nT[act].astype(np.float64) ** 3)),
                   "n_val": int(rep["n_val"]), "theta_per_step": len(thetas),
                   "precision": a.prec, "max_refine": a.max_refine,
                   "launch": ("graph replays of one launch per kernel for the step's theta values (batched)"
                         if len(thetas) > 1 else
                         ("graph replays; factorisation of the "
                          f"{n_first} largest subsets first, the other {int(act.sum()) - n_first} "
                          "factored on the same stream while the first group's solves, refinement "
                          "and kriging run on a second stream" if n_first < int(act.sum()) else
                          "graph replays, one launch per kernel over all subsets")),
              "autotune": tune},
    }
    peak = PEAK_FP32_MFMA if a.prec == "mixed" else PEAK_FP64_MFMA
    ach = flops_first / (ms_fac * 1e-3) / 1e12
    src = os.path.join(ROOT, "paper_1912_13132_amd", "csrc", "pcv_potrf.hip")
    # FP32 launches whose largest subset has npad <= 1536 use 256-thread workgroups
    # FP32 launches take 2-wave work-groups up to npad 704, 4-wave ones up to
    # the small-shape threshold, 8-wave ones above (from the launch's largest subset)
    small_npad = tune["small_npad"] if tune else 1536
    first_npad = int(npad[lpt[0]])
    shape = (128 if first_npad <= 704 else 256 if first_npad <= small_npad else 512) if a.prec == "mixed" else 512
    # the third template argument: the launch shares its largest subsets
    # between several workgroups
    n_coop = int(rep["n_coop_subsets"])
    kname = (f"k_potrf<{'float' if a.prec == 'mixed' else 'double'}, {shape}, {'true' if n_coop else 'false'}>"
             + (f" ({n_coop} largest subsets shared by several workgroups)" if n_coop else ""))
    out["roofline"] = {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                       "frac": ach / peak,
                       "traffic": (measured_traffic(src, a.prec, n_first)
                                   if a.workload == "large" and a.scale >= 1.0 else None),
                       "kernel": kname if n_first == int(act.sum()) else
                                 f"{kname}, first launch ({n_first} largest subsets)",
                       "kernel_ms": ms_fac, "flops_per_launch": flops_first,
                       "launch_subsets": n_first}
    # the factorisation of every subset, as seen on its stream (both launches)
    out["factorisation_all"] = {"ms": ms_fac_all, "flops": flops_potrf,
                                "frac": flops_potrf / (ms_fac_all * 1e-3) / 1e12 / peak}
    if copy_gbs is not None:
        out["copy_probe"] = {"mib": a.copy_probe_mib, "GB_per_s": copy_gbs}
    out["loss"] = losses[0]
    out["phase_ms"] = {k: rep[k] for k in ("ms_factor", "ms_solve", "ms_refine", "ms_predict", "ms_reduce")}
    out["max_rel_residual"] = max(r["max_rel_residual"] for r in reps)
    out["n_fallback_fp64"] = sum(r["n_fallback_fp64"] for r in reps)
    # the library's own estimate of the loss error against the FP64 path
    # (one more refinement sweep on a copy), beside the measured difference
    out["est_rel_err"] = reps[0]["est_rel_err"]
    if a.prec == "mixed" and not a.no_fp64:
        losses64, reps64, s64, ms64, ms64_all, tune64 = run("fp64", max(2, a.steps // 2), 1)
        n64 = int(reps64[0]["n_factor_first"])
        out["fp64_path"] = {"s_per_eval": s64, "loss": losses64[0], "factor_ms": ms64,
                            "factor_launch_subsets": n64,
                            "factor_frac_fp64_peak": flops_of(lpt[:n64]) / (ms64 * 1e-3) / 1e12 / PEAK_FP64_MFMA,
                            "factor_all_ms": ms64_all,
                            "factor_all_frac_fp64_peak": flops_potrf / (ms64_all * 1e-3) / 1e12 / PEAK_FP64_MFMA}
        out["rel_err_vs_fp64"] = max(abs(x - y) / abs(y) for x, y in zip(losses, losses64))
        out["speedup_vs_fp64_path"] = s64 / s_per
    if a.serve_seconds > 0 and a.workload == "large":
        out["serving"] = {
            "with_4_optimisers": serve(pcv, w, a.serve_seconds, log=log, warmup=a.serve_warmup,
                                       window=a.serve_window),
            "kriging_only": serve(pcv, w, min(a.serve_seconds, 15.0), with_evals=False, log=log,
                                  warmup=min(a.serve_warmup, 2.0), window=a.serve_window),
        }
    if not a.no_cpu:
        cb, rel = cpu_baseline(w, (thetas[0].range, thetas[0].lambda_), rep["per_subset_sspe"],
                               workload=a.workload)
        out["cpu_baseline"] = cb
        out["oracle_sample_max_rel_err"] = rel
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
