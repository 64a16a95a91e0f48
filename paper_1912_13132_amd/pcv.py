"""ctypes binding of libpcv.so (the C ABI declared in include/pcv.h).

Argument marshalling only: every step of an evaluation or a prediction runs
in the library's HIP kernels.  The library must have been built
(``paper_1912_13132_amd.build.build()``); there is no fallback path, so a
missing library raises at first use.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcv.so")

PCV_OK = 0
STATUS = {0: "PCV_OK", 1: "PCV_ERR_INVALID", 2: "PCV_ERR_OOM", 3: "PCV_ERR_NOT_PD",
          4: "PCV_ERR_DEVICE", 5: "PCV_ERR_STATE", 6: "PCV_ERR_BUSY"}
COV_EXP = 0
COV_MATERN32 = 1
PREC_FP64 = 0
PREC_MIXED = 1
MAX_SUBSET = 16384
KRIGE_Q = 16  # queries per kriging work item (variance scratch npad x KRIGE_Q doubles)

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int32_p = ctypes.POINTER(ctypes.c_int32)
_c_int64_p = ctypes.POINTER(ctypes.c_int64)


class PcvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Theta(ctypes.Structure):
    _fields_ = [("cov", ctypes.c_int32), ("range", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("sigma2", ctypes.c_double)]


class TuneReport(ctypes.Structure):
    _fields_ = [("small_npad", ctypes.c_int32), ("max_wg_per_subset", ctypes.c_int32),
                ("two_groups", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("n_timed", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("default_s", ctypes.c_double), ("best_s", ctypes.c_double), ("tuning_s", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("refine_tol", ctypes.c_double), ("hip_stream", ctypes.c_void_p),
                ("mem_cap_bytes", ctypes.c_size_t), ("profile", ctypes.c_int32),
                ("debug_flags", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("inputs_on_device", ctypes.c_int32), ("max_wg_per_subset", ctypes.c_int32),
                ("est_error", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class EvalReport(ctypes.Structure):
    _fields_ = [("sspe", ctypes.c_double), ("n_val", ctypes.c_int64), ("mse", ctypes.c_double),
                ("n_subsets_used", ctypes.c_int32), ("n_fallback_fp64", ctypes.c_int32),
                ("max_refine_iters", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("max_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("ms_factor", ctypes.c_double), ("ms_solve", ctypes.c_double),
                ("ms_refine", ctypes.c_double), ("ms_predict", ctypes.c_double),
                ("ms_reduce", ctypes.c_double),
                ("per_subset_sspe", _c_double_p), ("per_subset_logdet", _c_double_p),
                ("per_subset_iters", _c_int32_p), ("neg2loglik", ctypes.c_double),
                ("per_subset_neg2loglik", _c_double_p), ("n_factor_first", ctypes.c_int32),
                ("n_coop_subsets", ctypes.c_int32), ("ms_factor_all", ctypes.c_double),
                ("est_rel_err", ctypes.c_double)]


class ServerReport(ctypes.Structure):
    _fields_ = [("n_predict", ctypes.c_int64), ("n_eval", ctypes.c_int64),
                ("n_queries", ctypes.c_int64), ("n_batches", ctypes.c_int64),
                ("mean_batch_queries", ctypes.c_double),
                ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double), ("max_s", ctypes.c_double),
                ("eval_p50_s", ctypes.c_double), ("eval_p99_s", ctypes.c_double),
                ("elapsed_s", ctypes.c_double), ("qps", ctypes.c_double),
                ("evals_per_s", ctypes.c_double), ("admission_waits", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("batch_query_cap", ctypes.c_int64),
                ("batch_item_cap", ctypes.c_int64)]


_lib = None


def lib():
    """Load libpcv.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1912_13132_amd.build.build()")
    # torch's HIP runtime is loaded before the library's: once the library has
    # initialised the device, torch can no longer initialise it in the same
    # process, and device tensors (the inputs_on_device option) need torch
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    L.pcv_default_options.argtypes = [ctypes.POINTER(Options)]
    L.pcv_default_options.restype = None
    L.pcv_problem_create.argtypes = [ctypes.POINTER(P), ctypes.c_int64, _c_double_p, _c_double_p,
                                     ctypes.c_int32, _c_int64_p, _c_int32_p, _c_int64_p, _c_int32_p,
                                     _c_double_p, ctypes.POINTER(Options)]
    L.pcv_eval.argtypes = [P, ctypes.POINTER(Theta), _c_double_p, ctypes.POINTER(EvalReport)]
    L.pcv_eval_batch.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Theta), _c_double_p]
    L.pcv_autotune.argtypes = [P, ctypes.POINTER(Theta), ctypes.c_char_p, ctypes.c_int32,
                               ctypes.POINTER(TuneReport)]
    L.pcv_eval_batch_ex.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Theta), _c_double_p,
                                    ctypes.POINTER(EvalReport)]
    L.pcv_factor.argtypes = [P, ctypes.POINTER(Theta)]
    L.pcv_factor_local.argtypes = [P, ctypes.POINTER(Theta)]
    L.pcv_gls.argtypes = [P, ctypes.c_int32, _c_double_p, _c_double_p, _c_int32_p]
    L.pcv_eval_grid.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Theta), _c_double_p, _c_double_p,
                                _c_int32_p]
    L.pcv_predict.argtypes = [P, ctypes.c_int64, _c_double_p, _c_double_p, _c_double_p,
                              ctypes.c_int32, _c_int32_p]
    L.pcv_predict_noalloc.argtypes = L.pcv_predict.argtypes
    L.pcv_problem_destroy.argtypes = [P]
    L.pcv_problem_info.argtypes = [P, _c_int32_p, _c_int64_p, _c_int32_p,
                                   ctypes.POINTER(ctypes.c_size_t)]
    L.pcv_server_create.argtypes = [ctypes.POINTER(P), P, ctypes.c_size_t, ctypes.c_int32]
    L.pcv_server_submit_predict.argtypes = [P, ctypes.c_int64, _c_double_p, _c_double_p, _c_double_p,
                                            ctypes.c_int32, _c_int64_p]
    L.pcv_server_submit_eval.argtypes = [P, ctypes.POINTER(Theta), _c_double_p, _c_int64_p]
    L.pcv_server_wait.argtypes = [P, ctypes.c_int64, ctypes.c_double]
    L.pcv_server_set_batch_window.argtypes = [P, ctypes.c_double]
    L.pcv_server_stats.argtypes = [P, _c_double_p, _c_double_p, _c_double_p, _c_double_p]
    L.pcv_server_report_get.argtypes = [P, ctypes.POINTER(ServerReport)]
    L.pcv_server_destroy.argtypes = [P]
    L.pcv_part_divide.argtypes = [ctypes.c_int64, _c_double_p, _c_double_p, ctypes.c_int32, ctypes.c_double,
                                  _c_double_p]
    L.pcv_part_count.argtypes = [ctypes.c_int64, _c_double_p, ctypes.c_int32, _c_double_p, ctypes.c_double,
                                 _c_int64_p]
    L.pcv_part_subsets.argtypes = [ctypes.c_int64, _c_double_p, ctypes.c_int32, _c_double_p, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_uint8), _c_int32_p, _c_int64_p, _c_int32_p,
                                   _c_int64_p, _c_int32_p]
    L.pcv_selftest_math.argtypes = [ctypes.c_int64, _c_double_p, _c_double_p, _c_double_p, _c_double_p]
    L.pcv_status_string.argtypes = [ctypes.c_int]
    L.pcv_status_string.restype = ctypes.c_char_p
    L.pcv_last_error.argtypes = []
    L.pcv_last_error.restype = ctypes.c_char_p
    for f in ("pcv_problem_create", "pcv_eval", "pcv_eval_batch", "pcv_factor", "pcv_predict",
              "pcv_problem_destroy", "pcv_problem_info", "pcv_server_create", "pcv_factor_local",
              "pcv_eval_grid", "pcv_gls", "pcv_eval_batch_ex", "pcv_part_divide", "pcv_part_count",
              "pcv_part_subsets", "pcv_selftest_math",
              "pcv_server_submit_predict", "pcv_server_submit_eval", "pcv_server_wait",
              "pcv_server_stats", "pcv_server_report_get", "pcv_server_destroy"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(st):
    if st != PCV_OK:
        raise PcvError(st, lib().pcv_last_error().decode())


def selftest_math(t, x):
    """Testing hook: e^{-t} and sqrt(x) by the device's FP64 functions."""
    t = _as(t, np.float64)
    x = _as(x, np.float64)
    if t.shape != x.shape:
        raise ValueError("t and x must have the same shape")
    e = np.zeros_like(t)
    r = np.zeros_like(x)
    _check(lib().pcv_selftest_math(t.size, _ptr(t, ctypes.c_double), _ptr(x, ctypes.c_double),
                                   _ptr(e, ctypes.c_double), _ptr(r, ctypes.c_double)))
    return e, r


def theta(range_, lam, cov=COV_EXP, sigma2=1.0):
    return Theta(int(cov), float(range_), float(lam), float(sigma2))


def _as(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _is_device_tensor(a):
    return getattr(a, "is_cuda", False) is True


def _dev(a, dtype, device):
    """A contiguous torch tensor of the given dtype on the device (no copy
    when it already is one)."""
    import torch
    return torch.as_tensor(a, dtype=dtype, device=device).contiguous()


def _dptr(t, ctype):
    return ctypes.cast(ctypes.c_void_p(t.data_ptr()), ctypes.POINTER(ctype))


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):      # torch.cuda.Stream
        return int(stream.cuda_stream)
    return int(stream)


def part_divide(locs, domain, m, delta):
    """Recursive balanced division into m cores on the device (Sec. 2.4)."""
    P = _as(locs, np.float64).reshape(-1, 2)
    dom = _as(domain, np.float64)
    out = np.zeros((int(m), 4))
    _check(lib().pcv_part_divide(P.shape[0], _ptr(P, ctypes.c_double), _ptr(dom, ctypes.c_double), int(m),
                                 float(delta), _ptr(out, ctypes.c_double)))
    return out


def part_count(locs, core_rect, delta):
    """Total core + shell memberships of all points on the device."""
    P = _as(locs, np.float64).reshape(-1, 2)
    R = _as(core_rect, np.float64).reshape(-1, 4)
    c = ctypes.c_int64()
    _check(lib().pcv_part_count(P.shape[0], _ptr(P, ctypes.c_double), R.shape[0], _ptr(R, ctypes.c_double),
                                float(delta), ctypes.byref(c)))
    return c.value


def part_subsets(locs, core_rect, delta, is_val=None, lists=True):
    """Owner of every point and, with lists=True, the training / validation
    CSR of the subsets (device construction)."""
    P = _as(locs, np.float64).reshape(-1, 2)
    R = _as(core_rect, np.float64).reshape(-1, 4)
    n, S = P.shape[0], R.shape[0]
    owner = np.zeros(n, dtype=np.int32)
    tp = np.zeros(S + 1, dtype=np.int64)
    vp = np.zeros(S + 1, dtype=np.int64)
    iv = None if is_val is None else _as(is_val, np.uint8)
    ivp = None if iv is None else iv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    L = lib()
    args = (n, _ptr(P, ctypes.c_double), S, _ptr(R, ctypes.c_double), float(delta), ivp)
    if not lists:
        _check(L.pcv_part_subsets(*args, _ptr(owner, ctypes.c_int32), None, None, None, None))
        return owner
    _check(L.pcv_part_subsets(*args, _ptr(owner, ctypes.c_int32), _ptr(tp, ctypes.c_int64), None,
                              _ptr(vp, ctypes.c_int64), None))
    ti = np.zeros(int(tp[-1]), dtype=np.int32)
    vi = np.zeros(int(vp[-1]), dtype=np.int32)
    _check(L.pcv_part_subsets(*args, None, _ptr(tp, ctypes.c_int64), _ptr(ti, ctypes.c_int32),
                              _ptr(vp, ctypes.c_int64), _ptr(vi, ctypes.c_int32)))
    return owner, tp, ti, vp, vi


class Problem:
    """A divided problem resident on the current HIP device (Algorithm 1,
    steps 2-5: divide and read once, evaluate many zeta)."""

    def __init__(self, locs, y, train_ptr, train_idx, val_ptr, val_idx, core_rect=None,
                 prec="mixed", max_refine=2, refine_tol=1e-4, stream=None, mem_cap=0,
                 profile=False, debug_flags=0, graph=True, max_wg_per_subset=0, est_error=False):
        """Arrays are numpy-like (host) or, when locs is a torch tensor on the
        GPU, torch tensors on that device (the library's inputs_on_device
        option); predict then takes and returns device tensors too."""
        L = lib()
        self.on_device = _is_device_tensor(locs)
        if self.on_device:
            import torch
            self._device = locs.device
            conv = lambda a, dt: _dev(a, dt, self._device)
            f64, i64, i32 = torch.float64, torch.int64, torch.int32
            ptr = _dptr
        else:
            conv = _as
            f64, i64, i32 = np.float64, np.int64, np.int32
            ptr = _ptr
        locs_ = conv(locs, f64).reshape(-1, 2)
        y_ = conv(y, f64)
        tp_ = conv(train_ptr, i64)
        ti_ = conv(train_idx, i32)
        vp_ = conv(val_ptr, i64)
        vi_ = conv(val_idx, i32)
        rect_ = None if core_rect is None else conv(core_rect, f64).reshape(-1, 4)
        self.S = int(tp_.shape[0] - 1)
        opt = Options()
        L.pcv_default_options(ctypes.byref(opt))
        opt.prec = PREC_MIXED if prec == "mixed" else PREC_FP64
        opt.max_refine = int(max_refine)
        opt.refine_tol = float(refine_tol)
        opt.hip_stream = _stream_handle(stream)
        opt.mem_cap_bytes = int(mem_cap)
        opt.profile = 1 if profile else 0
        opt.debug_flags = int(debug_flags)
        opt.est_error = 1 if est_error else 0
        opt.graph = 1 if graph else 0
        opt.inputs_on_device = 1 if self.on_device else 0
        opt.max_wg_per_subset = int(max_wg_per_subset)
        self.prec = prec
        h = ctypes.c_void_p()
        _check(L.pcv_problem_create(
            ctypes.byref(h), locs_.shape[0], ptr(locs_, ctypes.c_double),
            ptr(y_, ctypes.c_double), self.S, ptr(tp_, ctypes.c_int64),
            ptr(ti_, ctypes.c_int32), ptr(vp_, ctypes.c_int64),
            ptr(vi_, ctypes.c_int32),
            None if rect_ is None else ptr(rect_, ctypes.c_double), ctypes.byref(opt)))
        self._h = h

    @classmethod
    def from_workload(cls, w, **kw):
        pt = w.part
        return cls(w.locs, w.y, pt.train_ptr, pt.train_idx, pt.val_ptr, pt.val_idx,
                   core_rect=pt.core_rect, **kw)

    def _handle(self):
        if self._h is None:
            raise PcvError(1, "problem destroyed")
        return self._h

    def eval(self, th, report=False):
        """One theta-evaluation; returns the loss (SSPE, eq. (7)), or
        (loss, report dict) when report=True."""
        L = lib()
        loss = ctypes.c_double()
        if not report:
            _check(L.pcv_eval(self._handle(), ctypes.byref(th), ctypes.byref(loss), None))
            return loss.value
        rep = EvalReport()
        z = np.zeros(self.S)
        ld = np.zeros(self.S)
        it = np.zeros(self.S, dtype=np.int32)
        rep.per_subset_sspe = _ptr(z, ctypes.c_double)
        rep.per_subset_logdet = _ptr(ld, ctypes.c_double)
        rep.per_subset_iters = _ptr(it, ctypes.c_int32)
        nll = np.zeros(self.S)
        rep.per_subset_neg2loglik = _ptr(nll, ctypes.c_double)
        _check(L.pcv_eval(self._handle(), ctypes.byref(th), ctypes.byref(loss), ctypes.byref(rep)))
        d = {k: getattr(rep, k) for k, _ in EvalReport._fields_
             if not k.startswith("per_subset") and k != "pad0"}
        d.update(per_subset_sspe=z, per_subset_logdet=ld, per_subset_iters=it,
                 per_subset_neg2loglik=nll)
        return loss.value, d

    def autotune(self, th, cache=None, reps=3):
        """Pick the launch shapes and schedule by timing pcv_eval at th
        (pcv_autotune); returns the chosen configuration and timings."""
        r = TuneReport()
        _check(lib().pcv_autotune(self._handle(), ctypes.byref(th),
                                  None if cache is None else os.fsencode(cache), int(reps), ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in TuneReport._fields_ if k != "pad0"}

    def eval_batch(self, thetas, report=False):
        """Losses of several theta values, evaluated together; with
        report=True also the batch report (wall time, summed phase times when
        profiling, theta values evaluated again on their own)."""
        L = lib()
        arr = (Theta * len(thetas))(*thetas)
        out = np.zeros(len(thetas))
        if not report:
            _check(L.pcv_eval_batch(self._handle(), len(thetas), arr, _ptr(out, ctypes.c_double)))
            return out
        rep = EvalReport()
        _check(L.pcv_eval_batch_ex(self._handle(), len(thetas), arr, _ptr(out, ctypes.c_double),
                                   ctypes.byref(rep)))
        d = {k: getattr(rep, k) for k, _ in EvalReport._fields_
             if not k.startswith("per_subset") and k != "pad0"}
        return out, d

    def eval_grid(self, thetas):
        """Losses, per-subset losses [K][S] and the best local theta index of
        each subset (-1 where nothing is evaluated)."""
        K = len(thetas)
        arr = (Theta * K)(*thetas)
        losses = np.zeros(K)
        z = np.zeros((K, self.S))
        best = np.zeros(self.S, dtype=np.int32)
        _check(lib().pcv_eval_grid(self._handle(), K, arr, _ptr(losses, ctypes.c_double),
                                   _ptr(z, ctypes.c_double), _ptr(best, ctypes.c_int32)))
        return losses, z, best

    def factor(self, th):
        _check(lib().pcv_factor(self._handle(), ctypes.byref(th)))

    def factor_local(self, thetas):
        """Factor subset i at thetas[i] (len(thetas) == S)."""
        if len(thetas) != self.S:
            raise PcvError(1, f"need {self.S} theta values, got {len(thetas)}")
        arr = (Theta * self.S)(*thetas)
        _check(lib().pcv_factor_local(self._handle(), arr))

    def predict(self, q, want_var=True, obs_noise=False, noalloc=False):
        """Kriging mean, variance (or None) and owning subset of every query;
        noalloc=True goes through pcv_predict_noalloc (no device allocation,
        at most 262,144 queries per call)."""
        fn = lib().pcv_predict_noalloc if noalloc else lib().pcv_predict
        if self.on_device:
            import torch
            q = _dev(q, torch.float64, self._device).reshape(-1, 2)
            nq = q.shape[0]
            mean = torch.zeros(nq, dtype=torch.float64, device=self._device)
            var = torch.zeros(nq, dtype=torch.float64, device=self._device) if want_var else None
            owner = torch.zeros(nq, dtype=torch.int32, device=self._device)
            _check(fn(self._handle(), nq, _dptr(q, ctypes.c_double),
                                     _dptr(mean, ctypes.c_double),
                                     None if var is None else _dptr(var, ctypes.c_double),
                                     1 if obs_noise else 0, _dptr(owner, ctypes.c_int32)))
            return mean, var, owner
        if _is_device_tensor(q):
            q = q.cpu().numpy()
        q = _as(q, np.float64).reshape(-1, 2)
        nq = q.shape[0]
        mean = np.zeros(nq)
        var = np.zeros(nq) if want_var else None
        owner = np.zeros(nq, dtype=np.int32)
        _check(fn(self._handle(), nq, _ptr(q, ctypes.c_double),
                                 _ptr(mean, ctypes.c_double),
                                 None if var is None else _ptr(var, ctypes.c_double),
                                 1 if obs_noise else 0, _ptr(owner, ctypes.c_int32)))
        return mean, var, owner

    def gls(self, X):
        """GLS mean coefficients [S][p] per subset from covariates X [n][p]
        (Sec. 5, eq. (8)), through the resident factors; also the status."""
        X = _as(X, np.float64)
        if X.ndim == 1:
            X = X[:, None]
        X = np.ascontiguousarray(X)
        beta = np.zeros((self.S, X.shape[1]))
        st = np.zeros(self.S, dtype=np.int32)
        _check(lib().pcv_gls(self._handle(), X.shape[1], _ptr(X, ctypes.c_double),
                             _ptr(beta, ctypes.c_double), _ptr(st, ctypes.c_int32)))
        return beta, st

    def info(self):
        S = ctypes.c_int32()
        nnz = ctypes.c_int64()
        mx = ctypes.c_int32()
        b = ctypes.c_size_t()
        _check(lib().pcv_problem_info(self._handle(), ctypes.byref(S), ctypes.byref(nnz),
                                      ctypes.byref(mx), ctypes.byref(b)))
        return dict(S=S.value, nnz_train=nnz.value, max_train=mx.value, device_bytes=b.value)

    def close(self):
        if self._h is not None:
            lib().pcv_problem_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop over a factored problem (continuous batching of kriging
    requests, concurrent theta-evaluations).  The problem must not be used
    directly while the server exists.  Submit calls may come from several
    threads; they release the GIL while they block on admission."""

    def __init__(self, problem, mem_budget=0, max_inflight=64, window=None):
        self.problem = problem
        h = ctypes.c_void_p()
        _check(lib().pcv_server_create(ctypes.byref(h), problem._handle(), int(mem_budget),
                                       int(max_inflight)))
        self._h = h
        self._keep = {}
        if window is not None:
            st = lib().pcv_server_set_batch_window(h, float(window))
            if st != 0:
                err = PcvError(st, lib().pcv_last_error().decode())
                self.close()
                raise err

    def _handle(self):
        if self._h is None:
            raise PcvError(1, "server destroyed")
        return self._h

    def submit_predict(self, q, want_var=True, obs_noise=False):
        """Queue kriging at query locations q ([k][2]); returns a ticket."""
        q = _as(q, np.float64).reshape(-1, 2)
        nq = q.shape[0]
        mean = np.zeros(nq)
        var = np.zeros(nq) if want_var else None
        t = ctypes.c_int64()
        _check(lib().pcv_server_submit_predict(
            self._handle(), nq, _ptr(q, ctypes.c_double), _ptr(mean, ctypes.c_double),
            None if var is None else _ptr(var, ctypes.c_double), 1 if obs_noise else 0,
            ctypes.byref(t)))
        self._keep[t.value] = ("predict", q, mean, var)
        return t.value

    def submit_eval(self, th):
        """Queue one theta-evaluation; returns a ticket."""
        loss = np.zeros(1)
        t = ctypes.c_int64()
        _check(lib().pcv_server_submit_eval(self._handle(), ctypes.byref(th),
                                            _ptr(loss, ctypes.c_double), ctypes.byref(t)))
        self._keep[t.value] = ("eval", th, loss)
        return t.value

    def wait(self, ticket, timeout=-1.0):
        """(mean, var) of a kriging request or the loss of an evaluation.
        Raises PcvError with status PCV_ERR_BUSY on timeout."""
        _check(lib().pcv_server_wait(self._handle(), int(ticket), float(timeout)))
        k = self._keep.pop(ticket)
        if k[0] == "predict":
            return k[2], k[3]
        return float(k[2][0])

    def stats(self):
        v = [ctypes.c_double() for _ in range(4)]
        _check(lib().pcv_server_stats(self._handle(), *[ctypes.byref(x) for x in v]))
        return dict(p50_s=v[0].value, p99_s=v[1].value, qps=v[2].value, evals_per_s=v[3].value)

    def report(self):
        r = ServerReport()
        _check(lib().pcv_server_report_get(self._handle(), ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in ServerReport._fields_}

    def close(self):
        if self._h is not None:
            lib().pcv_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
