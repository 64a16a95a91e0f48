"""Device-array arguments (the inputs_on_device option): a problem built from
torch tensors on the GPU, and predictions from device query tensors, give
the same bits as the host-array calls; pointers that are not device memory
of the right length are argument errors, caught on the host before any
copy."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1912_13132_amd import pcv
from paper_1912_13132_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def w_plain():
    return W.plain_fp64()


def _tensors(w, dev):
    import torch
    pt = w.part
    return (torch.tensor(w.locs, device=dev), torch.tensor(w.y, device=dev),
            torch.tensor(pt.train_ptr, device=dev), torch.tensor(pt.train_idx, dtype=torch.int32, device=dev),
            torch.tensor(pt.val_ptr, device=dev), torch.tensor(pt.val_idx, dtype=torch.int32, device=dev),
            torch.tensor(pt.core_rect, device=dev))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_device_inputs_same_bits_as_host(w_plain, prec):
    import torch
    say(f"[case] device inputs plain_fp64 prec={prec}")
    th = pcv.theta(0.1, 0.05, sigma2=1.3)
    r = np.random.default_rng(np.random.SeedSequence([1912, 13132, 700]))
    q = np.concatenate([r.uniform(0, 1, (257, 2)), [[1.0, 1.0], [1.3, -0.2]]])
    with pcv.Problem.from_workload(w_plain, prec=prec) as H:
        loss_h, rep_h = H.eval(th, report=True)
        H.factor(th)
        mh, vh, oh = H.predict(q)
    locs, y, tp, ti, vp, vi, rect = _tensors(w_plain, "cuda:0")
    with pcv.Problem(locs, y, tp, ti, vp, vi, core_rect=rect, prec=prec) as D:
        assert D.on_device
        del locs, y, tp, ti, vp, vi, rect  # nothing is kept after create
        torch.cuda.empty_cache()
        loss_d, rep_d = D.eval(th, report=True)
        D.factor(th)
        md, vd, od = D.predict(torch.tensor(q, device="cuda:0"))
        assert md.is_cuda and vd.is_cuda and od.is_cuda
        m0, v0, o0 = D.predict(torch.zeros((0, 2), dtype=torch.float64, device="cuda:0"))
        assert m0.numel() == 0
    assert loss_d == loss_h
    np.testing.assert_array_equal(rep_d["per_subset_sspe"], rep_h["per_subset_sspe"])
    np.testing.assert_array_equal(md.cpu().numpy(), mh)
    np.testing.assert_array_equal(vd.cpu().numpy(), vh)
    np.testing.assert_array_equal(od.cpu().numpy(), oh)


def _raw_create(w, ptrs, n=None):
    L = pcv.lib()
    opt = pcv.Options()
    L.pcv_default_options(ctypes.byref(opt))
    opt.inputs_on_device = 1
    h = ctypes.c_void_p()
    c = lambda a, t: ctypes.cast(ctypes.c_void_p(a), ctypes.POINTER(t))
    d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
    st = L.pcv_problem_create(ctypes.byref(h), len(w.y) if n is None else n, c(ptrs[0], d), c(ptrs[1], d),
                              w.part.n_subsets, c(ptrs[2], i64), c(ptrs[3], i32), c(ptrs[4], i64),
                              c(ptrs[5], i32), c(ptrs[6], d), ctypes.byref(opt))
    if st == 0:
        L.pcv_problem_destroy(h)
    return st, L.pcv_last_error().decode()


def test_device_option_rejects_host_pointers(w_plain):
    """inputs_on_device with host (numpy) arrays: PCV_ERR_INVALID, no copy."""
    pt = w_plain.part
    host = [np.ascontiguousarray(w_plain.locs), np.ascontiguousarray(w_plain.y),
            np.ascontiguousarray(pt.train_ptr, dtype=np.int64),
            np.ascontiguousarray(pt.train_idx, dtype=np.int32),
            np.ascontiguousarray(pt.val_ptr, dtype=np.int64),
            np.ascontiguousarray(pt.val_idx, dtype=np.int32), np.ascontiguousarray(pt.core_rect)]
    say("[case] inputs_on_device with host pointers")
    st, msg = _raw_create(w_plain, [a.ctypes.data for a in host])
    assert st == 1, msg
    assert "device" in msg


def test_device_option_rejects_short_array(w_plain):
    """A device locs array shorter than n points, reaching past its
    allocation: PCV_ERR_INVALID.  The test asks HIP for the allocation's
    extent first and only makes the call when the claimed length lies
    beyond it, which is what the library checks."""
    import torch
    hip = ctypes.CDLL("libamdhip64.so")
    ts = _tensors(w_plain, "cuda:0")
    short = torch.zeros((16, 2), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    base, size = ctypes.c_void_p(), ctypes.c_size_t()
    assert hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), ctypes.c_void_p(short.data_ptr())) == 0
    n_claim = len(w_plain.y) * 64
    end = base.value + size.value
    assert short.data_ptr() + 16 * n_claim > end, "allocation larger than expected: skip the call"
    say(f"[case] short device locs: allocation {size.value} B, claim {16 * n_claim} B")
    ptrs = [short.data_ptr()] + [t.data_ptr() for t in ts[1:]]
    st, msg = _raw_create(w_plain, ptrs, n=n_claim)
    assert st == 1, msg


def test_torch_usable_after_the_library():
    """A process that evaluates through the library before it touches torch
    can still use torch on the device (the binding loads torch's runtime
    first).  Run in a child process, so that nothing of this process's
    state decides the order."""
    import os
    import subprocess
    code = ("from paper_1912_13132_amd import pcv, workloads as W\n"
            "w = W.plain_fp64()\n"
            "P = pcv.Problem.from_workload(w)\n"
            "print('loss', P.eval(pcv.theta(0.1, 0.05)), flush=True)\n"
            "P.close()\n"
            "import torch\n"
            "t = torch.arange(5, dtype=torch.float64, device='cuda:0')\n"
            "print('torch', float(t.sum()), flush=True)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    say("[case] library first, then torch, in a child process")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=180)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "torch 10.0" in r.stdout, r.stdout
