"""C ABI checks that need no GPU: the library loads, exports every function
include/pcv.h declares, and rejects invalid arguments before any device
work (validation precedes the first HIP call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1912_13132_amd import pcv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "pcv.h")).read()
    txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)
    names = re.findall(r"\b(pcv_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("pcv_problem_create", "pcv_eval", "pcv_eval_batch", "pcv_factor",
                     "pcv_predict", "pcv_problem_destroy", "pcv_status_string", "pcv_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = pcv.lib()
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def _tiny():
    r = np.random.default_rng(0)
    locs = r.uniform(0, 1, (10, 2))
    y = r.standard_normal(10)
    return locs, y


def _create(locs, y, tp, ti, vp, vi, rect=None, **kw):
    return pcv.Problem(locs, y, tp, ti, vp, vi, core_rect=rect, **kw)


@pytest.mark.parametrize("case", [
    "idx_out_of_range", "neg_idx", "ptr_decreasing", "ptr_not_zero", "nan_y", "inf_loc",
    "too_large", "bad_prec_refine", "bad_max_wg",
])
def test_invalid_arguments_rejected_before_device_work(case):
    locs, y = _tiny()
    tp, ti = [0, 5, 8], [0, 1, 2, 3, 4, 5, 6, 7]
    vp, vi = [0, 1, 2], [8, 9]
    kw = {}
    if case == "idx_out_of_range":
        ti = [0, 1, 2, 3, 4, 5, 6, 10]
    elif case == "neg_idx":
        vi = [8, -1]
    elif case == "ptr_decreasing":
        tp = [0, 5, 4]
        ti = ti[:4]
    elif case == "ptr_not_zero":
        tp = [1, 5, 8]
    elif case == "nan_y":
        y = y.copy()
        y[3] = np.nan
    elif case == "inf_loc":
        locs = locs.copy()
        locs[2, 1] = np.inf
    elif case == "too_large":
        n = pcv.MAX_SUBSET + 1
        locs = np.zeros((n, 2))
        y = np.zeros(n)
        tp, ti = [0, n], np.arange(n)
        vp, vi = [0, 0], []
    elif case == "bad_prec_refine":
        kw = dict(max_refine=99)
    elif case == "bad_max_wg":
        kw = dict(max_wg_per_subset=9)
    with pytest.raises(pcv.PcvError) as e:
        _create(locs, y, tp, ti, vp, vi, **kw)
    assert e.value.status == 1


def test_status_strings():
    L = pcv.lib()
    assert L.pcv_status_string(0) == b"PCV_OK"
    assert L.pcv_status_string(3) == b"PCV_ERR_NOT_PD"


def test_server_calls_reject_null_handles():
    """The serving calls validate their handles before any device work."""
    L = pcv.lib()
    out = ctypes.c_void_p(1)
    assert L.pcv_server_create(ctypes.byref(out), None, 0, 4) == 1
    assert out.value is None
    assert L.pcv_server_create(None, None, 0, 4) == 1
    t = ctypes.c_int64()
    q = np.zeros((1, 2))
    m = np.zeros(1)
    assert L.pcv_server_submit_predict(None, 1, q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, 0,
                                       ctypes.byref(t)) == 1
    th = pcv.theta(0.1, 0.1)
    loss = ctypes.c_double()
    assert L.pcv_server_submit_eval(None, ctypes.byref(th), ctypes.byref(loss), ctypes.byref(t)) == 1
    assert L.pcv_server_wait(None, 1, 0.0) == 1
    assert L.pcv_server_stats(None, None, None, None, None) == 1
    assert L.pcv_server_report_get(None, None) == 1
    assert L.pcv_server_destroy(None) == 1
    assert b"NULL" in L.pcv_last_error()


def test_partition_calls_validate_before_device_work():
    P = np.array([[0.1, 0.2], [0.3, np.nan]])
    dom = np.array([0.0, 0.0, 1.0, 1.0])
    with pytest.raises(pcv.PcvError) as e:
        pcv.part_divide(P, dom, 4, 0.0)
    assert e.value.status == 1
    with pytest.raises(pcv.PcvError) as e:
        pcv.part_divide(np.zeros((3, 2)), dom, 4, -1.0)
    assert e.value.status == 1
    with pytest.raises(pcv.PcvError) as e:
        pcv.part_count(np.zeros((3, 2)), np.array([[0.0, 0.0, -1.0, 1.0]]), 0.1)
    assert e.value.status == 1
