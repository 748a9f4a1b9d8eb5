"""The C-ABI library: it loads, exports every symbol the header declares, and rejects
invalid problems synchronously (validation runs before any device call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1502_06974_amd import wcal

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "wcal.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wcal_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = wcal.lib()
    syms = header_symbols()
    assert len(syms) >= 8
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(wcal.EXPORTS)
    assert b"gfx950" in L.wcal_version()


def _create(n_ant, a1, a2, ns, **kw):
    p = wcal.Problem(n_ant, len(a1), kw.get("n_dir", 1), kw.get("n_corr", 1), len(ns),
                     kw.get("algo", 0), kw.get("schedule", 0), kw.get("max_iter", 10), kw.get("tol", 1e-6),
                     kw.get("mode", 0), kw.get("precision", 0))
    a1 = np.asarray(a1, np.int32)
    a2 = np.asarray(a2, np.int32)
    ns = np.asarray(ns, np.int64)
    h = C.c_void_p()
    rc = wcal.lib().wcal_plan_create(C.byref(p), a1.ctypes.data_as(C.c_void_p), a2.ctypes.data_as(C.c_void_p),
                                     ns.ctypes.data_as(C.c_void_p), 0, C.byref(h))
    return rc, h


@pytest.mark.parametrize("a1,a2,ns,kw,code", [
    ([0, 0, 1], [1, 3, 2], [2], {}, wcal.EINDEX),          # antenna 3 out of range (n_ant = 3)
    ([0, -1, 1], [1, 2, 2], [2], {}, wcal.EINDEX),          # negative index
    ([0, 1, 1], [1, 1, 2], [2], {}, wcal.EINDEX),           # autocorrelation
    ([0, 0, 1], [1, 2, 2], [2, 0], {}, wcal.ESHAPE),        # empty interval
    ([0, 0, 1], [1, 2, 2], [2], {"n_corr": 2}, wcal.EINVAL),
    ([0, 0, 1], [1, 2, 2], [2], {"n_dir": 2}, wcal.EINVAL),            # StefCal with 2 directions
    ([0, 0, 1], [1, 2, 2], [2], {"algo": 1, "n_corr": 4, "precision": 1}, wcal.EINVAL),  # 2x2 DD + BF16
    ([0, 0, 1], [1, 2, 2], [2], {"algo": 1, "n_corr": 4, "n_dir": 11}, wcal.ESHAPE),     # 2x2 DD, Nd > 10
    ([0, 0, 1], [1, 2, 2], [2], {"algo": 1, "n_dir": 15}, wcal.ESHAPE),                  # scalar DD, Nd > 14
    ([0, 0, 1], [1, 2, 2], [2], {"algo": 1, "n_dir": 14, "precision": 1}, wcal.ESHAPE),  # BF16 Gram, Nd > 13
    ([0, 0, 1], [1, 2, 2], [], {}, wcal.EINVAL),                                          # no interval
    ([], [], [2], {}, wcal.EINVAL),                                                       # no baseline
    ([0, 0, 1], [1, 2, 2], [2], {"max_iter": 100001}, wcal.ESHAPE),
    ([0, 0, 1], [1, 2, 2], [2], {"max_iter": 0}, wcal.EINVAL),
    ([0, 0, 1], [1, 2, 2], [2], {"tol": -1.0}, wcal.EINVAL),
    ([0, 0, 1], [1, 2, 2], [2], {"schedule": 7}, wcal.EINVAL),
    ([0, 0, 1], [1, 2, 2], [2], {"mode": 5}, wcal.EINVAL),
    ([0, 0, 1], [1, 2, 2], [2], {"precision": 1}, wcal.EINVAL),         # BF16 Gram with StefCal
    ([0, 0, 1], [1, 2, 2], [2], {"algo": 1, "n_dir": 2, "precision": 7}, wcal.EINVAL),
    ([0, 0, 1], [1, 2, 2], [2], {"algo": 1, "n_dir": 2, "precision": 1, "mode": 1}, wcal.EINVAL),  # BF16 + STATS
])
def test_plan_validation_errors(a1, a2, ns, kw, code):
    rc, h = _create(3, a1, a2, ns, **kw)
    assert rc == code
    assert not h.value
    assert len(wcal.lib().wcal_last_error()) > 0


def test_plan_needs_two_antennas():
    rc, h = _create(1, [0], [0], [2])
    assert rc == wcal.EINVAL and not h.value


def test_null_arguments():
    L = wcal.lib()
    h = C.c_void_p()
    assert L.wcal_plan_create(None, None, None, None, 0, C.byref(h)) == wcal.EINVAL
    assert L.wcal_solve(*([None] * 10), 0, None) == wcal.EINVAL
    assert L.wcal_solve_static(*([None] * 10)) == wcal.EINVAL
    assert L.wcal_accumulate(*([None] * 12), 0, None) == wcal.EINVAL
    assert L.wcal_residual(*([None] * 8), 0, None) == wcal.EINVAL
    assert L.wcal_plan_rows(None) == -1
    n = C.c_size_t(7)
    assert L.wcal_plan_workspace(None, C.byref(n)) == wcal.EINVAL
    assert L.wcal_plan_autotune_workspace(None, C.byref(n)) == wcal.EINVAL
    assert L.wcal_plan_smoothing(None, 1, 4, 0.0, 1.0) == wcal.EINVAL
    assert L.wcal_solve_smooth(*([None] * 10), 0, None) == wcal.EINVAL
    assert L.wcal_solve_points(None, None, *([None] * 8), 0, None) == wcal.EINVAL
    assert L.wcal_points_workspace(None, None, C.byref(n)) == wcal.EINVAL
    assert L.wcal_plan_watch(None, 2) == wcal.EINVAL
    assert L.wcal_mlp_save(None, b"/tmp/x") == wcal.EINVAL
    assert L.wcal_mlp_load(None, b"/tmp/x") == wcal.EINVAL
    L.wcal_plan_destroy(None)


def test_valid_plan_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    rc, h = _create(3, [0, 0, 1], [1, 2, 2], [2])
    assert rc == wcal.EHIP


def test_warm_start_host_entry_points():
    """Knot indices (a host computation) match the oracle's definition; the warm-start
    entry points reject bad arguments before touching a device."""
    from oracle import mlp as om
    for n_int, bw in [(14, 4), (1, 1), (4096, 64), (150, 32), (7, 16), (300, 7)]:
        assert wcal.bin_knots(n_int, bw).tolist() == list(om.knots(n_int, bw))
    L = wcal.lib()
    k = np.zeros(4, np.int32)
    assert L.wcal_bin_knots(0, 4, k.ctypes.data_as(C.c_void_p)) == wcal.EINVAL
    assert L.wcal_bin_knots(5, 0, k.ctypes.data_as(C.c_void_p)) == wcal.EINVAL
    assert L.wcal_gather_knots(None, 4, None, None, None, None, None, None, None) == wcal.EINVAL
    assert L.wcal_bins_to_gains(5, 3, 0, None, None, None) == wcal.EINVAL
    assert L.wcal_gains_to_bins(5, 3, 2, -1, None, None, None) == wcal.EINVAL
    assert L.wcal_reset_unconverged(None, None, None, None) == wcal.EINVAL
    h = C.c_void_p()
    assert L.wcal_mlp_create(4, 8, 5, 16, 1, 0, C.byref(h)) == wcal.EINVAL      # skip needs d_in == d_out
    assert L.wcal_mlp_create(0, 8, 5, 16, 0, 0, C.byref(h)) == wcal.EINVAL
    assert not h.value
