"""Python binding of the C ABI in include/wcal.h (ctypes).

Argument marshalling only: every step of the calibration runs in the HIP
kernels of libwcal.so.  torch tensors supply device memory and the stream.
The library must have been built (``paper_1502_06974_amd.build``); loading
fails loudly otherwise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libwcal.so")

OK, EINVAL, EINDEX, ESHAPE, EHIP, ENOMEM, EIO = 0, -1, -2, -3, -4, -5, -6
CONVERGED, MAXITER, SINGULAR_ANT, NONFINITE, ABORTED = 1, 2, 4, 8, 16
WS_ALIGN = 256
STATIC_WORKSPACE_BYTES = 64 << 20   # WCAL_STATIC_WORKSPACE_BYTES
STEFCAL, COHJONES, ALLJONES = 0, 1, 2
AVG_FIRST, GN_FIRST, GN_ONLY = 0, 1, 2
_ALGOS = {"stefcal": STEFCAL, "cohjones": COHJONES, "alljones": ALLJONES}
_SCHED = {"avg_first": AVG_FIRST, "gn_first": GN_FIRST, "gn_only": GN_ONLY}
MODE_PASS, MODE_STATS = 0, 1
_MODES = {"pass": MODE_PASS, "stats": MODE_STATS}
PREC_FP32, PREC_BF16_GRAM = 0, 1
_PRECS = {"fp32": PREC_FP32, "bf16": PREC_BF16_GRAM}

# every symbol the header declares
EXPORTS = ("wcal_last_error", "wcal_version", "wcal_plan_create", "wcal_plan_destroy",
           "wcal_plan_rows", "wcal_plan_workspace", "wcal_plan_autotune_workspace",
           "wcal_plan_pass_kernel", "wcal_plan_autotune", "wcal_solve", "wcal_solve_graph", "wcal_graph_launch",
           "wcal_graph_destroy", "wcal_accumulate", "wcal_residual",
           "wcal_profile_enable", "wcal_profile_read", "wcal_bin_knots", "wcal_gather_knots", "wcal_bins_to_gains",
           "wcal_gains_to_bins", "wcal_reset_unconverged", "wcal_mlp_create", "wcal_mlp_destroy",
           "wcal_mlp_num_params", "wcal_mlp_set_params", "wcal_mlp_get_params", "wcal_mlp_forward",
           "wcal_mlp_gradients", "wcal_mlp_train_step", "wcal_mlp_save", "wcal_mlp_load",
           "wcal_plan_smoothing", "wcal_solve_smooth", "wcal_solve_points", "wcal_points_workspace", "wcal_solve_static",
           "wcal_plan_watch")
K_CLASSES = ("pass", "update", "stats", "solve_stats", "resid", "other")


class WcalError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"wcal error {code}: {msg}")
        self.code = code


class Points(C.Structure):
    _fields_ = [("n_time", C.c_int32), ("n_chan", C.c_int32), ("freq0", C.c_double), ("dfreq", C.c_double),
                ("uvw", C.c_void_p), ("lmn", C.c_void_p), ("flux", C.c_void_p)]


class Problem(C.Structure):
    _fields_ = [("n_ant", C.c_int32), ("n_bl", C.c_int32), ("n_dir", C.c_int32),
                ("n_corr", C.c_int32), ("n_int", C.c_int32), ("algo", C.c_int32),
                ("schedule", C.c_int32), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("mode", C.c_int32), ("precision", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    """Load libwcal.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with paper_1502_06974_amd.build "
                           "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i32p, u8p = C.c_void_p, C.c_void_p, C.c_void_p
    L.wcal_last_error.restype = C.c_char_p
    L.wcal_version.restype = C.c_char_p
    L.wcal_plan_create.argtypes = [C.POINTER(Problem), vp, vp, vp, C.c_int, C.POINTER(C.c_void_p)]
    L.wcal_plan_create.restype = C.c_int
    L.wcal_plan_destroy.argtypes = [vp]
    L.wcal_plan_destroy.restype = None
    L.wcal_plan_rows.argtypes = [vp]
    L.wcal_plan_rows.restype = C.c_int64
    L.wcal_plan_workspace.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.wcal_plan_workspace.restype = C.c_int
    L.wcal_plan_autotune_workspace.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.wcal_plan_autotune_workspace.restype = C.c_int
    L.wcal_plan_autotune.argtypes = [vp, vp, vp, vp, vp, C.c_int32, vp, C.c_size_t, vp, vp, vp]
    L.wcal_plan_autotune.restype = C.c_int
    L.wcal_plan_pass_kernel.argtypes = [vp]
    L.wcal_plan_pass_kernel.restype = C.c_char_p
    L.wcal_solve.argtypes = [vp] * 10 + [C.c_size_t, vp]
    L.wcal_solve.restype = C.c_int
    L.wcal_solve_static.argtypes = [vp] * 10
    L.wcal_solve_static.restype = C.c_int
    L.wcal_solve_graph.argtypes = [vp] * 10 + [C.c_size_t, vp, C.POINTER(C.c_void_p)]
    L.wcal_solve_graph.restype = C.c_int
    L.wcal_graph_launch.argtypes = [vp, vp]
    L.wcal_graph_launch.restype = C.c_int
    L.wcal_graph_destroy.argtypes = [vp]
    L.wcal_graph_destroy.restype = None
    L.wcal_accumulate.argtypes = [vp] * 12 + [C.c_size_t, vp]
    L.wcal_accumulate.restype = C.c_int
    L.wcal_residual.argtypes = [vp] * 8 + [C.c_size_t, vp]
    L.wcal_residual.restype = C.c_int
    L.wcal_plan_smoothing.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, C.c_double]
    L.wcal_plan_smoothing.restype = C.c_int
    L.wcal_solve_smooth.argtypes = [vp] * 10 + [C.c_size_t, vp]
    L.wcal_solve_smooth.restype = C.c_int
    L.wcal_solve_points.argtypes = [vp, C.POINTER(Points)] + [vp] * 8 + [C.c_size_t, vp]
    L.wcal_solve_points.restype = C.c_int
    L.wcal_points_workspace.argtypes = [vp, C.POINTER(Points), C.POINTER(C.c_size_t)]
    L.wcal_points_workspace.restype = C.c_int
    L.wcal_profile_enable.argtypes = [vp, C.c_int]
    L.wcal_profile_enable.restype = C.c_int
    L.wcal_plan_watch.argtypes = [vp, C.c_int32]
    L.wcal_plan_watch.restype = C.c_int
    L.wcal_profile_read.argtypes = [vp, vp, vp]
    L.wcal_profile_read.restype = C.c_int
    L.wcal_bin_knots.argtypes = [C.c_int32, C.c_int32, vp]
    L.wcal_gather_knots.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, vp, vp]
    L.wcal_bins_to_gains.argtypes = [C.c_int32, C.c_int32, C.c_int32, vp, vp, vp]
    L.wcal_gains_to_bins.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp]
    L.wcal_reset_unconverged.argtypes = [vp, vp, vp, vp]
    L.wcal_mlp_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int,
                                  C.POINTER(C.c_void_p)]
    L.wcal_mlp_destroy.argtypes = [vp]
    L.wcal_mlp_destroy.restype = None
    L.wcal_mlp_num_params.argtypes = [vp]
    L.wcal_mlp_num_params.restype = C.c_int64
    L.wcal_mlp_set_params.argtypes = [vp, vp, vp]
    L.wcal_mlp_get_params.argtypes = [vp, vp, vp]
    L.wcal_mlp_forward.argtypes = [vp, vp, C.c_int32, vp, vp]
    L.wcal_mlp_gradients.argtypes = [vp, vp, vp, C.c_int32, vp, vp, vp]
    L.wcal_mlp_train_step.argtypes = [vp, vp, vp, C.c_int32, C.c_float, vp, vp]
    L.wcal_mlp_save.argtypes = [vp, C.c_char_p]
    L.wcal_mlp_load.argtypes = [vp, C.c_char_p]
    for f in ("wcal_bin_knots", "wcal_gather_knots", "wcal_bins_to_gains", "wcal_gains_to_bins", "wcal_reset_unconverged",
              "wcal_mlp_create", "wcal_mlp_set_params", "wcal_mlp_get_params", "wcal_mlp_forward",
              "wcal_mlp_gradients", "wcal_mlp_train_step", "wcal_mlp_save", "wcal_mlp_load", "wcal_plan_smoothing",
              "wcal_solve_smooth", "wcal_solve_points"):
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise WcalError(rc, lib().wcal_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


class Plan:
    """A validated calibration problem with its device tables (wraps wcal_plan)."""

    def __init__(self, n_ant: int, ant1, ant2, ns, n_dir: int = 1, n_corr: int = 1,
                 algo: str = "stefcal", schedule: str = "avg_first", max_iter: int = 100,
                 tol: float = 1e-6, device: int = 0, mode: str = "pass", precision: str = "fp32"):
        L = lib()
        a1 = torch.as_tensor(ant1, dtype=torch.int32).cpu().contiguous()
        a2 = torch.as_tensor(ant2, dtype=torch.int32).cpu().contiguous()
        nsv = torch.as_tensor(ns, dtype=torch.int64).cpu().contiguous()
        self.prob = Problem(n_ant, a1.numel(), n_dir, n_corr, nsv.numel(), _ALGOS[algo],
                            _SCHED[schedule], max_iter, tol, _MODES[mode], _PRECS[precision])
        self.n_ant, self.n_bl, self.n_dir, self.n_corr, self.n_int = n_ant, a1.numel(), n_dir, n_corr, nsv.numel()
        self.device = device
        self.ant1, self.ant2, self.ns = a1, a2, nsv
        self._h = C.c_void_p()
        _check(L.wcal_plan_create(C.byref(self.prob), _ptr(a1), _ptr(a2), _ptr(nsv), device,
                                  C.byref(self._h)))
        self.rows = int(L.wcal_plan_rows(self._h))
        self.pass_kernel = L.wcal_plan_pass_kernel(self._h).decode()
        self._ws = None
        self._pws = None   # workspace of the points solve (the plan's plus the phasor table)

    # ---------------------------------------------------------------- workspace
    def workspace_bytes(self) -> int:
        """wcal_plan_workspace: device scratch every compute call on this plan needs."""
        n = C.c_size_t(0)
        _check(lib().wcal_plan_workspace(self._h, C.byref(n)))
        return int(n.value)

    @staticmethod
    def _alloc(nbytes: int, device) -> torch.Tensor:
        ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
        if ws.data_ptr() % WS_ALIGN:
            raise RuntimeError("torch returned a workspace that is not 256-byte aligned")
        return ws

    def workspace(self, device=None) -> torch.Tensor:
        """The plan's workspace (a uint8 device tensor owned by this object, allocated by torch
        on first use and whenever the plan needs more)."""
        need = self.workspace_bytes()
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = self._alloc(need, device if device is not None else torch.device("cuda", self.device))
        return self._ws

    def _ws_args(self, workspace):
        ws = self.workspace() if workspace is None else workspace
        return _ptr(ws), C.c_size_t(ws.numel()), ws

    def close(self):
        if self._h:
            lib().wcal_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool = True):
        """Bracket every kernel of later solve/residual calls with HIP events."""
        _check(lib().wcal_profile_enable(self._h, int(enable)))

    def watch(self, depth: int = 4):
        """Host watch of the per-update launches (wcal_plan_watch): later eager solves stop
        enqueuing update slots once every interval has stopped, keeping at most `depth` slots
        in flight past the last count read (the call then blocks the host until the solve is
        that close to its end).  depth 0 turns it off."""
        _check(lib().wcal_plan_watch(self._h, int(depth)))

    def profile_read(self) -> dict:
        """{class: (total ms, launches)} since the previous read (waits for the events)."""
        ms = (C.c_double * len(K_CLASSES))()
        n = (C.c_int32 * len(K_CLASSES))()
        _check(lib().wcal_profile_read(self._h, ms, n))
        return {c: (ms[i], n[i]) for i, c in enumerate(K_CLASSES)}

    # ---------------------------------------------------------------- argument checks
    def _dev(self, t, name, dtype, shape):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def _inputs(self, data, model, flags, gains):
        R, nc, nd = self.rows, self.n_corr, self.n_dir
        self._dev(data, "data", torch.complex64, (R, nc))
        self._dev(model, "model", torch.complex64, (R, nd, nc))
        if flags is not None:
            self._dev(flags, "flags", torch.uint8, (R,))
        self._dev(gains, "gains", torch.complex64, (self.n_int, nd, self.n_ant, nc))

    @staticmethod
    def _stream(stream):
        if stream is None:
            stream = torch.cuda.current_stream()
        return C.c_void_p(stream.cuda_stream)

    # ---------------------------------------------------------------- calls
    def solve(self, data, model, flags, gains, residual=None, n_iter=None, status=None,
              chi2=None, stream=None, want_residual: bool = True, want_chi2: bool = True, workspace=None):
        """wcal_solve: gains are updated in place.  Returns dict of output tensors."""
        self._inputs(data, model, flags, gains)
        dev = gains.device
        if residual is None and want_residual:
            residual = torch.empty_like(data)
        if n_iter is None:
            n_iter = torch.empty(self.n_int, dtype=torch.int32, device=dev)
        if status is None:
            status = torch.empty(self.n_int, dtype=torch.int32, device=dev)
        if chi2 is None and want_chi2:
            chi2 = torch.empty(self.n_int, dtype=torch.float64, device=dev)
        self._dev(residual, "residual", torch.complex64, (self.rows, self.n_corr))
        self._dev(n_iter, "n_iter", torch.int32, (self.n_int,))
        self._dev(status, "status", torch.int32, (self.n_int,))
        self._dev(chi2, "chi2", torch.float64, (self.n_int,))
        wp, wn, _ = self._ws_args(workspace)
        _check(lib().wcal_solve(self._h, _ptr(data), _ptr(model), _ptr(flags), _ptr(gains),
                                _ptr(residual), _ptr(n_iter), _ptr(status), _ptr(chi2), wp, wn,
                                self._stream(stream)))
        return dict(gains=gains, residual=residual, n_iter=n_iter, status=status, chi2=chi2)

    def solve_static(self, data, model, flags, gains, residual=None, n_iter=None, status=None,
                     chi2=None, stream=None, want_residual: bool = True, want_chi2: bool = True):
        """wcal_solve_static: wcal_solve with the library's static device workspace (the call
        itself allocates nothing; outputs not passed in are allocated here, before it)."""
        self._inputs(data, model, flags, gains)
        dev = gains.device
        if residual is None and want_residual:
            residual = torch.empty_like(data)
        if n_iter is None:
            n_iter = torch.empty(self.n_int, dtype=torch.int32, device=dev)
        if status is None:
            status = torch.empty(self.n_int, dtype=torch.int32, device=dev)
        if chi2 is None and want_chi2:
            chi2 = torch.empty(self.n_int, dtype=torch.float64, device=dev)
        self._dev(residual, "residual", torch.complex64, (self.rows, self.n_corr))
        self._dev(n_iter, "n_iter", torch.int32, (self.n_int,))
        self._dev(status, "status", torch.int32, (self.n_int,))
        self._dev(chi2, "chi2", torch.float64, (self.n_int,))
        _check(lib().wcal_solve_static(self._h, _ptr(data), _ptr(model), _ptr(flags), _ptr(gains),
                                       _ptr(residual), _ptr(n_iter), _ptr(status), _ptr(chi2),
                                       self._stream(stream)))
        return dict(gains=gains, residual=residual, n_iter=n_iter, status=status, chi2=chi2)

    def autotune(self, data, model, flags, gains, n_updates: int = 0, stream=None) -> dict:
        """wcal_plan_autotune: time the candidate tilings on these inputs (n_updates updates,
        or whole solves to the plan's tolerance with 0) and keep the fastest."""
        self._inputs(data, model, flags, gains)
        tr, tri = C.c_int32(0), C.c_int32(0)
        n = C.c_size_t(0)
        _check(lib().wcal_plan_autotune_workspace(self._h, C.byref(n)))
        ws = self._alloc(n.value, gains.device)
        _check(lib().wcal_plan_autotune(self._h, _ptr(data), _ptr(model), _ptr(flags), _ptr(gains), n_updates,
                                        _ptr(ws), C.c_size_t(ws.numel()), self._stream(stream), C.byref(tr),
                                        C.byref(tri)))
        del ws
        self.pass_kernel = lib().wcal_plan_pass_kernel(self._h).decode()
        return {"tile_rows": tr.value, "triangle": bool(tri.value), "pass_kernel": self.pass_kernel}

    def solve_graph(self, data, model, flags, gains, residual=None, n_iter=None, status=None,
                    chi2=None, stream=None, want_residual: bool = True, want_chi2: bool = True,
                    workspace=None) -> "Graph":
        """wcal_solve_graph: the solve captured into a replayable HIP graph bound to these
        tensors (kept alive by the returned object)."""
        self._inputs(data, model, flags, gains)
        dev = gains.device
        if residual is None and want_residual:
            residual = torch.empty_like(data)
        if n_iter is None:
            n_iter = torch.empty(self.n_int, dtype=torch.int32, device=dev)
        if status is None:
            status = torch.empty(self.n_int, dtype=torch.int32, device=dev)
        if chi2 is None and want_chi2:
            chi2 = torch.empty(self.n_int, dtype=torch.float64, device=dev)
        self._dev(residual, "residual", torch.complex64, (self.rows, self.n_corr))
        self._dev(n_iter, "n_iter", torch.int32, (self.n_int,))
        self._dev(status, "status", torch.int32, (self.n_int,))
        self._dev(chi2, "chi2", torch.float64, (self.n_int,))
        h = C.c_void_p()
        # the graph holds the workspace's address: a private one, kept alive with the graph
        ws = self._alloc(self.workspace_bytes(), gains.device) if workspace is None else workspace
        _check(lib().wcal_solve_graph(self._h, _ptr(data), _ptr(model), _ptr(flags), _ptr(gains),
                                      _ptr(residual), _ptr(n_iter), _ptr(status), _ptr(chi2),
                                      _ptr(ws), C.c_size_t(ws.numel()), self._stream(stream), C.byref(h)))
        return Graph(h, self, dict(gains=gains, residual=residual, n_iter=n_iter, status=status, chi2=chi2,
                                   data=data, model=model, flags=flags, workspace=ws))

    def accumulate(self, data, model, flags, gains, residual=None, stream=None,
                   want_residual: bool = False, workspace=None):
        """wcal_accumulate: one fused pass at fixed gains."""
        self._inputs(data, model, flags, gains)
        dev = gains.device
        nd, nc, na, ni = self.n_dir, self.n_corr, self.n_ant, self.n_int
        blk = (2 * nd) ** 2 if nc == 4 else nd * nd
        jhj = torch.empty(ni, na, blk, dtype=torch.complex64, device=dev)
        jhd = torch.empty(ni, na, nd * nc, dtype=torch.complex64, device=dev)
        jhr = torch.empty(ni, na, nd * nc, dtype=torch.complex64, device=dev)
        count = torch.empty(ni, na, dtype=torch.int32, device=dev)
        chi2 = torch.empty(ni, dtype=torch.float64, device=dev)
        if residual is None and want_residual:
            residual = torch.empty_like(data)
        self._dev(residual, "residual", torch.complex64, (self.rows, nc))
        wp, wn, _ = self._ws_args(workspace)
        _check(lib().wcal_accumulate(self._h, _ptr(data), _ptr(model), _ptr(flags), _ptr(gains),
                                     _ptr(jhj), _ptr(jhd), _ptr(jhr), _ptr(count), _ptr(chi2),
                                     _ptr(residual), wp, wn, self._stream(stream)))
        return dict(jhj=jhj, jhd=jhd, jhr=jhr, count=count, chi2=chi2, residual=residual)

    def smoothing(self, n_time: int, n_chan: int, sigma_t: float, sigma_f: float):
        """wcal_plan_smoothing: every sample of an interval becomes a cell of an n_time x n_chan
        grid with its own gains, smoothed by a Gaussian of widths sigma_t, sigma_f cells."""
        _check(lib().wcal_plan_smoothing(self._h, int(n_time), int(n_chan), float(sigma_t), float(sigma_f)))
        self.smooth_cells = int(n_time) * int(n_chan)
        self._ws = None

    def solve_smooth(self, data, model, flags, gains, residual=None, n_iter=None, status=None,
                     chi2=None, stream=None, want_residual: bool = True, want_chi2: bool = True, workspace=None):
        """wcal_solve_smooth: gains [n_int][cells][n_ant] (complex64) are updated in place."""
        R = self.rows
        self._dev(data, "data", torch.complex64, (R, 1))
        self._dev(model, "model", torch.complex64, (R, 1, 1))
        if flags is not None:
            self._dev(flags, "flags", torch.uint8, (R,))
        self._dev(gains, "gains", torch.complex64, (self.n_int, self.smooth_cells, self.n_ant))
        dev = gains.device
        if residual is None and want_residual:
            residual = torch.empty_like(data)
        if n_iter is None:
            n_iter = torch.empty(self.n_int, dtype=torch.int32, device=dev)
        if status is None:
            status = torch.empty(self.n_int, dtype=torch.int32, device=dev)
        if chi2 is None and want_chi2:
            chi2 = torch.empty(self.n_int, dtype=torch.float64, device=dev)
        self._dev(residual, "residual", torch.complex64, (R, 1))
        wp, wn, _ = self._ws_args(workspace)
        _check(lib().wcal_solve_smooth(self._h, _ptr(data), _ptr(model), _ptr(flags), _ptr(gains), _ptr(residual),
                                       _ptr(n_iter), _ptr(status), _ptr(chi2), wp, wn, self._stream(stream)))
        return dict(gains=gains, residual=residual, n_iter=n_iter, status=status, chi2=chi2)

    def solve_points(self, n_time: int, n_chan: int, freq0: float, dfreq: float, uvw, lmn, flux, data, flags,
                     gains, residual=None, n_iter=None, status=None, chi2=None, stream=None,
                     want_residual: bool = True, want_chi2: bool = True, workspace=None):
        """wcal_solve_points: the point-source model (uvw [n_int][n_time][n_bl][3] float64,
        lmn [n_dir][3] float64, flux [n_dir] float32, device) predicted in the passes."""
        R = self.rows
        self._dev(data, "data", torch.complex64, (R, 1))
        if flags is not None:
            self._dev(flags, "flags", torch.uint8, (R,))
        self._dev(gains, "gains", torch.complex64, (self.n_int, self.n_dir, self.n_ant, 1))
        self._dev(uvw, "uvw", torch.float64, (self.n_int, n_time, self.n_bl, 3))
        self._dev(lmn, "lmn", torch.float64, (self.n_dir, 3))
        self._dev(flux, "flux", torch.float32, (self.n_dir,))
        dev = gains.device
        if residual is None and want_residual:
            residual = torch.empty_like(data)
        if n_iter is None:
            n_iter = torch.empty(self.n_int, dtype=torch.int32, device=dev)
        if status is None:
            status = torch.empty(self.n_int, dtype=torch.int32, device=dev)
        if chi2 is None and want_chi2:
            chi2 = torch.empty(self.n_int, dtype=torch.float64, device=dev)
        self._dev(residual, "residual", torch.complex64, (R, 1))
        pts = Points(int(n_time), int(n_chan), float(freq0), float(dfreq), _ptr(uvw), _ptr(lmn), _ptr(flux))
        if workspace is None:
            nb = C.c_size_t(0)
            _check(lib().wcal_points_workspace(self._h, C.byref(pts), C.byref(nb)))
            if self._pws is None or self._pws.numel() < nb.value:
                self._pws = None
                self._pws = self._alloc(nb.value, dev)
            workspace = self._pws
        wp, wn, _ = self._ws_args(workspace)
        _check(lib().wcal_solve_points(self._h, C.byref(pts), _ptr(data), _ptr(flags), _ptr(gains), _ptr(residual),
                                       _ptr(n_iter), _ptr(status), _ptr(chi2), wp, wn, self._stream(stream)))
        return dict(gains=gains, residual=residual, n_iter=n_iter, status=status, chi2=chi2)

    def residual(self, data, model, flags, gains, residual=None, stream=None, workspace=None):
        """wcal_residual: R = D - sum_d G_p M G_q^H and chi^2 per interval."""
        self._inputs(data, model, flags, gains)
        if residual is None:
            residual = torch.empty_like(data)
        self._dev(residual, "residual", torch.complex64, (self.rows, self.n_corr))
        chi2 = torch.empty(self.n_int, dtype=torch.float64, device=gains.device)
        wp, wn, _ = self._ws_args(workspace)
        _check(lib().wcal_residual(self._h, _ptr(data), _ptr(model), _ptr(flags), _ptr(gains),
                                   _ptr(residual), _ptr(chi2), wp, wn, self._stream(stream)))
        return dict(residual=residual, chi2=chi2)


class Graph:
    """A captured solve (wraps wcal_graph); `outputs` holds the bound tensors."""

    def __init__(self, h, plan: "Plan", tensors: dict):
        self._h, self.plan, self.outputs = h, plan, tensors

    def launch(self, stream=None):
        _check(lib().wcal_graph_launch(self._h, self.plan._stream(stream)))
        return self.outputs

    def close(self):
        if self._h:
            lib().wcal_graph_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _cur_stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def bin_knots(n_int: int, bin_width: int) -> torch.Tensor:
    """wcal_bin_knots: knot interval of every bin (host int32 tensor)."""
    n_bins = (n_int + bin_width - 1) // bin_width
    k = torch.empty(n_bins, dtype=torch.int32)
    _check(lib().wcal_bin_knots(n_int, bin_width, _ptr(k)))
    return k


def gather_knots(plan: "Plan", bin_width: int, data, model, flags, data_out, model_out, flags_out=None,
                 stream=None):
    """wcal_gather_knots: rows of the knot intervals into the caller's compact buffers."""
    plan._inputs(data, model, flags, torch.empty(plan.n_int, plan.n_dir, plan.n_ant, plan.n_corr,
                                                 dtype=torch.complex64, device=data.device))
    for t in (data_out, model_out, flags_out):
        assert t is None or (t.is_cuda and t.is_contiguous())
    _check(lib().wcal_gather_knots(plan._h, bin_width, _ptr(data), _ptr(model), _ptr(flags), _ptr(data_out),
                                   _ptr(model_out), _ptr(flags_out), _cur_stream(stream)))


def bins_to_gains(y, n_int: int, bin_width: int, stream=None) -> torch.Tensor:
    """wcal_bins_to_gains: knot values [n_ant][2 n_bins] -> gains [n_int][1][n_ant][1]."""
    assert y.is_cuda and y.dtype == torch.float32 and y.is_contiguous()
    n_ant = y.shape[0]
    g = torch.empty(n_int, 1, n_ant, 1, dtype=torch.complex64, device=y.device)
    _check(lib().wcal_bins_to_gains(n_int, n_ant, bin_width, _ptr(y), _ptr(g), _cur_stream(stream)))
    return g


def gains_to_bins(gains, bin_width: int, halfwidth: int = 0, stream=None) -> torch.Tensor:
    """wcal_gains_to_bins: gains [n_int][1][n_ant][1] -> referenced knot-window means [n_ant][2 n_bins]."""
    assert gains.is_cuda and gains.dtype == torch.complex64 and gains.is_contiguous()
    n_int, n_ant = gains.shape[0], gains.shape[2]
    n_bins = (n_int + bin_width - 1) // bin_width
    y = torch.empty(n_ant, 2 * n_bins, dtype=torch.float32, device=gains.device)
    _check(lib().wcal_gains_to_bins(n_int, n_ant, bin_width, halfwidth, _ptr(gains), _ptr(y),
                                    _cur_stream(stream)))
    return y


def reset_unconverged(plan: "Plan", status, gains, stream=None):
    """wcal_reset_unconverged: unit gains for every interval that did not converge."""
    _check(lib().wcal_reset_unconverged(plan._h, _ptr(status), _ptr(gains), _cur_stream(stream)))


class Mlp:
    """The warm-start network (wraps wcal_mlp)."""

    def __init__(self, d_in: int, d_hidden: int, d_out: int, max_batch: int = 4096, skip: bool = False,
                 device: int = 0):
        self._h = C.c_void_p()
        _check(lib().wcal_mlp_create(d_in, d_hidden, d_out, max_batch, int(skip), device, C.byref(self._h)))
        self.skip = skip
        self.d_in, self.d_hidden, self.d_out, self.max_batch = d_in, d_hidden, d_out, max_batch
        self.n_params = int(lib().wcal_mlp_num_params(self._h))
        self.device = torch.device("cuda", device)

    def close(self):
        if self._h:
            lib().wcal_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta: torch.Tensor):
        assert theta.is_cuda and theta.dtype == torch.float32 and theta.numel() == self.n_params
        _check(lib().wcal_mlp_set_params(self._h, _ptr(theta.contiguous()), _cur_stream()))

    def get_params(self) -> torch.Tensor:
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(lib().wcal_mlp_get_params(self._h, _ptr(out), _cur_stream()))
        return out

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.shape[1] == self.d_in
        y = torch.empty(x.shape[0], self.d_out, dtype=torch.float32, device=x.device)
        _check(lib().wcal_mlp_forward(self._h, _ptr(x), x.shape[0], _ptr(y), _cur_stream()))
        return y

    def gradients(self, x, t):
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float64, device=x.device)
        _check(lib().wcal_mlp_gradients(self._h, _ptr(x), _ptr(t), x.shape[0], _ptr(g), _ptr(loss), _cur_stream()))
        return g, loss

    def train_step(self, x, t, lr: float, loss: Optional[torch.Tensor] = None):
        _check(lib().wcal_mlp_train_step(self._h, _ptr(x), _ptr(t), x.shape[0], float(lr), _ptr(loss),
                                         _cur_stream()))

    def save(self, path: str):
        """wcal_mlp_save: JSON header line + float32 parameters and Adam moments (waits for the
        current stream first)."""
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().wcal_mlp_save(self._h, os.fsencode(path)))

    def load(self, path: str):
        """wcal_mlp_load: parameters and Adam state from a weight file of the same shape."""
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().wcal_mlp_load(self._h, os.fsencode(path)))


def plan_for(problem, algo: Optional[str] = None, **kw) -> Plan:
    """Plan for a synthetic ``synth.Problem`` (uses its baseline table and interval sizes)."""
    if algo is None:
        algo = "stefcal" if problem.n_dir == 1 else "cohjones"
    return Plan(problem.n_ant, problem.ant1.cpu(), problem.ant2.cpu(), problem.ns,
                n_dir=problem.n_dir, n_corr=problem.n_corr, algo=algo, **kw)
