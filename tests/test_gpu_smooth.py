"""GPU parity of StefCal with time/frequency smoothing (Sect. 3.4, Eq. JHJ:diag:smooth)
against the CPU oracle, through wcal_plan_smoothing / wcal_solve_smooth.

Gains are per cell (t, nu); comparisons are update by update (lockstep, tol = 0) within
1e-5 relative; a converged solve is checked by replaying the oracle for the GPU's update
count and confirming the stopping decision.  The full-size case (256 antennas, 4096
channels, one 1 x 4096 grid) is checked on sampled channels by the smoothed fixed point:
one oracle update from the GPU's gains, over the rows of the kernel's window, returns them
up to one common phase.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import calib as oc
from paper_1502_06974_amd import synth, wcal
from gains_check import gain_err

pytestmark = pytest.mark.gpu
DEV = "cuda"


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def chunk_problem(n_ant, n_time, n_chan, n_int=2, sigma=0.05, flag_frac=0.05, seed=0):
    """Scalar rows of n_int chunks of n_time x n_chan cells (sample-major, as every plan)."""
    return synth.scalar_di(n_ant, [n_time * n_chan] * n_int, sigma=sigma, flag_frac=flag_frac, seed=seed,
                           device=DEV)


def chunk_plan(P, n_time, n_chan, st, sf, **kw):
    plan = wcal.plan_for(P, algo="stefcal", **kw)
    plan.smoothing(n_time, n_chan, st, sf)
    return plan


def oracle_chunk(P, k, g0, n_time, n_chan, st, sf, **kw):
    iv = P.interval(k)
    nbl = P.n_bl
    cell = np.arange(iv["d"].shape[0]) // nbl
    return oc.stefcal_smooth(iv["d"][:, 0], iv["m"][:, 0, 0], iv["p"], iv["q"], cell, iv["flags"], g0,
                             n_time, n_chan, st, sf, **kw)


def unit_cells(P, ncell):
    return torch.ones(P.n_int, ncell, P.n_ant, dtype=torch.complex64, device=DEV)


# the last two cases have radii ceil(3 sigma) = 75 and 66 cells, above the 64 the LDS-tiled
# convolution takes: they run the one-pass-per-value convolution instead
@pytest.mark.parametrize("n_ant,n_time,n_chan,st,sf", [(12, 3, 8, 1.0, 2.0), (12, 1, 16, 0.0, 3.0),
                                                       (64, 2, 6, 0.7, 1.5), (16, 4, 1, 1.5, 0.0),
                                                       (12, 1, 160, 0.0, 25.0), (12, 150, 1, 22.0, 0.0)])
def test_smooth_lockstep(n_ant, n_time, n_chan, st, sf):
    log(f"[smooth lockstep] n_ant={n_ant} grid={n_time}x{n_chan} sigma=({st},{sf})")
    P = chunk_problem(n_ant, n_time, n_chan, seed=1)
    plan = chunk_plan(P, n_time, n_chan, st, sf, tol=0.0, max_iter=6)
    nc = n_time * n_chan
    out = plan.solve_smooth(P.data, P.model, P.flags, unit_cells(P, nc))
    torch.cuda.synchronize()
    g = out["gains"].cpu().numpy()
    for k in range(P.n_int):
        o = oracle_chunk(P, k, np.ones((nc, n_ant), complex), n_time, n_chan, st, sf, tol=0.0, max_iter=6)
        e = gain_err(g[k], o["g"], 1)
        log(f"  interval {k}: err={e:.2e}")
        assert e <= 1e-5
        assert int(out["n_iter"][k]) == 6 and int(out["status"][k]) == o["status"]
        assert abs(float(out["chi2"][k]) - o["chi2"]) <= 1e-4 * o["chi2"]
        a, b = int(P.row_off[k]), int(P.row_off[k + 1])
        res = out["residual"][a:b, 0].cpu().numpy()
        assert np.abs(res - o["residual"]).max() <= 1e-4 * np.abs(o["residual"]).max()
        assert np.all(res[P.interval(k)["flags"]] == 0)


def test_smooth_stopping_decision():
    """Converged solve: the oracle replayed for the GPU's update count gives the same gains,
    and its own modulo-phase change crosses the tolerance exactly at that update."""
    log("[smooth stop]")
    n_ant, nt, nf, st, sf = 12, 2, 10, 1.0, 2.0
    P = chunk_problem(n_ant, nt, nf, sigma=0.1, seed=2)
    plan = chunk_plan(P, nt, nf, st, sf, tol=1e-6, max_iter=300)
    out = plan.solve_smooth(P.data, P.model, P.flags, unit_cells(P, nt * nf))
    torch.cuda.synchronize()
    g = out["gains"].cpu().numpy()
    for k in range(P.n_int):
        n = int(out["n_iter"][k])
        assert int(out["status"][k]) & oc.CONVERGED
        o = oracle_chunk(P, k, np.ones((nt * nf, n_ant), complex), nt, nf, st, sf, tol=0.0, max_iter=n)
        h = o["history"]
        log(f"  interval {k}: updates {n}, oracle change at the last two {h[-2]:.3e} {h[-1]:.3e}")
        assert gain_err(g[k], o["g"], 1) <= 1e-5
        assert h[-1] < 1e-6 * (1 + 1e-2) and h[-2] >= 1e-6 * (1 - 1e-2)


def test_smooth_delta_kernel_equals_per_cell_solve():
    """sigma = 0 on both axes: every cell is its own StefCal problem, as in a plan whose
    intervals are the cells."""
    log("[smooth delta]")
    n_ant, nt, nf = 20, 2, 5
    P = chunk_problem(n_ant, nt, nf, seed=3)
    plan = chunk_plan(P, nt, nf, 0.0, 0.0, tol=0.0, max_iter=7)
    a = plan.solve_smooth(P.data, P.model, P.flags, unit_cells(P, nt * nf))["gains"]
    cells = wcal.Plan(n_ant, P.ant1.cpu(), P.ant2.cpu(), [1] * (P.n_int * nt * nf), tol=0.0, max_iter=7)
    g = torch.ones(P.n_int * nt * nf, 1, n_ant, 1, dtype=torch.complex64, device=DEV)
    b = cells.solve(P.data, P.model.reshape(-1, 1, 1), P.flags, g)["gains"]
    torch.cuda.synchronize()
    assert gain_err(a.cpu().numpy().ravel(), b.cpu().numpy().ravel(), 1) <= 1e-6


def test_smooth_status_and_flags():
    """An antenna flagged in every cell of a chunk is singular (gain kept bit-for-bit); NaN
    under flags changes no output bit; unflagged NaN stops the chunk before any update."""
    log("[smooth status]")
    n_ant, nt, nf = 12, 2, 6
    P = chunk_problem(n_ant, nt, nf, n_int=3, flag_frac=0.1, seed=4)
    nc = nt * nf
    flags = P.flags.clone()
    a1, a2 = P.ant1.cpu().numpy(), P.ant2.cpu().numpy()
    bad = torch.as_tensor(np.where((a1 == 5) | (a2 == 5))[0], device=DEV)
    for s in range(nc):
        flags[int(P.row_off[0]) + s * P.n_bl + bad] = 1
    flags[int(P.row_off[2]) + 7] = 0          # the row that carries the unflagged NaN
    g0 = unit_cells(P, nc)
    g0[0, :, 5] = 0.75 - 0.5j
    data = P.data.clone()
    data[flags.bool()] = float("nan")
    data[int(P.row_off[2]) + 7, 0] = float("nan")
    clean = P.data.clone()
    clean[int(P.row_off[2]) + 7, 0] = float("nan")
    plan = chunk_plan(P, nt, nf, 1.0, 1.5, tol=1e-6, max_iter=400)
    o1 = plan.solve_smooth(clean, P.model, flags, g0.clone())
    o2 = plan.solve_smooth(data, P.model, flags, g0.clone())
    torch.cuda.synchronize()
    for key in ("gains", "status", "n_iter"):
        assert torch.equal(o1[key], o2[key]), key
    # chi^2 of the stopped interval is NaN on both sides: compare bit patterns
    assert torch.equal(o1["chi2"].view(torch.int64), o2["chi2"].view(torch.int64))
    st = o1["status"].cpu().numpy()
    g = o1["gains"].cpu().numpy()
    assert st[0] & oc.SINGULAR_ANT and not st[0] & oc.NONFINITE
    assert np.array_equal(g[0, :, 5], g0[0, :, 5].cpu().numpy())
    assert st[1] in (oc.CONVERGED, oc.MAXITER)
    assert st[2] == oc.NONFINITE and int(o1["n_iter"][2]) == 0
    assert np.array_equal(g[2], g0[2].cpu().numpy())
    for k in range(2):
        iv = P.interval(k)
        fl = flags[int(P.row_off[k]):int(P.row_off[k + 1])].cpu().numpy() != 0
        cell = np.arange(iv["d"].shape[0]) // P.n_bl
        o = oc.stefcal_smooth(iv["d"][:, 0], iv["m"][:, 0, 0], iv["p"], iv["q"], cell, fl,
                              g0[k].cpu().numpy().astype(complex), nt, nf, 1.0, 1.5, tol=1e-6, max_iter=400)
        assert st[k] == o["status"], (k, st[k], o["status"])


def test_smooth_bandpass_full_size():
    """256 antennas, 4096 channels as one 1 x 4096 grid, smoothing width 4 channels: the
    solve converges, and on sampled channels one oracle update over the rows of the
    kernel's window returns the GPU's gains up to one common phase."""
    log("[smooth bandpass full]")
    P = synth.workload("bandpass_na256", device=DEV)
    nf, sf = P.n_int, 4.0
    plan = wcal.Plan(P.n_ant, P.ant1.cpu(), P.ant2.cpu(), [nf], tol=1e-6, max_iter=1000)
    plan.smoothing(1, nf, 0.0, sf)
    g0 = torch.ones(1, nf, P.n_ant, dtype=torch.complex64, device=DEV)
    out = plan.solve_smooth(P.data, P.model, P.flags, g0, want_residual=False)
    torch.cuda.synchronize()
    st, n = int(out["status"][0]), int(out["n_iter"][0])
    log(f"  status={st} updates={n}")
    assert st & oc.CONVERGED
    g = out["gains"][0].cpu().numpy().astype(np.complex128)
    r = int(np.ceil(3 * sf))
    nbl = P.n_bl
    worst = 0.0
    for c0 in (0, 7, 2048, 4095):
        lo, hi = max(0, c0 - 2 * r), min(nf, c0 + 2 * r + 1)     # cells whose windows reach c0's
        rows = slice(lo * nbl, hi * nbl)
        d = P.data[rows, 0].cpu().numpy().astype(np.complex128)
        m = P.model[rows, 0, 0].cpu().numpy().astype(np.complex128)
        p = np.tile(P.ant1.cpu().numpy(), hi - lo)
        q = np.tile(P.ant2.cpu().numpy(), hi - lo)
        fl = None if P.flags is None else P.flags[rows].cpu().numpy() != 0
        cell = np.repeat(np.arange(hi - lo), nbl)
        o = oc.stefcal_smooth(d, m, p, q, cell, fl, g[lo:hi], 1, hi - lo, 0.0, sf, tol=0.0, max_iter=1,
                              schedule=oc.GN_ONLY)
        j = c0 - lo       # the window of c0 lies inside [lo, hi)
        e = gain_err(oc.align_phase(o["g"][j], g[c0]), g[c0], 1)
        log(f"  channel {c0}: smoothed fixed-point residual {e:.2e}")
        worst = max(worst, e)
    assert worst <= 1e-5
