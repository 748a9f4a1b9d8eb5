"""GPU parity of the CohJones / AllJones solve with point-source models predicted in the
passes (wcal_solve_points, Sect. 3.2.1) against the CPU oracle run on the model of the
definition (oracle.calib.point_model, FP64), and against the solve that reads the same
model from HBM.

The predicted model carries ~1e-6 relative error (FP32 sine/cosine of an FP64-reduced phase,
stepped from channel to channel and re-based at every time slot and every 16 channels), well
inside the 1e-5 bound on gains.  The grids cover time slots shorter than the Gram pass's
four-sample groups (1 and 2 channels), channel counts that are not multiples of four, and a
200-channel slot in which the phasors are re-based inside the slot.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import calib as oc
from oracle import driver as glue
from paper_1502_06974_amd import synth, wcal
from gains_check import gain_err

pytestmark = pytest.mark.gpu
DEV = "cuda"


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def problem(n_ant=12, n_dir=3, n_time=3, n_chan=8, n_int=2, flag_frac=0.05, seed=0, noise=True):
    return synth.dd_point(n_ant, n_dir, n_time=n_time, n_chan=n_chan, n_int=n_int, seed=seed, device=DEV,
                          flag_frac=flag_frac, fov_deg=2.0, disk_diam=2e4, noise=noise)


def points_args(P):
    m = P.meta
    return dict(n_time=m["n_time"], n_chan=m["n_chan"], freq0=m["freq0"], dfreq=m["dfreq"],
                uvw=m["uvw"].contiguous(), lmn=m["lmn"].to(DEV).contiguous(),
                flux=m["flux"].to(DEV, torch.float32).contiguous())


def oracle_model(P, k):
    """The model of the definition for interval k's rows, complex128 [rows, Nd]."""
    m = P.meta
    nt, nf, nbl = m["n_time"], m["n_chan"], P.n_bl
    s = np.arange(nt * nf)
    t, f = np.repeat(s // nf, nbl), np.repeat(s % nf, nbl)
    b = np.tile(np.arange(nbl), nt * nf)
    u = m["uvw"][k].cpu().numpy()[t, b]
    return oc.point_model(u, m["lmn"].cpu().numpy(), m["flux"].cpu().numpy(), m["freq0"] + f * m["dfreq"])


@pytest.mark.parametrize("algo", ["cohjones", "alljones"])
@pytest.mark.parametrize("mode", ["pass", "stats"])
@pytest.mark.parametrize("n_time,n_chan", [(3, 8), (3, 5), (5, 2), (12, 1), (1, 200)])
def test_points_lockstep(algo, mode, n_time, n_chan):
    log(f"[points lockstep] algo={algo} mode={mode} grid={n_time}x{n_chan}")
    P = problem(n_time=n_time, n_chan=n_chan, seed=1)
    plan = wcal.plan_for(P, algo=algo, tol=0.0, max_iter=6, mode=mode)
    out = plan.solve_points(**points_args(P), data=P.data, flags=P.flags, gains=P.unit_gains())
    ref = plan.solve(P.data, P.model, P.flags, P.unit_gains())
    torch.cuda.synchronize()
    g = out["gains"][:, :, :, 0].cpu().numpy()
    gr = ref["gains"][:, :, :, 0].cpu().numpy()
    e_ref = gain_err(g, gr, 1)
    log(f"  vs model read from HBM: {e_ref:.2e}")
    assert e_ref <= 1e-5
    fn = oc.cohjones if algo == "cohjones" else oc.alljones
    for k in range(P.n_int):
        iv = P.interval(k)
        o = fn(iv["d"][:, 0], oracle_model(P, k), iv["p"], iv["q"], iv["flags"], np.ones((P.n_dir, P.n_ant), complex),
               tol=0.0, max_iter=6)
        e = gain_err(g[k], o["g"], 1)
        log(f"  interval {k}: vs oracle {e:.2e}")
        assert e <= 1e-5
        assert int(out["n_iter"][k]) == 6 and int(out["status"][k]) == o["status"]
        assert abs(float(out["chi2"][k]) - o["chi2"]) <= 1e-4 * o["chi2"]
        a, b = int(P.row_off[k]), int(P.row_off[k + 1])
        res = out["residual"][a:b, 0].cpu().numpy()
        assert np.abs(res - o["residual"]).max() <= 1e-4 * np.abs(o["residual"]).max()
        assert np.all(res[iv["flags"]] == 0)


@pytest.mark.parametrize("algo", ["cohjones", "alljones"])
@pytest.mark.parametrize("n_dir,n_time,n_chan", [(3, 3, 5), (3, 5, 13), (3, 1, 200), (14, 8, 17)])
def test_points_unflagged_lockstep(algo, n_dir, n_time, n_chan):
    """Without flags the pass takes the predicted phasor itself as the MFMA operand (no weight
    product).  Sample counts 15, 65, 200 and 136 per interval: partial last groups of 3 and 1
    samples, whose absent samples must add nothing, a second chunk of a single sample, four
    64-channel table segments, and 14 model lanes with the data lane at column 14 (the oracle's
    gains move by under 3e-7 there when only its model is rounded to FP32).  At 6 x 17 samples
    and this seed the 14-direction problem is too weakly determined for the bound: there the
    solve that reads the model from HBM, whose kernel is not this one, lands 8.6e-6 from the
    oracle, and FP32 rounding alone moves the predicted-model gains between 8e-6 and 1.4e-5.  Six updates against the oracle on the model of the
    definition, and against the solve that reads the same model from HBM."""
    log(f"[points unflagged lockstep] algo={algo} nd={n_dir} grid={n_time}x{n_chan}")
    P = problem(n_ant=16 if n_dir > 3 else 12, n_dir=n_dir, n_time=n_time, n_chan=n_chan, seed=3, flag_frac=0.0)
    assert P.flags is None
    plan = wcal.plan_for(P, algo=algo, tol=0.0, max_iter=6)
    out = plan.solve_points(**points_args(P), data=P.data, flags=None, gains=P.unit_gains())
    ref = plan.solve(P.data, P.model, None, P.unit_gains())
    torch.cuda.synchronize()
    g = out["gains"][:, :, :, 0].cpu().numpy()
    e_ref = gain_err(g, ref["gains"][:, :, :, 0].cpu().numpy(), 1)
    log(f"  vs model read from HBM: {e_ref:.2e}")
    assert e_ref <= 1e-5
    fn = oc.cohjones if algo == "cohjones" else oc.alljones
    for k in range(P.n_int):
        iv = P.interval(k)
        o = fn(iv["d"][:, 0], oracle_model(P, k), iv["p"], iv["q"], iv["flags"],
               np.ones((P.n_dir, P.n_ant), complex), tol=0.0, max_iter=6)
        e = gain_err(g[k], o["g"], 1)
        log(f"  interval {k}: vs oracle {e:.2e}")
        assert e <= 1e-5
        assert abs(float(out["chi2"][k]) - o["chi2"]) <= 1e-4 * o["chi2"]


def test_points_most_directions_lockstep():
    """14 point sources, the most the library takes: 14 model lanes, the data lane at column 14,
    one padding lane.  Six updates on both sides against the oracle on the model of the
    definition, and against the solve that reads the same model from HBM.

    The problem has 6 x 16 samples per interval: with 14 directions on 16 antennas, 3 x 8
    samples leave the gains so weakly determined that the oracle's own gains move by 2e-6
    (and, at 32 antennas, 1e-5) when only the model is rounded to FP32, so no FP32 input could
    meet the bound there.  The oracle's sensitivity to that rounding is checked first."""
    log("[points most directions] nd=14")
    P = problem(n_dir=14, n_ant=16, n_time=6, n_chan=16, seed=5)
    plan = wcal.plan_for(P, algo="cohjones", tol=0.0, max_iter=6)
    out = plan.solve_points(**points_args(P), data=P.data, flags=P.flags, gains=P.unit_gains())
    ref = plan.solve(P.data, P.model, P.flags, P.unit_gains())
    torch.cuda.synchronize()
    g = out["gains"][:, :, :, 0].cpu().numpy()
    e_ref = gain_err(g, ref["gains"][:, :, :, 0].cpu().numpy(), 1)
    log(f"  vs model read from HBM: {e_ref:.2e}")
    assert e_ref <= 1e-5
    for k in range(P.n_int):
        iv = P.interval(k)
        m = oracle_model(P, k)
        g0 = np.ones((P.n_dir, P.n_ant), complex)
        o = oc.cohjones(iv["d"][:, 0], m, iv["p"], iv["q"], iv["flags"], g0, tol=0.0, max_iter=6)
        o32 = oc.cohjones(iv["d"][:, 0], m.astype(np.complex64).astype(complex), iv["p"], iv["q"], iv["flags"],
                          g0, tol=0.0, max_iter=6)
        sens = gain_err(o32["g"], o["g"], 1)
        e = gain_err(g[k], o["g"], 1)
        log(f"  interval {k}: vs oracle {e:.2e} (oracle with the model rounded to FP32: {sens:.2e})")
        assert sens <= 1e-6
        assert e <= 1e-5
        assert abs(float(out["chi2"][k]) - o["chi2"]) <= 1e-4 * o["chi2"]


def test_points_na64_full_size():
    """cohjones_na64 at full size (30 x 64 samples per interval): the predicted-model solve
    reaches the same solution as the solve that reads the model, and noise-free gains."""
    log("[points na64 full]")
    P = synth.workload("cohjones_na64", device=DEV, n_int=2)
    plan = wcal.plan_for(P, algo="cohjones", tol=1e-6, max_iter=300)
    out = plan.solve_points(**points_args(P), data=P.data, flags=P.flags, gains=P.unit_gains(),
                            want_residual=False)
    ref = plan.solve(P.data, P.model, P.flags, P.unit_gains(), want_residual=False)
    torch.cuda.synchronize()
    assert torch.all(out["status"] & oc.CONVERGED)
    for k in range(P.n_int):
        g = out["gains"][k, :, :, 0].cpu().numpy()
        gr = ref["gains"][k, :, :, 0].cpu().numpy()
        e = gain_err(glue.align(g, gr, P.n_dir), gr, 1)
        log(f"  interval {k}: updates {int(out['n_iter'][k])} (read: {int(ref['n_iter'][k])}), vs read model {e:.2e}")
        assert e <= 1e-5
    Q = synth.workload("cohjones_na64", device=DEV, n_int=1, noise=False)
    plan_q = wcal.plan_for(Q, algo="cohjones", tol=1e-7, max_iter=500)
    out = plan_q.solve_points(**points_args(Q), data=Q.data, flags=Q.flags, gains=Q.unit_gains(),
                              want_residual=False)
    torch.cuda.synchronize()
    g = out["gains"][0, :, :, 0].cpu().numpy()
    gt = Q.g_true[0, :, :, 0].cpu().numpy()
    e = gain_err(glue.align(g, gt, Q.n_dir), gt, 1)
    log(f"  noise-free recovery err={e:.2e} iters={int(out['n_iter'][0])}")
    assert e <= 1e-5


@pytest.mark.parametrize("mode", ["pass", "stats"])
def test_points_garbage_under_flags_is_bit_identical(mode):
    """NaN in the data under flags leaves every output of the predicted-model solve
    bit-identical: a flagged sample enters the pass as a zeroed value with weight 0."""
    log(f"[points garbage under flags] mode={mode}")
    P = problem(n_time=3, n_chan=13, n_int=3, flag_frac=0.1, seed=9)
    plan = wcal.plan_for(P, algo="cohjones", tol=1e-6, max_iter=60, mode=mode)
    clean = plan.solve_points(**points_args(P), data=P.data, flags=P.flags, gains=P.unit_gains())
    clean = {k: (v.clone() if v is not None else None) for k, v in clean.items()}
    d2 = P.data.clone()
    d2[P.flags.bool()] = float("nan")
    dirty = plan.solve_points(**points_args(P), data=d2, flags=P.flags, gains=P.unit_gains())
    torch.cuda.synchronize()
    for key in ("gains", "residual", "n_iter", "status", "chi2"):
        x, y = clean[key].cpu(), dirty[key].cpu()
        assert torch.equal(x.view(torch.uint8) if x.is_complex() else x,
                           y.view(torch.uint8) if y.is_complex() else y), key


def test_points_rejects_bad_grids():
    P = problem(seed=2)
    plan = wcal.plan_for(P, algo="cohjones")
    args = points_args(P)
    args["n_chan"] = 7
    with pytest.raises(wcal.WcalError):
        plan.solve_points(**args, data=P.data, flags=P.flags, gains=P.unit_gains())
    plan2 = wcal.plan_for(P, algo="cohjones", precision="bf16")
    with pytest.raises(wcal.WcalError):
        plan2.solve_points(**points_args(P), data=P.data, flags=P.flags, gains=P.unit_gains())


def test_points_workspace_holds_the_phasor_table():
    """wcal_points_workspace is the plan's workspace plus the phasor table (40 B per slot,
    baseline and direction at up to 64 channels, 8 B more per 64 channels beyond); a
    workspace one byte short is refused before anything is launched, and the call with
    the exact size solves like the default one."""
    import ctypes as C
    P = problem(n_time=3, n_chan=8, seed=9)
    plan = wcal.plan_for(P, algo="cohjones", tol=1e-6, max_iter=30)
    a = points_args(P)
    pts = wcal.Points(a["n_time"], a["n_chan"], a["freq0"], a["dfreq"], a["uvw"].data_ptr(),
                      a["lmn"].data_ptr(), a["flux"].data_ptr())
    n = C.c_size_t(0)
    assert wcal.lib().wcal_points_workspace(plan._h, C.byref(pts), C.byref(n)) == wcal.OK
    base = -(-plan.workspace_bytes() // wcal.WS_ALIGN) * wcal.WS_ALIGN
    per = P.n_int * a["n_time"] * P.n_bl * P.n_dir
    table = -(-per * 32 // wcal.WS_ALIGN) * wcal.WS_ALIGN + -(-per * 8 // wcal.WS_ALIGN) * wcal.WS_ALIGN
    assert n.value == base + table, (n.value, base, table)
    log(f"[points workspace] plan {plan.workspace_bytes()} B, with the table {n.value} B")
    ws = torch.empty(n.value, dtype=torch.uint8, device=DEV)
    status = torch.full((P.n_int,), 77, dtype=torch.int32, device=DEV)
    with pytest.raises(wcal.WcalError) as ei:
        plan.solve_points(**a, data=P.data, flags=P.flags, gains=P.unit_gains(), status=status,
                          workspace=ws[:n.value - 1])
    assert ei.value.code == wcal.ENOMEM
    torch.cuda.synchronize()
    assert torch.all(status == 77)
    out = plan.solve_points(**a, data=P.data, flags=P.flags, gains=P.unit_gains(), workspace=ws)
    ref = plan.solve_points(**a, data=P.data, flags=P.flags, gains=P.unit_gains())
    torch.cuda.synchronize()
    for key in ("gains", "n_iter", "status", "chi2", "residual"):
        assert torch.equal(out[key], ref[key]), key
