"""The largest arrays the library takes, solved against the oracle.

Plan creation refuses an array whose per-interval LDS working set (per-antenna gains and
per-wavefront accumulators) does not fit a workgroup, with WCAL_ESHAPE.  For each solve
family the largest accepted antenna count is found by probing plan creation (the refusal is
monotone in n_ant), the next one up must be refused, the accumulate entry point runs there,
and a few lockstep updates at the largest one are compared with the oracle (Sect. 2.3 StefCal, Sect. 4 2x2 StefCal, Sect. 3.2
CohJones): the kernels' LDS layouts are then at their fullest."""
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


def accepted(n_ant, **kw):
    a1, a2 = synth.baselines(n_ant)
    try:
        wcal.Plan(n_ant, a1, a2, [1], **kw)
        return True
    except wcal.WcalError as e:
        assert e.code == wcal.ESHAPE, e
        return False


def largest(lo, hi, **kw):
    """Largest n_ant in [lo, hi) that plan creation accepts (lo accepted, hi refused)."""
    assert accepted(lo, **kw) and not accepted(hi, **kw)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if accepted(mid, **kw):
            lo = mid
        else:
            hi = mid
    return lo


def accumulate_runs(plan, P):
    """The one-pass accumulate entry point at the same size (its per-antenna kernels take the
    largest LDS): every output finite, and the chi^2 of the unit-gain residual equal to the
    solve's own residual pass at unit gains."""
    out = plan.accumulate(P.data, P.model, P.flags, P.unit_gains(), want_residual=False)
    res = plan.residual(P.data, P.model, P.flags, P.unit_gains())
    torch.cuda.synchronize()
    for key, v in out.items():
        if torch.is_tensor(v) and (v.is_floating_point() or v.is_complex()):
            assert bool(torch.isfinite(torch.view_as_real(v) if v.is_complex() else v).all()), key
    c1, c2 = out["chi2"].cpu().double(), res["chi2"].cpu().double()
    assert torch.allclose(c1, c2, rtol=1e-6, atol=0.0), (c1, c2)


def lockstep(P, algo, n_upd=3):
    plan = wcal.plan_for(P, algo=algo, tol=0.0, max_iter=n_upd)
    accumulate_runs(wcal.plan_for(P, algo=algo), P)
    out = plan.solve(P.data, P.model, P.flags, P.unit_gains())
    torch.cuda.synchronize()
    g = out["gains"].cpu().numpy()
    for k in range(P.n_int):
        o = glue.solve(P, k, P.unit_gains()[k].cpu().numpy(), algo=algo, tol=0.0, max_iter=n_upd)
        go = glue.gains_from_oracle(o["g"], P.n_corr, P.n_dir)
        e = gain_err(g[k], go, P.n_corr)
        log(f"  interval {k}: {e:.2e}")
        assert e <= 1e-5, (k, e)
        assert int(out["n_iter"][k]) == n_upd
        assert abs(float(out["chi2"][k]) - o["chi2"]) <= 1e-4 * o["chi2"]


@pytest.mark.parametrize("tri", ["1", "0"])
def test_largest_scalar_array(tri, monkeypatch):
    """Scalar StefCal: the triangle pass (fused for the one-sample interval, unfused for the
    three-sample one) and the generic tiled pass."""
    monkeypatch.setenv("WCAL_TRI", tri)
    na = largest(64, 1024)
    log(f"[limits] scalar StefCal: largest n_ant {na}, tri={tri}")
    P = synth.scalar_di(na, [1, 3], sigma=0.01, flag_frac=0.05, seed=41, device=DEV)
    lockstep(P, "stefcal")


def test_largest_pol_array():
    na = largest(16, 1024, n_corr=4)
    log(f"[limits] 2x2 StefCal: largest n_ant {na}")
    P = synth.pol_di(na, [2], sigma=0.01, flag_frac=0.05, seed=42, device=DEV)
    lockstep(P, "stefcal")


def test_largest_cohjones_array():
    """CohJones with 10 directions: the per-antenna solve's LDS (H, c and the gains of every
    antenna and direction) is the limit."""
    na = largest(16, 2048, n_dir=10, algo="cohjones")
    log(f"[limits] CohJones Nd=10: largest n_ant {na}")
    P = synth.dd_point(na, 10, n_time=2, n_chan=2, n_int=1, seed=43, device=DEV, flag_frac=0.05,
                       fov_deg=2.0, disk_diam=2e4)
    lockstep(P, "cohjones", n_upd=2)


def test_largest_pol_cohjones_array():
    """Polarized CohJones with 10 directions (one sample per baseline: the oracle's 2Nd x 2Nd
    solves over ~10^5 baselines take ~10 s)."""
    na = largest(16, 2048, n_dir=10, n_corr=4, algo="cohjones")
    log(f"[limits] polarized CohJones Nd=10: largest n_ant {na}")
    P = synth.pol_dd(na, [1], 10, sigma=0.01, flag_frac=0.05, seed=44, device=DEV)
    lockstep(P, "cohjones", n_upd=2)
