"""The plan autotuner (wcal_plan_autotune): it picks one of its candidate tilings, leaves
the caller's gains untouched, and the solve with the chosen tiling reaches the same
solution as the default tiling (1e-5 relative, converged; summation orders differ)."""
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
CANDIDATES = {8192, 16384, 32768, 65536, 131072, 262144}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "pol": lambda: synth.pol_di(40, [4, 30, 66, 2], sigma=0.01, flag_frac=0.05, seed=31, device=DEV),
    "triangle": lambda: synth.scalar_di(90, [1, 2, 1, 5], sigma=0.01, flag_frac=0.05, seed=32, device=DEV),
}


@pytest.mark.parametrize("n_updates", [3, 0])
@pytest.mark.parametrize("mode", ["pass", "stats"])
@pytest.mark.parametrize("case", list(CASES))
def test_autotune_picks_a_candidate_and_keeps_the_solution(case, mode, n_updates):
    log(f"[autotune] case={case} mode={mode} n_updates={n_updates}")
    P = CASES[case]()
    ref_plan = wcal.plan_for(P, tol=1e-6, max_iter=200, mode=mode)
    ref = ref_plan.solve(P.data, P.model, P.flags, P.unit_gains())
    plan = wcal.plan_for(P, tol=1e-6, max_iter=200, mode=mode)
    g0 = P.unit_gains()
    before = g0.clone()
    choice = plan.autotune(P.data, P.model, P.flags, g0, n_updates=n_updates)
    torch.cuda.synchronize()
    log(f"  chose {choice}")
    assert choice["tile_rows"] in CANDIDATES
    assert torch.equal(g0, before)
    if case != "triangle" or mode == "stats":
        assert not choice["triangle"]
    out = plan.solve(P.data, P.model, P.flags, P.unit_gains())
    torch.cuda.synchronize()
    assert np.all(out["status"].cpu().numpy() & oc.CONVERGED)
    g, gr = out["gains"].cpu().numpy(), ref["gains"].cpu().numpy()
    for k in range(P.n_int):
        assert gain_err(glue.align(g[k], gr[k], 1), gr[k], P.n_corr) <= 1e-5, k


def test_autotune_dd_and_bad_arguments():
    P = synth.dd_point(12, 3, n_time=2, n_chan=4, n_int=1, seed=33, device=DEV, fov_deg=2.0, disk_diam=2e4)
    plan = wcal.plan_for(P)
    choice = plan.autotune(P.data, P.model, P.flags, P.unit_gains(), n_updates=2)
    assert choice["pass_kernel"] == "dd_gram_dmaf_kernel"
    Q = CASES["pol"]()
    plan_q = wcal.plan_for(Q, max_iter=5)
    with pytest.raises(wcal.WcalError):
        plan_q.autotune(Q.data, Q.model, Q.flags, Q.unit_gains(), n_updates=6)
    with pytest.raises(wcal.WcalError):
        plan_q.autotune(Q.data, Q.model, Q.flags, Q.unit_gains(), n_updates=-1)
