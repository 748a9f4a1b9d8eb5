"""A solve captured into a HIP graph (wcal_solve_graph) replays exactly the eager solve.

Every case replays the graph three times, resetting the gains and running unrelated eager
work and host synchronisations between replays, and compares every output of every replay
with the eager solve bit for bit (the kernels' reductions run in a fixed order, so a
replay computes exactly what the eager call computes)."""
import sys

import pytest
import torch

from paper_1502_06974_amd import synth, wcal

pytestmark = pytest.mark.gpu
DEV = "cuda"


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(a, b):
    if a is None or b is None:
        return a is None and b is None
    a, b = a.cpu(), b.cpu()
    return torch.equal(a.view(torch.uint8) if a.is_complex() else a, b.view(torch.uint8) if b.is_complex() else b)


CASES = {
    "scalar": lambda: synth.scalar_di(30, [3, 10, 1], sigma=0.01, flag_frac=0.1, seed=21, device=DEV),
    "triangle": lambda: synth.scalar_di(80, [1, 1, 4], sigma=0.01, flag_frac=0.1, seed=22, device=DEV),
    # from 127 antennas on the triangle pass walks packed rows
    "triangle_paired": lambda: synth.scalar_di(130, [1, 1, 4], sigma=0.01, flag_frac=0.1, seed=23, device=DEV),
    "pol": lambda: synth.pol_di(24, [2, 9, 5], sigma=0.01, flag_frac=0.1, seed=23, device=DEV),
    "cohjones": lambda: synth.dd_point(12, 3, n_time=3, n_chan=4, n_int=2, seed=24, device=DEV, flag_frac=0.05,
                                       fov_deg=2.0, disk_diam=2e4),
}


@pytest.mark.parametrize("mode", ["pass", "stats"])
@pytest.mark.parametrize("case", list(CASES))
def test_graph_replays_match_eager(case, mode):
    log(f"[graph] case={case} mode={mode}")
    P = CASES[case]()
    plan = wcal.plan_for(P, tol=1e-6, max_iter=60, mode=mode)
    eager = plan.solve(P.data, P.model, P.flags, P.unit_gains())
    torch.cuda.synchronize()
    eager = {k: (v.clone() if v is not None else None) for k, v in eager.items()}
    gains = P.unit_gains()
    graph = plan.solve_graph(P.data, P.model, P.flags, gains)
    junk = torch.randn(1 << 20, device=DEV)
    for r in range(3):
        gains.copy_(P.unit_gains())
        out = graph.launch()
        torch.cuda.synchronize()
        for key in ("gains", "residual", "n_iter", "status", "chi2"):
            assert same(out[key], eager[key]), (r, key)
        junk.mul_(1.0001).add_(0.5)            # unrelated eager work between replays
        torch.cuda.synchronize()
    graph.close()


def test_graph_rejects_capture_while_profiling():
    P = CASES["scalar"]()
    plan = wcal.plan_for(P)
    plan.profile(True)
    with pytest.raises(wcal.WcalError):
        plan.solve_graph(P.data, P.model, P.flags, P.unit_gains())
    plan.profile(False)
