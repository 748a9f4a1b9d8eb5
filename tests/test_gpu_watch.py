"""Host watch of the per-update launches (wcal_plan_watch).

A watched solve stops enqueuing update slots once every interval has stopped.  The slots it
leaves out would have found nothing listed, so every output (gains, residual, update counts,
status bits, chi^2) must equal the unwatched solve's bit for bit, while the number of pass
launches (counted by the plan's profiler) drops from max_iter to at most the updates the
slowest interval applies plus the watch depth.  Under stream capture the watch records every
slot, and the graph replays the eager result.  Every solve family with per-update launches
is covered: StefCal scalar (tiled, fused and unfused triangle) and 2x2, CohJones in PASS
and STATS mode, polarized CohJones, the smoothed solve and the predicted-model solve."""
import sys

import pytest
import torch

from paper_1502_06974_amd import synth, wcal

pytestmark = pytest.mark.gpu
DEV = "cuda"
MAX_ITER = 60


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(a, b):
    if a is None or b is None:
        return a is None and b is None
    a, b = a.cpu(), b.cpu()
    return torch.equal(a.view(torch.uint8) if a.is_complex() else a, b.view(torch.uint8) if b.is_complex() else b)


def dd_problem(n_corr=1):
    if n_corr == 4:
        return synth.pol_dd(12, [6, 2, 9], 2, sigma=0.01, flag_frac=0.05, seed=31, device=DEV)
    return synth.dd_point(12, 3, n_time=3, n_chan=4, n_int=3, seed=32, device=DEV, flag_frac=0.05,
                          fov_deg=2.0, disk_diam=2e4)


CASES = {
    "scalar": lambda: synth.scalar_di(30, [3, 10, 1, 7], sigma=0.01, flag_frac=0.1, seed=21, device=DEV),
    "triangle_fused": lambda: synth.scalar_di(80, [1] * 6, sigma=0.05, flag_frac=0.1, seed=22, device=DEV),
    "triangle": lambda: synth.scalar_di(80, [1, 1, 4], sigma=0.01, flag_frac=0.1, seed=22, device=DEV),
    "pol": lambda: synth.pol_di(24, [2, 9, 5], sigma=0.01, flag_frac=0.1, seed=23, device=DEV),
    "cohjones": dd_problem,
    "pol_cohjones": lambda: dd_problem(4),
}


def run(plan, fn, depth, *args):
    plan.watch(depth)
    plan.profile(True)
    out = fn(*args)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    plan.watch(0)
    return {k: (v.clone() if v is not None else None) for k, v in out.items()}, prof


def compare(name, plan, fn, make_args, mode="pass"):
    """The unwatched solve, then watched solves of depth 1, 2 and 5, from the same start."""
    ref, pref = run(plan, fn, 0, *make_args())
    cls = "pass" if mode == "pass" else "solve_stats"
    n_full = pref[cls][1]
    slowest = int(ref["n_iter"].max())
    assert n_full == MAX_ITER
    for depth in (1, 2, 5):
        out, prof = run(plan, fn, depth, *make_args())
        n = prof[cls][1]
        log(f"  {name} depth={depth}: {n} {cls} launches (unwatched {n_full}, slowest interval {slowest} updates)")
        for key in ("gains", "residual", "n_iter", "status", "chi2"):
            assert same(out.get(key), ref.get(key)), (depth, key)
        assert n <= min(MAX_ITER, slowest + depth + 1)


@pytest.mark.parametrize("case", list(CASES))
def test_watched_solve_matches_unwatched(case):
    log(f"[watch] case={case}")
    P = CASES[case]()
    modes = ["pass", "stats"] if case in ("cohjones", "pol_cohjones") else ["pass"]
    for mode in modes:
        plan = wcal.plan_for(P, tol=1e-6, max_iter=MAX_ITER, mode=mode)
        compare(f"{case}/{mode}", plan, plan.solve, lambda: (P.data, P.model, P.flags, P.unit_gains()), mode)


def test_watched_smoothed_solve():
    log("[watch] smoothed solve")
    nt, nf = 2, 6
    P = synth.scalar_di(20, [nt * nf] * 3, sigma=0.05, flag_frac=0.05, seed=33, device=DEV)
    plan = wcal.plan_for(P, algo="stefcal", tol=1e-6, max_iter=MAX_ITER)
    plan.smoothing(nt, nf, 0.7, 1.5)
    cells = lambda: torch.ones(P.n_int, nt * nf, P.n_ant, dtype=torch.complex64, device=DEV)
    compare("smooth", plan, plan.solve_smooth, lambda: (P.data, P.model, P.flags, cells()))


@pytest.mark.parametrize("flag_frac", [0.05, 0.0])
def test_watched_points_solve(flag_frac):
    log(f"[watch] predicted-model solve, flags {flag_frac}")
    P = synth.dd_point(12, 3, n_time=3, n_chan=8, n_int=3, seed=34, device=DEV, flag_frac=flag_frac,
                       fov_deg=2.0, disk_diam=2e4)
    m = P.meta
    pts = dict(n_time=m["n_time"], n_chan=m["n_chan"], freq0=m["freq0"], dfreq=m["dfreq"],
               uvw=m["uvw"].contiguous(), lmn=m["lmn"].to(DEV).contiguous(),
               flux=m["flux"].to(DEV, torch.float32).contiguous())
    plan = wcal.plan_for(P, algo="cohjones", tol=1e-6, max_iter=MAX_ITER)
    fn = lambda data, flags, gains: plan.solve_points(**pts, data=data, flags=flags, gains=gains)
    compare("points", plan, fn, lambda: (P.data, P.flags, P.unit_gains()))


def test_watch_records_every_slot_under_capture():
    """With the watch on, a captured solve still holds all max_iter slots: its replays equal
    the eager watched solve, and the watch is live again for the next eager call."""
    P = CASES["scalar"]()
    plan = wcal.plan_for(P, tol=1e-6, max_iter=MAX_ITER)
    plan.watch(2)
    eager = plan.solve(P.data, P.model, P.flags, P.unit_gains())
    torch.cuda.synchronize()
    eager = {k: (v.clone() if v is not None else None) for k, v in eager.items()}
    gains = P.unit_gains()
    graph = plan.solve_graph(P.data, P.model, P.flags, gains)
    for r in range(2):
        gains.copy_(P.unit_gains())
        out = graph.launch()
        torch.cuda.synchronize()
        for key in ("gains", "residual", "n_iter", "status", "chi2"):
            assert same(out[key], eager[key]), (r, key)
    graph.close()
    plan.profile(True)
    again = plan.solve(P.data, P.model, P.flags, P.unit_gains())
    torch.cuda.synchronize()
    n = plan.profile_read()["pass"][1]
    plan.profile(False)
    assert n < MAX_ITER
    assert same(again["gains"], eager["gains"])
    plan.watch(0)


def test_watch_depth_limits():
    P = CASES["scalar"]()
    plan = wcal.plan_for(P)
    for bad in (-1, 65):
        with pytest.raises(wcal.WcalError):
            plan.watch(bad)
    plan.watch(64)
    plan.watch(0)
    plan.watch(0)
