"""Run the CPU oracle on one interval of a synthetic problem (TEST INFRASTRUCTURE ONLY).

Inputs are the same complex64 values the GPU receives, upcast to complex128.
"""
import numpy as np

from . import calib as oc

SCHED = {0: oc.AVG_FIRST, 1: oc.GN_FIRST, 2: oc.GN_ONLY, "avg_first": oc.AVG_FIRST,
         "gn_first": oc.GN_FIRST, "gn_only": oc.GN_ONLY}


def split(iv, n_corr, n_dir):
    """Interval dict -> (d, m) in the oracle's per-kind shapes."""
    if n_dir == 1 and n_corr == 1:
        return iv["d"][:, 0], iv["m"][:, 0, 0]
    if n_corr == 4:
        return iv["d"].reshape(-1, 2, 2), iv["m"][:, 0].reshape(-1, 2, 2)
    return iv["d"][:, 0], iv["m"][:, :, 0]


def gains_to_oracle(g, n_corr, n_dir):
    """[n_dir][n_ant][n_corr] complex -> oracle layout."""
    g = np.asarray(g, dtype=np.complex128)
    if n_dir == 1 and n_corr == 1:
        return g[0, :, 0].copy()
    if n_corr == 4:
        return g[0].reshape(-1, 2, 2).copy()
    return g[:, :, 0].copy()


def gains_from_oracle(g, n_corr, n_dir):
    if n_dir == 1 and n_corr == 1:
        return g[None, :, None]
    if n_corr == 4:
        return g.reshape(1, -1, 4)
    return g[:, :, None]


def solve(problem, k, g0, algo="stefcal", tol=1e-6, max_iter=100, schedule="avg_first", flags=True):
    iv = problem.interval(k)
    d, m = split(iv, problem.n_corr, problem.n_dir)
    fl = iv["flags"] if flags else None
    g0o = gains_to_oracle(g0, problem.n_corr, problem.n_dir)
    s = SCHED[schedule]
    if algo == "stefcal":
        fn = oc.stefcal_scalar if problem.n_corr == 1 else oc.stefcal_2x2
    elif algo == "cohjones":
        fn = oc.cohjones
    else:
        fn = oc.alljones
    return fn(d, m, iv["p"], iv["q"], fl, g0o, tol=tol, max_iter=max_iter, schedule=s)


def accumulate(problem, k, g, flags=True):
    iv = problem.interval(k)
    d, m = split(iv, problem.n_corr, problem.n_dir)
    fl = iv["flags"] if flags else None
    go = gains_to_oracle(g, problem.n_corr, problem.n_dir)
    if problem.n_dir > 1:
        return oc.accumulate_dd(d, m, iv["p"], iv["q"], fl, go)
    if problem.n_corr == 1:
        return oc.accumulate_scalar(d, m, iv["p"], iv["q"], fl, go)
    return oc.accumulate_2x2(d, m, iv["p"], iv["q"], fl, go)


def align(g, ref, n_dir):
    return oc.align_phase_per_direction(g, ref) if n_dir > 1 else oc.align_phase(g, ref)
