"""Run the CPU oracle on one interval of a synthetic problem (TEST INFRASTRUCTURE ONLY).

Inputs are the same complex64 values the GPU receives, upcast to complex128.
"""
import numpy as np

from . import calib as oc

SCHED = {0: oc.AVG_FIRST, 1: oc.GN_FIRST, 2: oc.GN_ONLY, "avg_first": oc.AVG_FIRST,
         "gn_first": oc.GN_FIRST, "gn_only": oc.GN_ONLY}


def _dd(n_dir, algo):
    return n_dir > 1 or algo in ("cohjones", "alljones")


def split(iv, n_corr, n_dir, algo=None):
    """Interval dict -> (d, m) in the oracle's per-kind shapes."""
    if n_corr == 4:
        D = iv["d"].reshape(-1, 2, 2)
        if _dd(n_dir, algo):
            return D, iv["m"].reshape(-1, n_dir, 2, 2)
        return D, iv["m"][:, 0].reshape(-1, 2, 2)
    if n_dir == 1 and not _dd(n_dir, algo):
        return iv["d"][:, 0], iv["m"][:, 0, 0]
    return iv["d"][:, 0], iv["m"][:, :, 0]


def gains_to_oracle(g, n_corr, n_dir, algo=None):
    """[n_dir][n_ant][n_corr] complex -> oracle layout."""
    g = np.asarray(g, dtype=np.complex128)
    if n_corr == 4:
        if _dd(n_dir, algo):
            return g.reshape(n_dir, -1, 2, 2).copy()
        return g[0].reshape(-1, 2, 2).copy()
    if n_dir == 1 and not _dd(n_dir, algo):
        return g[0, :, 0].copy()
    return g[:, :, 0].copy()


def gains_from_oracle(g, n_corr, n_dir, algo=None):
    if n_corr == 4:
        if _dd(n_dir, algo):
            return g.reshape(n_dir, -1, 4)
        return g.reshape(1, -1, 4)
    if n_dir == 1 and not _dd(n_dir, algo):
        return g[None, :, None]
    return g[:, :, None]


def _solver(algo, nc):
    if algo == "stefcal":
        return oc.stefcal_scalar if nc == 1 else oc.stefcal_2x2
    if algo == "cohjones":
        return oc.cohjones if nc == 1 else oc.cohjones_2x2
    return oc.alljones if nc == 1 else oc.alljones_2x2


def solve(problem, k, g0, algo="stefcal", tol=1e-6, max_iter=100, schedule="avg_first", flags=True):
    iv = problem.interval(k)
    nc, nd = problem.n_corr, problem.n_dir
    d, m = split(iv, nc, nd, algo)
    fl = iv["flags"] if flags else None
    g0o = gains_to_oracle(g0, nc, nd, algo)
    return _solver(algo, nc)(d, m, iv["p"], iv["q"], fl, g0o, tol=tol, max_iter=max_iter, schedule=SCHED[schedule])


def worker_ready(i):
    """A no-op for starting a process pool before timing it."""
    return i


def solve_arrays(job):
    """One interval (or the leading rows of one) solved from host arrays alone, for a pool of
    worker processes: job = (iv, n_corr, n_dir, g0, algo, tol, max_iter) with iv holding d, m,
    p, q and flags as Problem.interval gives them.  Returns (rows x updates, seconds)."""
    import time
    iv, nc, nd, g0, algo, tol, max_iter = job
    d, m = split(iv, nc, nd, algo)
    g0o = gains_to_oracle(g0, nc, nd, algo)
    t0 = time.perf_counter()
    o = _solver(algo, nc)(d, m, iv["p"], iv["q"], iv["flags"], g0o, tol=tol, max_iter=max_iter,
                          schedule=oc.AVG_FIRST)
    return d.shape[0] * o["n_iter"], time.perf_counter() - t0


def accumulate(problem, k, g, flags=True, algo=None):
    iv = problem.interval(k)
    nc, nd = problem.n_corr, problem.n_dir
    d, m = split(iv, nc, nd, algo)
    fl = iv["flags"] if flags else None
    go = gains_to_oracle(g, nc, nd, algo)
    if _dd(nd, algo):
        fn = oc.accumulate_dd if nc == 1 else oc.accumulate_dd_2x2
        return fn(d, m, iv["p"], iv["q"], fl, go)
    if nc == 1:
        return oc.accumulate_scalar(d, m, iv["p"], iv["q"], fl, go)
    return oc.accumulate_2x2(d, m, iv["p"], iv["q"], fl, go)


def residual(problem, k, g, flags=True, algo=None):
    """R and chi^2 of interval k at gains g ([n_dir][n_ant][n_corr])."""
    iv = problem.interval(k)
    nc, nd = problem.n_corr, problem.n_dir
    d, m = split(iv, nc, nd, algo)
    fl = iv["flags"] if flags else None
    go = gains_to_oracle(g, nc, nd, algo)
    if _dd(nd, algo):
        fn = oc.residual_dd if nc == 1 else oc.residual_dd_2x2
    else:
        fn = oc.residual_scalar if nc == 1 else oc.residual_2x2
    return fn(d, m, iv["p"], iv["q"], fl, go)


def align(g, ref, n_dir):
    return oc.align_phase_per_direction(g, ref) if n_dir > 1 else oc.align_phase(g, ref)
