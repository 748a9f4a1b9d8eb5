"""Benchmark of the calibration hot path on one MI355X.

A step is one complete batched solve of the workload: every interval from unit gains to
the 1e-6 relative-change tolerance (per-sample J^H J / J^H D passes, per-antenna solves,
schedule, convergence test) followed by the residual / chi^2 pass, all in one launch.

  value        = sum_k rows_k * n_iter_k / step time   (visibility-iterations per second)
  solve_time   = wall time of one step (inputs resident in HBM)
  roofline     = algorithmic HBM bytes of the solve launch / its duration (HIP events on the
                 launch stream) against the 8 TB/s HBM peak
  cpu_baseline = the CPU oracle on a bounded sample of the same workload (host cores)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "visibility-iterations/s (JHJ+JHr+residual) and solve time to 1e-6 rel. tol."
HBM_PEAK_GBS = 8000.0
MFMA_FP32_PEAK_TFS = 157.3     # dense FP32 matrix peak of one MI355X
MFMA_BF16_PEAK_TFS = 2500.0    # dense BF16 matrix peak of one MI355X


def gram_flop_per_row(n_corr: int, n_dir: int) -> float:
    """Algorithmic flops of the Gram pass per row: the Hermitian model block (complex HERK,
    4 n^2 per sample for n model columns) and the model-data block (complex GEMM, 8 flops
    per complex product): n = Nd, one data column (scalar); n = 4 Nd, four (2x2)."""
    n_m, n_d = n_dir * n_corr, n_corr
    return 4.0 * n_m * n_m + 8.0 * n_m * n_d


def unit_gram_flop_per_row(n_corr: int, n_dir: int) -> float:
    """Algorithmic Gram flops per visibility row as the per-unit figure of the roofline: for
    scalar CohJones the per-antenna Nd x Nd Hermitian block (Eq. JHJ:DD:unpol) on both antennas
    of the row, unique entries only, 8 flops per complex product: 8 Nd (Nd + 1) (880 at Nd = 10).
    The polarized Gram has no such figure; it keeps the pass's own count (gram_flop_per_row)."""
    if n_corr == 1:
        return 8.0 * n_dir * (n_dir + 1)
    return gram_flop_per_row(n_corr, n_dir)


def gram_issued_flop_per_row(n_corr: int, n_dir: int) -> float:
    """Flops the MFMAs issue per row: per 4 samples three 16x16x4 MFMAs per diagonal
    16-column tile and three per off-diagonal tile pair (Gauss's complex product; the BF16
    pass issues the same per 16 samples with 16x16x16 MFMAs)."""
    nt = 1 if n_corr == 1 else (4 * n_dir + 4 + 15) // 16
    return (3 * nt + 3 * nt * (nt - 1) // 2) * 2 * 16 * 16 * 4 / 4


KERNEL_SOURCES = {
    "di": ("di_kernels.hip", "di_common.h"),
    "dd": ("dd_kernels.hip", "dd_common.h", "di_common.h"),
    "ddp": ("ddp_kernels.hip", "dd_common.h", "di_common.h"),
}


def _code_only(text: str) -> str:
    """C / C++ source without its comments (string literals kept), so that edits to comments
    alone leave a kernel family's hash unchanged."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"':
            j = i + 1
            while j < n and text[j] != '"':
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return "".join(out)


# update slots an eager solve keeps enqueued past the last convergence count it has read
WATCH_DEPTH = 2


def source_hash(family: str) -> str:
    """sha256 of what decides a kernel family's memory traffic: its kernel sources, the plan
    and launch code, and the public header, comments removed."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1502_06974_amd", "csrc")
    files = [os.path.join(csrc, f) for f in KERNEL_SOURCES[family] + ("wcal_internal.h", "wcal_api.hip")]
    files.append(os.path.join(ROOT, "include", "wcal.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(_code_only(open(f, encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(key: str, default_solve: bool = True):
    """HBM bytes per launch from the committed counter runs, if the sources are unchanged.

    The counter runs solve each workload with its default settings (tolerance 1e-6, no update cap,
    no smoothing, the default host watch); a run with other settings has other launches (a fixed
    number of full passes, the smoothed solve's passes over the whole grid, or the empty slots an
    unwatched solve launches), so no record applies to it."""
    if not default_solve:
        return None
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "pmc_traffic.json")))[key]
    except (OSError, KeyError, ValueError):
        return None
    family = key.split("_", 1)[0]
    try:
        sha = source_hash(family)
    except OSError:    # sources not shipped: the record cannot be matched to this build
        return None
    return rec["traffic_bytes_per_launch"] if rec.get("src_sha") == sha else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu() -> dict:
    """The host's CPU model (from /proc/cpuinfo) and the logical CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def bytes_per_row(n_corr: int, n_dir: int, flags: bool) -> int:
    return 8 * n_corr + 8 * n_corr * n_dir + (1 if flags else 0)


def cpu_baseline_dd(P, budget_s: float = 15.0):
    """CPU oracle CohJones on the first samples of one interval (the oracle forms every
    row's Nd x Nd (2x2: 2Nd x 2Nd) product in complex128, so whole 1920-sample intervals
    do not fit)."""
    import numpy as np
    from oracle import calib as oc
    from oracle import driver as glue
    ns_take = 32 if P.n_corr == 1 else 8
    iv = P.interval(0)
    nsel = ns_take * P.n_bl
    d, m = glue.split(iv, P.n_corr, P.n_dir, "cohjones")
    d, m = d[:nsel], m[:nsel]
    p, q, fl = iv["p"][:nsel], iv["q"][:nsel], iv["flags"][:nsel]
    g0 = glue.gains_to_oracle(P.unit_gains()[0].cpu().numpy(), P.n_corr, P.n_dir, "cohjones")
    fn = oc.cohjones if P.n_corr == 1 else oc.cohjones_2x2
    t0 = time.perf_counter()
    o = fn(d, m, p, q, fl, g0, tol=1e-6, max_iter=100)
    dt = time.perf_counter() - t0
    return dict(value=nsel * o["n_iter"] / dt, unit="vis-iter/s", cores=1, kind="oracle",
                sample=f"{'' if P.n_corr == 1 else '2x2 '}CohJones on the first {ns_take} samples x "
                       f"{P.n_bl} baselines of one interval, {P.n_dir} directions, unit start, tol 1e-6, "
                       f"{o['n_iter']} updates, one process",
                seconds=round(dt, 2))


def cpu_baseline_smooth(P, smooth, n_chan: int = 16):
    """CPU oracle StefCal with smoothing on the first n_chan cells of the 1 x n_int grid."""
    import numpy as np
    from oracle import calib as oc
    nbl = P.n_bl
    rows = slice(0, n_chan * nbl)
    d = P.data[rows, 0].cpu().numpy().astype(np.complex128)
    m = P.model[rows, 0, 0].cpu().numpy().astype(np.complex128)
    p = np.tile(P.ant1.cpu().numpy(), n_chan)
    q = np.tile(P.ant2.cpu().numpy(), n_chan)
    fl = None if P.flags is None else P.flags[rows].cpu().numpy() != 0
    cell = np.repeat(np.arange(n_chan), nbl)
    t0 = time.perf_counter()
    o = oc.stefcal_smooth(d, m, p, q, cell, fl, np.ones((n_chan, P.n_ant), complex), 1, n_chan, smooth[0],
                          smooth[1], tol=1e-6, max_iter=100)
    dt = time.perf_counter() - t0
    return dict(value=n_chan * nbl * o["n_iter"] / dt, unit="vis-iter/s", cores=1, kind="oracle",
                sample=f"StefCal with smoothing on the first {n_chan} channels x {nbl} baselines of the grid, "
                       f"unit start, tol 1e-6, {o['n_iter']} updates, one process",
                seconds=round(dt, 2))


def cpu_baseline(P, budget_s: float = 15.0):
    """Time the CPU oracle (as it stands) on whole intervals of the workload until about
    budget_s seconds of CPU work; report visibility-iterations per second."""
    import numpy as np
    from oracle import driver as glue
    if P.n_dir > 1:
        return cpu_baseline_dd(P, budget_s)
    rng = np.random.default_rng(0)
    order = rng.permutation(P.n_int)
    vis_it = 0
    t_used = 0.0
    used = []
    for k in order:
        iv_rows = int(P.row_off[k + 1] - P.row_off[k])
        g0 = P.unit_gains()[k].cpu().numpy()
        t0 = time.perf_counter()
        o = glue.solve(P, int(k), g0, tol=1e-6, max_iter=100)
        dt = time.perf_counter() - t0
        vis_it += iv_rows * o["n_iter"]
        t_used += dt
        used.append(int(k))
        if t_used > budget_s:
            break
    return dict(value=vis_it / t_used, unit="vis-iter/s", cores=1, kind="oracle",
                sample=f"{len(used)} whole intervals ({sum(int(P.ns[k]) for k in used)} samples x "
                       f"{P.n_bl} baselines) of the same workload, unit start, tol 1e-6, "
                       f"one process (numpy bincount scatter, single-threaded)",
                seconds=round(t_used, 2))


def _host_rows(P, k: int, nrows):
    """The first nrows rows of interval k (all if None) as host complex128 arrays, in the
    layout of Problem.interval."""
    import numpy as np
    a = int(P.row_off[k])
    n = int(P.row_off[k + 1]) - a if nrows is None else nrows
    ns = (n + P.n_bl - 1) // P.n_bl
    a1 = P.ant1.cpu().numpy().astype(np.int64)
    a2 = P.ant2.cpu().numpy().astype(np.int64)
    return dict(d=P.data[a:a + n].cpu().numpy().astype(np.complex128),
                m=P.model[a:a + n].cpu().numpy().astype(np.complex128),
                p=np.tile(a1, ns)[:n], q=np.tile(a2, ns)[:n],
                flags=(np.zeros(n, dtype=bool) if P.flags is None else P.flags[a:a + n].cpu().numpy() != 0))


def cpu_baseline_all_cores(P, budget_s: float = 15.0):
    """The same oracle, interval-parallel over the host cores (at most 16 worker processes, the
    CPU share of one GPU; one BLAS thread each): whole intervals for StefCal, the first 32
    samples of every interval for CohJones (8 for 2x2), one job per worker in flight, new jobs
    dispatched for budget_s seconds; the jobs then running finish.  The figure is the summed
    visibility-iterations over the wall time of the pool."""
    import multiprocessing as mp
    from concurrent.futures import FIRST_COMPLETED, ProcessPoolExecutor, wait
    import numpy as np
    from oracle import driver as glue
    workers = max(1, min(16, os.cpu_count() or 1))
    dd = P.n_dir > 1
    algo = "cohjones" if dd else "stefcal"
    nsel = (32 if P.n_corr == 1 else 8) * P.n_bl if dd else None
    order = iter(np.random.default_rng(0).permutation(P.n_int).tolist())
    g0 = P.unit_gains().cpu().numpy()
    saved = {v: os.environ.get(v) for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for v in saved:
        os.environ[v] = "1"
    vis, n_done, busy = 0, 0, 0.0
    try:
        with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            list(ex.map(glue.worker_ready, range(2 * workers)))
            t0 = time.perf_counter()
            pending = set()

            def submit():
                k = next(order, None)
                if k is not None:
                    job = (_host_rows(P, k, nsel), P.n_corr, P.n_dir, g0[k], algo, 1e-6, 100)
                    pending.add(ex.submit(glue.solve_arrays, job))

            for _ in range(workers):
                submit()
            while pending:
                done, pending = wait(pending, return_when=FIRST_COMPLETED)
                for f in done:
                    v, dt = f.result()
                    vis += v
                    busy += dt
                    n_done += 1
                    if time.perf_counter() - t0 < budget_s:
                        submit()
            wall = time.perf_counter() - t0
    finally:
        for v, x in saved.items():
            if x is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = x
    what = (f"the first {nsel // P.n_bl} samples of {n_done} intervals" if dd else f"{n_done} whole intervals")
    return dict(value=vis / wall, unit="vis-iter/s", cores=workers, kind="oracle",
                sample=f"{what} of the same workload, unit start, tol 1e-6, {workers} worker processes "
                       f"(one thread each), {busy / wall:.1f} of them busy on average",
                seconds=round(wall, 2))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="pol2x2_na64")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=None,
                    help="update cap (default 100; 300 with --smooth, whose updates converge slower)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-all-cores", action="store_true",
                    help="skip the interval-parallel oracle run beside the one-process baseline")
    ap.add_argument("--mode", default="pass", choices=["pass", "stats"],
                    help="pass: every update streams all samples (the measured metric); "
                         "stats: per-baseline statistics once, updates on them")
    ap.add_argument("--no-alt-mode", action="store_true",
                    help="skip timing the other solve mode")
    ap.add_argument("--out-json", default=None, help="also write the JSON line to this file")
    ap.add_argument("--no-autotune", action="store_true", help="keep the plan's default tiling")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"],
                    help="CohJones Gram products: FP32 MFMA, or BF16 MFMA with FP32 accumulation")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager wcal_solve calls instead of replays of a captured HIP graph")
    ap.add_argument("--smooth", default=None, metavar="SIGMA_T,SIGMA_F",
                    help="StefCal with time/frequency smoothing (Sect. 3.4): a workload of one-sample "
                         "intervals is taken as one 1 x n_int grid of cells, smoothed with these widths")
    ap.add_argument("--points", action="store_true",
                    help="point-source workloads (cohjones_na64): predict the model in the passes "
                         "(wcal_solve_points) instead of reading it from HBM")
    ap.add_argument("--watch", type=int, default=WATCH_DEPTH, metavar="DEPTH",
                    help="host watch of the per-update launches (wcal_plan_watch): eager solves stop "
                         "enqueuing update slots once every interval has stopped, DEPTH slots ahead; "
                         "0: every slot is launched, and solves are timed as HIP graph replays")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before the timed steps, run one plain device copy of this many MiB "
                         "(a known-size reference for hardware byte counters)")
    args = ap.parse_args()

    # the solve the counter runs measured: default tolerance and update cap, unsmoothed, PASS mode
    default_run = (args.max_iter is None and args.tol == 1e-6 and args.smooth is None and args.mode == "pass"
                   and args.watch == WATCH_DEPTH)
    if args.max_iter is None:
        args.max_iter = 300 if args.smooth else 100
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(solution intervals are independent: a batch shards by interval over GPUs with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1502_06974_amd import synth, wcal

    dev = "cuda:0"
    torch.cuda.set_device(0)
    log(f"[bench] generating workload {args.workload}")
    wl_kw = {"n_int": 16} if args.workload == "cohjones_na64" else {}
    P = synth.workload(args.workload, device=dev, **wl_kw)
    torch.cuda.synchronize()
    log(f"[bench] rows={P.n_rows} intervals={P.n_int} n_ant={P.n_ant} n_corr={P.n_corr} n_dir={P.n_dir}")
    algo = "stefcal" if P.n_dir == 1 else "cohjones"
    smooth = None
    if args.smooth:
        smooth = tuple(float(x) for x in args.smooth.split(","))
        if P.n_dir != 1 or P.n_corr != 1 or int(P.ns.max()) != 1:
            sys.exit("--smooth needs a scalar workload of one-sample intervals (bandpass_na256)")
        # the intervals' rows are the samples of one 1 x n_int grid, in the same order
        plan = wcal.Plan(P.n_ant, P.ant1.cpu(), P.ant2.cpu(), [P.n_int], tol=args.tol, max_iter=args.max_iter)
        plan.smoothing(1, P.n_int, smooth[0], smooth[1])
        args.no_graph, args.no_autotune, args.no_alt_mode = True, True, True
    else:
        plan = wcal.plan_for(P, algo=algo, tol=args.tol, max_iter=args.max_iter, mode=args.mode,
                             precision=args.precision)
    pts = None
    if args.points:
        if "uvw" not in P.meta:
            sys.exit("--points needs a point-source workload (cohjones_na64)")
        m = P.meta
        pts = dict(n_time=m["n_time"], n_chan=m["n_chan"], freq0=m["freq0"], dfreq=m["dfreq"],
                   uvw=m["uvw"].contiguous(), lmn=m["lmn"].to(dev).contiguous(),
                   flux=m["flux"].to(dev, torch.float32).contiguous())
        args.no_graph, args.no_autotune = True, True
    graph_too = args.watch > 0 and not args.no_graph    # also time graph replays (every slot)
    if args.watch > 0:
        plan.watch(args.watch)     # captured graphs record every slot: time eager calls
        args.no_graph = True
    g0 = P.unit_gains() if smooth is None else torch.ones(1, P.n_int, P.n_ant, dtype=torch.complex64, device=dev)
    n_out = P.n_int if smooth is None else 1
    tuned = None
    if not args.no_autotune:
        # tiling chosen by the plan autotuner on this workload (before the timed region)
        tuned = plan.autotune(P.data, P.model, P.flags, g0, n_updates=0)    # whole solves to tol
        log(f"[bench] autotune: {tuned}")
    gains = g0.clone()
    residual = torch.empty_like(P.data)
    n_iter = torch.empty(n_out, dtype=torch.int32, device=dev)
    status = torch.empty(n_out, dtype=torch.int32, device=dev)
    chi2 = torch.empty(n_out, dtype=torch.float64, device=dev)

    def step():
        gains.copy_(g0)
        if pts is not None:
            plan.solve_points(**pts, data=P.data, flags=P.flags, gains=gains, residual=residual, n_iter=n_iter,
                              status=status, chi2=chi2)
            return
        solve = plan.solve if smooth is None else plan.solve_smooth
        solve(P.data, P.model, P.flags, gains, residual=residual, n_iter=n_iter, status=status, chi2=chi2)

    if args.calib_copy_mb > 0:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] reference copy of {args.calib_copy_mb} MiB done")
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed steps (the headline time): eager solves under the host watch, which stop enqueuing
    # update slots once every interval has stopped (with --watch 0: each solve replayed from a
    # HIP graph capture of wcal_solve, or eager calls with --no-graph); then the same number of
    # eager steps with HIP events on the launch stream around every kernel launch, for the
    # per-kernel durations (an event pair costs a few microseconds per launch, kept out of the
    # headline)
    timed = step
    if not args.no_graph:
        graph = plan.solve_graph(P.data, P.model, P.flags, gains, residual=residual, n_iter=n_iter,
                                 status=status, chi2=chi2)

        def timed():
            gains.copy_(g0)
            graph.launch()

        timed()
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        timed()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    ms_graph = None
    if graph_too:
        # the same solve replayed from a HIP graph capture, which records all max_iter slots
        graph = plan.solve_graph(P.data, P.model, P.flags, gains, residual=residual, n_iter=n_iter,
                                 status=status, chi2=chi2)
        gains.copy_(g0)
        graph.launch()
        torch.cuda.synchronize()
        tg0 = time.perf_counter()
        for i in range(args.steps):
            gains.copy_(g0)
            graph.launch()
        torch.cuda.synchronize()
        ms_graph = (time.perf_counter() - tg0) * 1e3 / args.steps
        graph.close()
        log(f"[bench] graph replays (every slot): {ms_graph:.3f} ms/solve")
    plan.profile(True)
    plan.profile_read()
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step_profiled = (time.perf_counter() - tp0) * 1e3 / args.steps
    prof = plan.profile_read()
    plan.profile(False)

    rows_k = (P.row_off[1:] - P.row_off[:-1]).to(torch.float64)
    if smooth is not None:
        rows_k = torch.tensor([float(P.n_rows)], dtype=torch.float64)
    it = n_iter.cpu().to(torch.float64)
    st = status.cpu()
    vis_iter = float((rows_k * it).sum())
    value = vis_iter / (ms_step * 1e-3)
    bpr = bytes_per_row(P.n_corr, P.n_dir, P.flags is not None)
    if pts is not None:
        # data and flag per row; the phasor table of a (time slot, baseline), 40 B per direction
        # per 64 channels (four re-base phasors and the step), serves n_chan rows
        nseg = (pts["n_chan"] + 63) // 64
        bpr = 8 * P.n_corr + (1 if P.flags is not None else 0) + 8.0 * P.n_dir * (4 * nseg + 1) / pts["n_chan"]
    # the residual pass reads data, flags and model (or, predicting it, the uvw: 24 B per (time, baseline))
    rbpr = bpr if pts is None else 8 * P.n_corr + (1 if P.flags is not None else 0) + 24.0 / pts["n_chan"]
    resid_bytes = P.n_rows * (rbpr + 8 * P.n_corr)
    dd = P.n_dir > 1
    # wcal_solve_points runs its own Gram kernel, which predicts the model instead of reading it
    kname = "dd_gram_pts_kernel" if pts is not None else plan.pass_kernel
    if args.mode == "pass":
        # every update's pass streams D, M and flags of the interval once
        kcls = "pass"
        krows = float((rows_k * it).sum()) * args.steps
    else:
        kcls = "stats"
        krows = float(P.n_rows) * args.steps
    kbytes = krows * bpr
    kms, klaunch = prof[kcls]
    achieved = kbytes / (kms * 1e-3) / 1e9
    if dd:
        useful = krows * unit_gram_flop_per_row(P.n_corr, P.n_dir)
        own = krows * gram_flop_per_row(P.n_corr, P.n_dir)
        issued = krows * gram_issued_flop_per_row(P.n_corr, P.n_dir)
        tfs = useful / (kms * 1e-3) / 1e12
        tfs_own = own / (kms * 1e-3) / 1e12
        tfs_issued = issued / (kms * 1e-3) / 1e12
    conv = float((st & 1).float().mean())
    log(f"[bench] {ms_step:.3f} ms/step, {kname}: {kms / args.steps:.3f} ms/step over "
        f"{klaunch // args.steps} launches, mean iters {float(it.mean()):.2f}, converged {conv:.4f}, "
        f"{achieved:.1f} GB/s")
    log("[bench] per-class ms/step: " + ", ".join(f"{c}={v[0] / args.steps:.3f}({v[1] // args.steps})"
                                                  for c, v in prof.items()))

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "vis-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32" if args.precision == "fp32" else "bf16 products, fp32 accumulation",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "n_ant": P.n_ant, "n_bl": P.n_bl, "n_dir": P.n_dir, "n_corr": P.n_corr,
            "n_int": P.n_int, "rows": P.n_rows, "tol": args.tol,
            "flag_frac": 0.0 if P.flags is None else round(float(P.flags.float().mean()), 4),
        },
        "solve_time_ms": ms_step,
        "smoothing": None if smooth is None else {"grid": [1, P.n_int], "sigma_t": smooth[0], "sigma_f": smooth[1]},
        "predicted_model": pts is not None,
        "timed_as": ("eager wcal_solve_points calls" if pts else "eager wcal_solve_smooth calls" if smooth else
                     "eager wcal_solve calls" if args.no_graph else "HIP graph replays of wcal_solve")
                    + (f", host watch of depth {args.watch}" if args.watch > 0 else ""),
        "autotune": tuned,
        "solve_time_ms_with_kernel_events": ms_step_profiled,
        "solve_time_ms_graph_every_slot": ms_graph,
        "mode": args.mode,
        "pass_form": ("every update streams the samples once and accumulates J^H J and J^H D per antenna "
                      "(data form, Eq. ghat; J^H r = J^H D - J^H J g); the residual R and chi^2 are formed "
                      "once, by the residual pass after the last update"),
        "mean_iters": float(it.mean()),
        "converged_frac": conv,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(f"{kname}/{args.workload}", default_run),
            "kernel": kname,
            "kernel_ms_per_launch": kms / max(klaunch, 1),
            "launches_per_step": klaunch / args.steps,
            "alg_bytes_per_launch": kbytes / max(klaunch, 1),
        },
        "kernel_ms_per_step": {c: v[0] / args.steps for c, v in prof.items()},
        "solve_effective_GBs": (kbytes / args.steps + resid_bytes) / (ms_step * 1e-3) / 1e9,
    }
    if dd:
        peak = MFMA_FP32_PEAK_TFS if args.precision == "fp32" else MFMA_BF16_PEAK_TFS
        mfma = {
            "bound": "mfma",
            "achieved": tfs,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": tfs / peak,
            "traffic": measured_traffic(f"{kname}/{args.workload}", default_run),
            "kernel": kname,
            "kernel_ms_per_launch": kms / max(klaunch, 1),
            "launches_per_step": klaunch / args.steps,
            "alg_flops_per_launch": useful / max(klaunch, 1),
            "pass_alg_TFLOPs": tfs_own,
            "issued_TFLOPs": tfs_issued,
            "issued_frac": tfs_issued / peak,
        }
        if args.precision == "fp32":
            # FP32 MFMA: the products are the contended resource
            out["roofline_hbm"] = out["roofline"]
            out["roofline"] = mfma
        else:
            # BF16 MFMA issues 16x faster: the pass is bound by HBM
            out["roofline_mfma"] = mfma
    if not args.no_alt_mode and args.precision == "fp32":     # the BF16 Gram runs in PASS mode only
        alt = "stats" if args.mode == "pass" else "pass"
        plan_alt = wcal.plan_for(P, algo=algo, tol=args.tol, max_iter=args.max_iter, mode=alt,
                                 precision=args.precision)
        if args.watch > 0:
            plan_alt.watch(args.watch)
        plan, plan_main = plan_alt, plan
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ms_alt = (time.perf_counter() - t0) * 1e3 / args.steps
        out[f"solve_time_ms_{alt}_mode"] = ms_alt
        out[f"mean_iters_{alt}_mode"] = float(n_iter.cpu().double().mean())
        log(f"[bench] {alt} mode: {ms_alt:.3f} ms/solve")
        plan = plan_main
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(P, args.cpu_budget) if smooth is None else cpu_baseline_smooth(P, smooth)
        out["cpu_baseline"].update(host_cpu())
        if smooth is None and not args.no_cpu_all_cores:
            log("[bench] timing the CPU oracle interval-parallel over the host cores")
            out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(P, args.cpu_budget)
            out["cpu_baseline_all_cores"].update(host_cpu())
    line = json.dumps(out)
    print(line, flush=True)
    if args.out_json:
        with open(args.out_json, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
