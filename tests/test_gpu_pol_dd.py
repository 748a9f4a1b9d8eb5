"""GPU parity of the polarized direction-dependent path (2x2 Jones CohJones and AllJones,
Sect. 4.4) against the CPU oracle.

Tolerances as for the scalar path: gains within 1e-5 relative (one phase per direction
aligned when both sides converge independently), per-antenna blocks of one pass within
2e-5 of the block scale, integer row counts and status bits exact.  The direction counts
cover every tile shape of the Gram pass (1, 2 and 3 sixteen-column tiles, with and
without the residual columns of the accumulate pass).  At the full 64-antenna,
10-direction, 1920-sample size the solution is checked through properties that hold at
any size: the CohJones fixed point G H_p = N_p evaluated by the oracle on the rows of
sampled antennas, and recovery of noise-free gains.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import calib as oc
from oracle import driver as glue
from paper_1502_06974_amd import synth, wcal
from gains_check import gain_err, oracle_stop, stop_decision_is_clear

pytestmark = pytest.mark.gpu
DEV = "cuda"
MODES = ["pass", "stats"]
NDS = [1, 2, 3, 6, 10]


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small(n_dir=3, seed=0, flag_frac=0.1, ns=(5, 11), n_ant=12, noise=True):
    return synth.pol_dd(n_ant, list(ns), n_dir, seed=seed, device=DEV, flag_frac=flag_frac, noise=noise)


def perturbed(P, scale=0.2, seed=0):
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    return (P.g_true + scale * torch.randn(P.g_true.shape, dtype=torch.complex64, device=DEV,
                                           generator=g)).contiguous()


def unit(P):
    return P.unit_gains()


def by_dir(X, nd):
    """Oracle [Na, 2, 2Nd] row blocks -> the library layout [Na][Nd * 4] (entry 4 d + 2 i + l)."""
    return np.swapaxes(X.reshape(X.shape[0], 2, nd, 2), 1, 2).reshape(X.shape[0], 4 * nd)


@pytest.mark.parametrize("nd", NDS)
def test_pol_dd_accumulate_parity(nd):
    log(f"[pol dd accumulate] nd={nd}")
    P = small(n_dir=nd, seed=1)
    g = perturbed(P)
    plan = wcal.plan_for(P, algo="cohjones")
    out = plan.accumulate(P.data, P.model, P.flags, g, want_residual=True)
    torch.cuda.synchronize()
    gh = g.cpu().numpy()
    na = P.n_ant
    for k in range(P.n_int):
        o = glue.accumulate(P, k, gh[k], algo="cohjones")
        assert np.array_equal(out["count"][k].cpu().numpy(), o["count"])
        H = out["jhj"][k].cpu().numpy().reshape(na, 2 * nd, 2 * nd)
        assert np.abs(H - o["H"]).max() <= 2e-5 * np.abs(o["H"]).max()
        N = out["jhd"][k].cpu().numpy()
        No = by_dir(o["N"], nd)
        assert np.abs(N - No).max() <= 2e-5 * np.abs(No).max()
        R = out["jhr"][k].cpu().numpy()
        assert np.abs(R - by_dir(o["jhr"], nd)).max() <= 2e-5 * np.abs(No).max()
        rr, chi = glue.residual(P, k, gh[k], algo="cohjones")
        a, b = int(P.row_off[k]), int(P.row_off[k + 1])
        res = out["residual"][a:b].cpu().numpy().reshape(-1, 2, 2)
        assert np.abs(res - rr).max() <= 1e-5 * np.abs(rr).max()
        fl = P.interval(k)["flags"]
        assert np.all(res[fl] == 0)
        assert abs(float(out["chi2"][k]) - chi) <= 1e-5 * chi
        # the residual entry point gives the same R and chi^2
        r2 = plan.residual(P.data, P.model, P.flags, g)
        torch.cuda.synchronize()
        res2 = r2["residual"][a:b].cpu().numpy().reshape(-1, 2, 2)
        assert np.abs(res2 - rr).max() <= 1e-5 * np.abs(rr).max()
        assert abs(float(r2["chi2"][k]) - chi) <= 1e-5 * chi


@pytest.mark.parametrize("algo", ["cohjones", "alljones"])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("nd", [2, 6, 10])
def test_pol_dd_lockstep(algo, mode, nd):
    """Both sides apply exactly 6 updates from unit gains (tol = 0)."""
    log(f"[pol dd lockstep] algo={algo} mode={mode} nd={nd}")
    P = small(n_dir=nd, seed=2, flag_frac=0.05)
    plan = wcal.plan_for(P, algo=algo, tol=0.0, max_iter=6, mode=mode)
    out = plan.solve(P.data, P.model, P.flags, unit(P))
    torch.cuda.synchronize()
    g = out["gains"].cpu().numpy()
    for k in range(P.n_int):
        o = glue.solve(P, k, unit(P)[k].cpu().numpy(), algo=algo, tol=0.0, max_iter=6)
        go = glue.gains_from_oracle(o["g"], 4, nd, algo)
        e = gain_err(g[k], go, 4)
        log(f"  interval {k}: err={e:.2e}")
        assert e <= 1e-5, (k, e)
        assert int(out["n_iter"][k]) == 6 and int(out["status"][k]) == o["status"]
        assert abs(float(out["chi2"][k]) - o["chi2"]) <= 1e-4 * o["chi2"]


@pytest.mark.parametrize("algo", ["cohjones", "alljones"])
def test_pol_dd_converged(algo):
    log(f"[pol dd converged] algo={algo}")
    nd = 3
    P = small(n_dir=nd, seed=3, flag_frac=0.05, ns=(8, 12))
    plan = wcal.plan_for(P, algo=algo, tol=1e-6, max_iter=400)
    out = plan.solve(P.data, P.model, P.flags, unit(P))
    torch.cuda.synchronize()
    g = out["gains"].cpu().numpy()
    for k in range(P.n_int):
        o = glue.solve(P, k, unit(P)[k].cpu().numpy(), algo=algo, tol=1e-12, max_iter=5000)
        go = glue.gains_from_oracle(o["g"], 4, nd, algo)
        assert int(out["status"][k]) & oc.CONVERGED
        e = gain_err(glue.align(g[k], go, nd), go, 4)
        n_stop = oracle_stop(o["history"], 1e-6, 400)
        clear = stop_decision_is_clear(o["history"], 1e-6, n_stop)
        log(f"  interval {k}: gpu_iter={int(out['n_iter'][k])} oracle_stop={n_stop} (clear={clear}) err={e:.2e}")
        assert e <= 1e-5
        if clear:
            assert int(out["n_iter"][k]) == n_stop


@pytest.mark.parametrize("algo", ["cohjones", "alljones"])
def test_pol_dd_status_bits(algo):
    """A fully flagged antenna is singular (gain kept bit-for-bit); NaN unflagged stops the
    interval before any update."""
    log(f"[pol dd status] algo={algo}")
    P = small(n_dir=2, seed=4, flag_frac=0.0, ns=(6, 6, 6))
    flags = torch.zeros(P.n_rows, dtype=torch.uint8, device=DEV)
    a1, a2 = P.ant1.cpu().numpy(), P.ant2.cpu().numpy()
    bad = torch.as_tensor(np.where((a1 == 5) | (a2 == 5))[0], device=DEV)
    r0, ns0 = int(P.row_off[0]), int(P.ns[0])
    for s in range(ns0):
        flags[r0 + s * P.n_bl + bad] = 1
    data = P.data.clone()
    data[int(P.row_off[1]) + 3, 2] = float("nan")
    g0 = unit(P)
    g0[:, :, 5, 0] = 0.75 - 0.5j
    plan = wcal.plan_for(P, algo=algo, tol=1e-6, max_iter=200)
    out = plan.solve(data, P.model, flags, g0.clone())
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    g = out["gains"].cpu().numpy()
    fn = oc.cohjones_2x2 if algo == "cohjones" else oc.alljones_2x2
    for k in range(3):
        iv = P.interval(k)
        D, M = glue.split(iv, 4, 2, algo)
        D = D.copy()
        if k == 1:
            D[3, 1, 0] = np.nan
        fl = flags[int(P.row_off[k]):int(P.row_off[k + 1])].cpu().numpy() != 0
        o = fn(D, M, iv["p"], iv["q"], fl, glue.gains_to_oracle(g0[k].cpu().numpy(), 4, 2, algo),
               tol=1e-6, max_iter=200)
        assert st[k] == o["status"], (k, st[k], o["status"])
    assert st[0] & oc.SINGULAR_ANT and st[0] & oc.CONVERGED
    assert np.array_equal(g[0, :, 5], g0[0, :, 5].cpu().numpy())
    assert st[1] == oc.NONFINITE and int(out["n_iter"][1]) == 0
    assert np.array_equal(g[1], g0[1].cpu().numpy())


def test_pol_dd_garbage_under_flags_is_bit_identical():
    """Flagged rows enter no sum: NaN and 1e30 written into them change no output bit."""
    log("[pol dd flags]")
    P = small(n_dir=3, seed=5, flag_frac=0.2)
    fl = P.flags.bool()
    data, model = P.data.clone(), P.model.clone()
    data[fl] = float("nan")
    model[fl] = 1e30
    outs = []
    for d, m in ((P.data, P.model), (data, model)):
        for algo in ("cohjones", "alljones"):
            plan = wcal.plan_for(P, algo=algo, tol=0.0, max_iter=5)
            outs.append(plan.solve(d, m, P.flags, unit(P)))
    torch.cuda.synchronize()
    for a, b in ((outs[0], outs[2]), (outs[1], outs[3])):
        assert torch.equal(a["gains"], b["gains"])
        assert torch.equal(a["chi2"], b["chi2"]) and torch.equal(a["status"], b["status"])
        assert torch.equal(a["residual"][~fl], b["residual"][~fl])
        assert torch.all(b["residual"][fl] == 0)


def test_pol_dd_model_must_be_16_byte_aligned():
    """The 2x2 Gram copies model rows to LDS in 16-byte pieces: a model array that is only
    8-byte aligned is refused before any launch."""
    log("[pol dd alignment]")
    P = small(n_dir=2, seed=8)
    buf = torch.empty(P.model.numel() + 1, dtype=P.model.dtype, device=DEV)
    model_u = buf[1:].view(P.model.shape)
    model_u.copy_(P.model)
    assert model_u.data_ptr() % 16 == 8
    plan = wcal.plan_for(P, algo="cohjones", tol=0.0, max_iter=2)
    with pytest.raises(wcal.WcalError):
        plan.solve(P.data, model_u, P.flags, unit(P))


@pytest.mark.parametrize("algo", ["cohjones", "alljones"])
def test_pol_dd_antenna_with_many_rows(algo):
    """Repeated baseline pairs give antenna 0 more rows than the per-antenna update stages
    at once (256): lockstep parity with the oracle."""
    log(f"[pol dd many rows] algo={algo}")
    a1 = [0] * 140 + [0] * 130 + [1, 1, 2, 0]
    a2 = [1] * 140 + [2] * 130 + [2, 3, 3, 3]
    P = synth.pol_dd(4, [3, 2], 2, seed=8, device=DEV, flag_frac=0.05, pairs=(a1, a2))
    plan = wcal.plan_for(P, algo=algo, tol=0.0, max_iter=4)
    out = plan.solve(P.data, P.model, P.flags, unit(P))
    torch.cuda.synchronize()
    g = out["gains"].cpu().numpy()
    for k in range(P.n_int):
        o = glue.solve(P, k, unit(P)[k].cpu().numpy(), algo=algo, tol=0.0, max_iter=4)
        go = glue.gains_from_oracle(o["g"], 4, 2, algo)
        e = gain_err(g[k], go, 4)
        log(f"  interval {k}: err={e:.2e}")
        assert e <= 1e-5, (k, e)


def test_pol_dd_nd1_matches_pol_stefcal():
    """One direction: polarized CohJones and AllJones are polarized StefCal."""
    log("[pol dd nd1]")
    P = synth.pol_di(20, [5, 9], sigma=0.01, flag_frac=0.05, seed=7, device=DEV)
    outs = {}
    for algo in ("stefcal", "cohjones", "alljones"):
        plan = wcal.plan_for(P, algo=algo, tol=0.0, max_iter=8)
        outs[algo] = plan.solve(P.data, P.model, P.flags, unit(P))["gains"].cpu().numpy()
    assert gain_err(outs["cohjones"], outs["stefcal"], 4) <= 1e-5
    assert gain_err(outs["alljones"], outs["stefcal"], 4) <= 1e-5


@pytest.mark.parametrize("algo", ["cohjones", "alljones"])
def test_pol_dd_full_sample_count_lockstep(algo):
    """The per-interval sample count of the polarized CohJones workload (30 time slots x 64
    channels = 1920 samples, 120 sixteen-sample Gram chunks per baseline) with 10 directions,
    on 10 antennas so that the oracle holds every row's 2Nd x 2Nd product: three updates from
    unit gains on both sides, PASS and STATS modes, gains per antenna and direction, chi^2
    and the residual (Sect. 4.4)."""
    log(f"[pol dd full samples] algo={algo}")
    P = synth.pol_dd(10, [1920], 10, seed=33, device=DEV, flag_frac=0.05)
    o = glue.solve(P, 0, unit(P)[0].cpu().numpy(), algo=algo, tol=0.0, max_iter=3)
    go = glue.gains_from_oracle(o["g"], 4, 10, algo)
    for mode in MODES:
        plan = wcal.plan_for(P, algo=algo, tol=0.0, max_iter=3, mode=mode)
        out = plan.solve(P.data, P.model, P.flags, unit(P))
        torch.cuda.synchronize()
        e = gain_err(out["gains"][0].cpu().numpy(), go, 4)
        log(f"  {mode}: rows={P.n_rows} gains vs oracle {e:.2e}")
        assert e <= 1e-5
        assert int(out["n_iter"][0]) == 3 and int(out["status"][0]) == o["status"]
        assert abs(float(out["chi2"][0]) - o["chi2"]) <= 1e-4 * o["chi2"]
        res = out["residual"].cpu().numpy().reshape(-1, 2, 2)
        assert np.abs(res - o["residual"]).max() <= 1e-4 * np.abs(o["residual"]).max()
        assert np.all(res[P.interval(0)["flags"]] == 0)


def _fixed_point_residual(P, k, G, ants):
    """max over sampled antennas of ||G_p H_p - N_p|| / ||N_p|| with H_p, N_p from the oracle
    on exactly the rows touching p (the polarized CohJones fixed point)."""
    iv = P.interval(k)
    D, M = glue.split(iv, 4, P.n_dir, "cohjones")
    worst = 0.0
    for a in ants:
        sel = (iv["p"] == a) | (iv["q"] == a)
        acc = oc.accumulate_dd_2x2(D[sel], M[sel], iv["p"][sel], iv["q"][sel], iv["flags"][sel], G)
        Gs = np.swapaxes(G[:, a], 0, 1).reshape(2, -1)    # stacked [G^0 .. G^{Nd-1}]
        r = np.linalg.norm(Gs @ acc["H"][a] - acc["N"][a]) / np.linalg.norm(acc["N"][a])
        worst = max(worst, r)
    return worst


@pytest.mark.parametrize("mode", MODES)
def test_pol_cohjones_na64_full_size(mode):
    """Full size (64 antennas, 10 directions, 30 x 64 samples per interval): the solution
    satisfies the fixed point on sampled antennas, and noise-free data recover the true
    gains."""
    log(f"[pol cohjones na64 full] mode={mode}")
    P = synth.workload("pol_cohjones_na64", device=DEV, n_int=2, flag_frac=0.05)
    plan = wcal.plan_for(P, algo="cohjones", tol=1e-6, max_iter=300, mode=mode)
    out = plan.solve(P.data, P.model, P.flags, unit(P), want_residual=False)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    log(f"  status={st.tolist()} iters={out['n_iter'].cpu().tolist()}")
    assert np.all(st & oc.CONVERGED)
    for k in range(P.n_int):
        G = glue.gains_to_oracle(out["gains"][k].cpu().numpy(), 4, P.n_dir, "cohjones")
        fp = _fixed_point_residual(P, k, G, [0, 31, 63])
        log(f"  interval {k}: fixed-point residual {fp:.2e}")
        assert fp <= 2e-5
    Q = synth.workload("pol_cohjones_na64", device=DEV, n_int=1, noise=False)
    plan_q = wcal.plan_for(Q, algo="cohjones", tol=1e-7, max_iter=500, mode=mode)
    out = plan_q.solve(Q.data, Q.model, Q.flags, unit(Q), want_residual=False)
    torch.cuda.synchronize()
    g = out["gains"][0].cpu().numpy()
    gt = Q.g_true[0].cpu().numpy()
    e = gain_err(glue.align(g, gt, Q.n_dir), gt, 4)
    log(f"  noise-free recovery err={e:.2e} iters={int(out['n_iter'][0])}")
    assert e <= 1e-5


def test_pol_dd_rejects_bf16_and_too_many_directions():
    P = small(n_dir=2, seed=6)
    with pytest.raises(wcal.WcalError):
        wcal.plan_for(P, algo="cohjones", precision="bf16")
    Q = small(n_dir=11, seed=6, ns=(1,))
    with pytest.raises(wcal.WcalError):
        wcal.plan_for(Q, algo="cohjones")
