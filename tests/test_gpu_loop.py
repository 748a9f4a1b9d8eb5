"""The device-side iteration loop of the StefCal PASS solve and the caller-owned workspace.

The device-side loop is switched off in the library (a plan that asks for it is refused): on
the GPU its first solve did not finish within 120 s, and did not again after the cross-workgroup
values were moved to coherent atomic loads and stores and the ring's positions were bounded.
Its two tests below stay, skipped with that reason, until the cause is found.

* One persistent launch (the work ring of loop_ring.h) computes exactly what one pass launch
  and one update launch per update compute (WCAL_LOOP=0): every output bit for bit, for the
  tiled scalar and 2x2 passes and the triangle pass (one tile per interval, and tiles that
  split intervals), with flags, a singular antenna, a non-finite row and the update cap.
* A wait bound of zero (forced from the host) makes the loop give up: the call still ends,
  every interval is either finished normally or marked WCAL_ABORTED, and an aborted
  interval holds exactly the gains of its applied updates (the oracle replayed for n_iter).
* Every compute call takes its scratch from the caller's workspace: a workspace filled with
  garbage gives the same bits as a fresh one, a workspace one byte short is refused with
  WCAL_ENOMEM before anything runs, and a misaligned one with WCAL_EINVAL.
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
KEYS = ("gains", "residual", "n_iter", "status", "chi2")


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(a, b):
    if a is None or b is None:
        return a is None and b is None
    a, b = a.cpu(), b.cpu()
    return torch.equal(a.view(torch.uint8) if a.is_complex() else a, b.view(torch.uint8) if b.is_complex() else b)


def clone(out):
    return {k: (v.clone() if isinstance(v, torch.Tensor) else v) for k, v in out.items()}


CASES = {
    "scalar": (lambda: synth.scalar_di(30, [3, 10, 1, 40], sigma=0.01, flag_frac=0.1, seed=41, device=DEV), {}),
    "pol": (lambda: synth.pol_di(24, [2, 9, 5, 31], sigma=0.01, flag_frac=0.1, seed=42, device=DEV), {}),
    "pol_split": (lambda: synth.pol_di(40, [1, 7, 64, 65], sigma=0.01, flag_frac=0.05, seed=43, device=DEV),
                  {"WCAL_TILE_ROWS": "700"}),
    "triangle": (lambda: synth.scalar_di(80, [1, 1, 1, 1, 1], sigma=0.01, flag_frac=0.1, seed=44, device=DEV), {}),
    "triangle_split": (lambda: synth.scalar_di(100, [1, 3, 8], sigma=0.01, flag_frac=0.05, seed=45, device=DEV),
                       {"WCAL_TRI": "1", "WCAL_TILE_ROWS": "700"}),
    "triangle_paired": (lambda: synth.scalar_di(130, [1, 2, 1], sigma=0.01, flag_frac=0.1, seed=46, device=DEV), {}),
}


def _faults(P):
    """Antenna 3 fully flagged in interval 0, NaN in an unflagged row of interval 1."""
    flags = torch.zeros(P.n_rows, dtype=torch.uint8, device=DEV) if P.flags is None else P.flags.clone()
    a1, a2 = P.ant1.cpu().numpy(), P.ant2.cpu().numpy()
    bad = torch.as_tensor(np.where((a1 == 3) | (a2 == 3))[0], device=DEV)
    for s in range(int(P.ns[0])):
        flags[int(P.row_off[0]) + s * P.n_bl + bad] = 1
    data = P.data.clone()
    r1 = int(P.row_off[1]) + int(torch.nonzero(flags[int(P.row_off[1]):int(P.row_off[2])] == 0)[0])
    data[r1, 0] = float("nan")
    return data, flags


LOOP_OFF = pytest.mark.skip(reason="device-side loop switched off: its first GPU solve did not finish "
                                   "(twice, the second time after a fix); cause not found")


@LOOP_OFF
@pytest.mark.parametrize("case", list(CASES))
def test_loop_equals_per_update_launches(case, monkeypatch):
    make, env = CASES[case]
    log(f"[loop vs launches] case={case}")
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    P = make()
    data, flags = _faults(P)
    for max_iter, tol in ((60, 1e-6), (4, 0.0)):
        outs = {}
        for loop in ("1", "0"):
            monkeypatch.setenv("WCAL_LOOP", loop)
            plan = wcal.plan_for(P, tol=tol, max_iter=max_iter)
            if loop == "1":
                assert "loop" in plan.pass_kernel, plan.pass_kernel
            outs[loop] = clone(plan.solve(data, P.model, flags, P.unit_gains()))
            torch.cuda.synchronize()
        for key in KEYS:
            assert same(outs["1"][key], outs["0"][key]), (max_iter, key)
        st = outs["1"]["status"].cpu().numpy()
        log(f"  max_iter={max_iter}: status {st.tolist()} n_iter {outs['1']['n_iter'].cpu().tolist()}")
        assert st[0] & oc.SINGULAR_ANT and st[1] == oc.NONFINITE
        assert not np.any(st & wcal.ABORTED)


@LOOP_OFF
def test_loop_abort_leaves_every_interval_consistent(monkeypatch):
    """WCAL_WAIT_MS=0: the first wait of the loop runs out at once.  The call ends; intervals
    not finished are WCAL_ABORTED, and every interval's gains are the oracle's after exactly
    n_iter updates from the start (an update is applied whole or not at all)."""
    log("[loop abort]")
    monkeypatch.setenv("WCAL_WAIT_MS", "0")
    P = synth.pol_di(16, [4, 1, 9, 2, 6, 3], sigma=0.01, flag_frac=0.05, seed=47, device=DEV)
    # interval 1 stops at its first update (NaN in an unflagged row): from then on the loop
    # has more workgroups than tiles in the ring, so some workgroup waits, and gives up
    data = P.data.clone()
    r1 = int(P.row_off[1]) + int(torch.nonzero(P.flags[int(P.row_off[1]):int(P.row_off[2])] == 0)[0])
    data[r1, 0] = float("nan")
    plan = wcal.plan_for(P, tol=1e-6, max_iter=40)
    out = plan.solve(data, P.model, P.flags, P.unit_gains())
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    ni = out["n_iter"].cpu().numpy()
    g = out["gains"].cpu().numpy()
    log(f"  status {st.tolist()} n_iter {ni.tolist()}")
    assert np.any(st & wcal.ABORTED)
    for k in range(P.n_int):
        if st[k] & wcal.ABORTED:
            assert not st[k] & (oc.CONVERGED | oc.MAXITER)
        else:
            assert st[k] & (oc.CONVERGED | oc.MAXITER | oc.NONFINITE)
        o = glue.solve(P, k, P.unit_gains()[k].cpu().numpy(), tol=0.0, max_iter=int(ni[k])) if ni[k] else None
        ref = P.unit_gains()[k].cpu().numpy() if o is None else glue.gains_from_oracle(o["g"], 4, 1)
        assert gain_err(g[k], ref, 4) <= 1e-5, k
    # a normal wait bound again: the same plan solves to the end
    monkeypatch.setenv("WCAL_WAIT_MS", "20000")
    plan2 = wcal.plan_for(P, tol=1e-6, max_iter=40)
    out2 = plan2.solve(data, P.model, P.flags, P.unit_gains())
    assert not torch.any(out2["status"] & wcal.ABORTED)
    assert int(out2["status"][1]) == oc.NONFINITE


WS_CASES = {
    "scalar_pass": (lambda: synth.scalar_di(30, [3, 10, 1], sigma=0.01, flag_frac=0.1, seed=51, device=DEV),
                    dict(mode="pass")),
    "pol_stats": (lambda: synth.pol_di(24, [2, 9, 5], sigma=0.01, flag_frac=0.1, seed=52, device=DEV),
                  dict(mode="stats")),
    "triangle": (lambda: synth.scalar_di(80, [1, 1, 1], sigma=0.01, flag_frac=0.1, seed=53, device=DEV), {}),
    "cohjones": (lambda: synth.dd_point(12, 3, n_time=3, n_chan=4, n_int=2, seed=54, device=DEV, flag_frac=0.05,
                                        fov_deg=2.0, disk_diam=2e4), dict(algo="cohjones")),
    "pol_alljones_stats": (lambda: synth.pol_dd(10, [3, 4], 2, seed=55, device=DEV, flag_frac=0.05),
                           dict(algo="alljones", mode="stats")),
}


@pytest.mark.parametrize("case", list(WS_CASES))
def test_workspace_contents_do_not_matter(case):
    """Solve, accumulate and residual on a zeroed workspace and on one full of 0xff bytes (NaN
    patterns, negative counters) give the same bits: every call initialises what it uses."""
    make, kw = WS_CASES[case]
    log(f"[workspace contents] case={case}")
    P = make()
    plan = wcal.plan_for(P, tol=1e-6, max_iter=30, **kw)
    n = plan.workspace_bytes()
    assert n > 0
    outs = []
    for fill in (0x00, 0xFF):
        ws = torch.full((n,), fill, dtype=torch.uint8, device=DEV)
        o = clone(plan.solve(P.data, P.model, P.flags, P.unit_gains(), workspace=ws))
        ws.fill_(fill)
        g = P.g_true.contiguous()
        a = clone(plan.accumulate(P.data, P.model, P.flags, g, want_residual=True, workspace=ws))
        ws.fill_(fill)
        r = clone(plan.residual(P.data, P.model, P.flags, g, workspace=ws))
        torch.cuda.synchronize()
        outs.append((o, a, r))
    for x, y in zip(outs[0], outs[1]):
        for key in x:
            assert same(x[key], y[key]), key


def test_workspace_too_small_or_misaligned_is_refused():
    """One byte short: WCAL_ENOMEM before any launch (the outputs keep their sentinel values);
    an address off the 256-byte grid: WCAL_EINVAL."""
    log("[workspace size]")
    P = synth.pol_di(24, [2, 9, 5], sigma=0.01, flag_frac=0.1, seed=56, device=DEV)
    plan = wcal.plan_for(P)
    n = plan.workspace_bytes()
    small = torch.zeros(n - 1, dtype=torch.uint8, device=DEV)
    gains = P.unit_gains()
    n_iter = torch.full((P.n_int,), -7, dtype=torch.int32, device=DEV)
    with pytest.raises(wcal.WcalError) as ei:
        plan.solve(P.data, P.model, P.flags, gains, n_iter=n_iter, workspace=small)
    assert ei.value.code == wcal.ENOMEM
    torch.cuda.synchronize()
    assert torch.all(n_iter == -7) and torch.equal(gains, P.unit_gains())
    with pytest.raises(wcal.WcalError) as ei:
        plan.residual(P.data, P.model, P.flags, gains, workspace=small)
    assert ei.value.code == wcal.ENOMEM
    big = torch.zeros(n + 512, dtype=torch.uint8, device=DEV)
    with pytest.raises(wcal.WcalError) as ei:
        plan.solve(P.data, P.model, P.flags, gains, workspace=big[8:])
    assert ei.value.code == wcal.EINVAL
    out = plan.solve(P.data, P.model, P.flags, gains, workspace=big[256:])
    torch.cuda.synchronize()
    assert torch.all(out["status"] & oc.CONVERGED)


def test_workspace_size_follows_tiling_and_smoothing():
    """The size is reported again after the autotuner re-tiles and after smoothing is set up;
    the autotuner's own workspace holds every candidate."""
    log("[workspace size changes]")
    P = synth.scalar_di(40, [1, 1, 1, 1], sigma=0.05, seed=57, device=DEV)
    plan = wcal.plan_for(P, tol=1e-6, max_iter=50)
    n0 = plan.workspace_bytes()
    plan.autotune(P.data, P.model, P.flags, P.unit_gains(), n_updates=2)
    n1 = plan.workspace_bytes()
    assert n1 > 0
    out = plan.solve(P.data, P.model, P.flags, P.unit_gains())
    torch.cuda.synchronize()
    assert torch.all(out["status"] & oc.CONVERGED)
    sp = wcal.Plan(P.n_ant, P.ant1.cpu(), P.ant2.cpu(), [P.n_int], tol=1e-6, max_iter=100)
    m0 = sp.workspace_bytes()
    sp.smoothing(1, P.n_int, 0.0, 1.0)
    m1 = sp.workspace_bytes()
    log(f"  plan {n0} -> {n1} bytes after autotune; smoothing plan {m0} -> {m1} bytes")
    assert m1 > m0


def test_mlp_weight_file_round_trip(tmp_path):
    """wcal_mlp_save / wcal_mlp_load: the JSON header names the network, the parameters and
    Adam moments come back bit for bit (the next Adam step of the loaded copy equals the
    original's), and a network of another shape or a damaged file is refused."""
    import json
    log("[mlp save/load]")
    torch.manual_seed(3)
    a = wcal.Mlp(6, 12, 6, max_batch=32, skip=True)
    a.set_params(0.1 * torch.randn(a.n_params, device=DEV))
    x = torch.randn(20, 6, device=DEV)
    t = torch.randn(20, 6, device=DEV)
    for _ in range(3):
        a.train_step(x, t, 1e-2)
    path = str(tmp_path / "net.wmlp")
    a.save(path)
    with open(path, "rb") as f:
        head = json.loads(f.readline())
    assert head["format"] == "wcal-mlp" and head["n_params"] == a.n_params and head["adam_step"] == 3
    assert (head["d_in"], head["d_hidden"], head["d_out"], head["skip"]) == (6, 12, 6, 1)
    b = wcal.Mlp(6, 12, 6, max_batch=32, skip=True)
    b.load(path)
    assert torch.equal(a.get_params(), b.get_params())
    a.train_step(x, t, 1e-2)
    b.train_step(x, t, 1e-2)
    assert torch.equal(a.get_params(), b.get_params())
    assert torch.equal(a.forward(x), b.forward(x))
    c = wcal.Mlp(6, 13, 6, max_batch=32, skip=True)
    with pytest.raises(wcal.WcalError) as ei:
        c.load(path)
    assert ei.value.code == wcal.EINVAL
    raw = open(path, "rb").read()
    open(str(tmp_path / "short.wmlp"), "wb").write(raw[:-4])
    with pytest.raises(wcal.WcalError) as ei:
        b.load(str(tmp_path / "short.wmlp"))
    assert ei.value.code == wcal.EIO
    open(str(tmp_path / "junk.wmlp"), "wb").write(b'{"format": "other"}\n' + raw)
    with pytest.raises(wcal.WcalError) as ei:
        b.load(str(tmp_path / "junk.wmlp"))
    assert ei.value.code == wcal.EIO


def test_loop_request_is_refused(monkeypatch):
    """WCAL_LOOP=1 asks for the switched-off loop: plan creation refuses it (no launch)."""
    monkeypatch.setenv("WCAL_LOOP", "1")
    P = synth.scalar_di(12, [2], sigma=0.01, seed=58, device=DEV)
    with pytest.raises(wcal.WcalError) as ei:
        wcal.plan_for(P)
    assert ei.value.code == wcal.EINVAL
