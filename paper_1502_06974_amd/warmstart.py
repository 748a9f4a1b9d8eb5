"""Learned warm start for batched single-channel StefCal (argument marshalling only).

Every step runs in libwcal kernels:
  coarse pass: rows of one knot channel per bin gathered (wcal_gather_knots) and solved
    from unit gains by a second plan (wcal_solve); its gains referenced to antenna 0
    are the features                                                (wcal_gains_to_bins)
  network over frequency: knot features -> knot gains, with a skip connection so that the
    untrained network (zero last layer) passes the coarse solution through  (wcal_mlp_*)
  interpolation: knot gains -> every channel, amplitude and phase linear (wcal_bins_to_gains)
  solve from those gains; intervals that do not converge are reset to unit gains and the
    batch is solved again                                           (wcal_reset_unconverged)
Training targets are the gains the plain solver reaches from unit starts on synthetic
observations of one sky (fresh gains and noise), referenced and averaged in a window
around each knot; the network trains with its own backward and Adam kernels.
"""
from __future__ import annotations

import math
import time

import torch

from . import synth, wcal


def init_params(d_in: int, d_h: int, d_out: int, seed: int, device, zero_last: bool = False) -> torch.Tensor:
    """Uniform(+-sqrt(6/(fan_in+fan_out))) weights, zero biases, from a seeded generator;
    zero_last leaves the output layer at zero (with the skip connection: identity map)."""
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    parts = []
    for i, (fi, fo) in enumerate(((d_in, d_h), (d_h, d_h), (d_h, d_out))):
        lim = math.sqrt(6.0 / (fi + fo))
        w = (torch.rand(fi * fo, generator=g, device=device) * 2 - 1) * lim
        if zero_last and i == 2:
            w = torch.zeros_like(w)
        parts += [w, torch.zeros(fo, device=device)]
    return torch.cat(parts).float().contiguous()


class WarmStart:
    """Warm start for a scalar StefCal plan whose intervals are consecutive channels."""

    def __init__(self, plan: wcal.Plan, bin_width: int = 64, hidden: int = 256, halfwidth: int = 0,
                 coarse_tol: float = 1e-4, coarse_max_iter: int = 200, seed: int = 0, max_batch: int = 8192):
        assert plan.n_corr == 1 and plan.n_dir == 1
        self.plan, self.bin_width, self.halfwidth = plan, bin_width, halfwidth
        self.n_ant, self.n_int = plan.n_ant, plan.n_int
        self.knots = wcal.bin_knots(plan.n_int, bin_width)
        self.n_bins = int(self.knots.numel())
        ns_k = plan.ns[self.knots.long()]
        self.coarse = wcal.Plan(plan.n_ant, plan.ant1, plan.ant2, ns_k, tol=coarse_tol,
                                max_iter=coarse_max_iter, device=plan.device)
        # the full plan's solve restricted to the knot channels (intervals are independent, so
        # its solutions there are the full solve's): training targets without the other channels
        self.fine = wcal.Plan(plan.n_ant, plan.ant1, plan.ant2, ns_k, tol=plan.prob.tol,
                              max_iter=plan.prob.max_iter, device=plan.device)
        dev = torch.device("cuda", plan.device)
        rows = self.coarse.rows
        self._d = torch.empty(rows, 1, dtype=torch.complex64, device=dev)
        self._m = torch.empty(rows, 1, 1, dtype=torch.complex64, device=dev)
        self._f = torch.empty(rows, dtype=torch.uint8, device=dev)
        d = 2 * self.n_bins
        self.mlp = wcal.Mlp(d, hidden, d, max_batch=max(max_batch, plan.n_ant), skip=True, device=plan.device)
        self.mlp.set_params(init_params(d, hidden, d, seed, dev, zero_last=True))

    # ---------------------------------------------------------------- coarse pass
    def features(self, data, model, flags) -> tuple:
        """Knot-channel solve from unit gains; returns (features [n_ant][2 n_bins], coarse
        solve outputs)."""
        fl = self._f if flags is not None else None
        wcal.gather_knots(self.plan, self.bin_width, data, model, flags, self._d, self._m, fl)
        g = torch.zeros(self.n_bins, 1, self.n_ant, 1, dtype=torch.complex64, device=data.device)
        g[..., 0] = 1
        out = self.coarse.solve(self._d, self._m, fl, g, want_residual=False, want_chi2=False)
        return wcal.gains_to_bins(out["gains"], 1, 0), out

    # ---------------------------------------------------------------- inference
    def predict(self, data, model, flags, use_network: bool = True) -> torch.Tensor:
        f, _ = self.features(data, model, flags)
        y = self.mlp.forward(f) if use_network else f
        return wcal.bins_to_gains(y, self.n_int, self.bin_width)

    def solve(self, data, model, flags, use_network: bool = True, **kw) -> dict:
        """Warm-started solve of the full plan (see solve_from)."""
        return self.solve_from(self.plan, data, model, flags, self.predict(data, model, flags, use_network), **kw)

    @staticmethod
    def solve_from(plan: wcal.Plan, data, model, flags, gains, **kw) -> dict:
        """Solve from the given start; every interval that does not converge (non-finite
        values, iteration cap) is reset to unit gains and the batch is solved again.
        Returns the solve outputs plus 'fallback' (intervals reset) and 'n_iter_total'
        (updates over both solves)."""
        out = plan.solve(data, model, flags, gains, **kw)
        conv = (out["status"] & wcal.CONVERGED) != 0
        n_fail = int((~conv).sum())
        total = out["n_iter"].clone()
        if n_fail:
            wcal.reset_unconverged(plan, out["status"], gains)
            out = plan.solve(data, model, flags, gains, **kw)
            total = total + out["n_iter"]
        out["fallback"] = n_fail
        out["n_iter_total"] = total
        return out

    # ---------------------------------------------------------------- training
    def make_example(self, P: synth.Problem):
        """(features, targets, all converged) for one observation: the targets come from the
        plain solver's unit-start solution."""
        f, _ = self.features(P.data, P.model, P.flags)
        out = self.plan.solve(P.data, P.model, P.flags, P.unit_gains(), want_residual=False, want_chi2=False)
        t = wcal.gains_to_bins(out["gains"], self.bin_width, self.halfwidth)
        ok = bool(((out["status"] & wcal.CONVERGED) != 0).all())
        return f, t, ok

    def make_example_knots(self, K: synth.Problem):
        """make_example from the knot channels alone (K holds only their rows, one interval per
        knot in knot order, e.g. synth.bandpass_di(..., channels=knots)): the coarse pass and the
        unit-start solve of the knots, which is what the full solve gives there.  Needs
        halfwidth 0 (a wider target window reads channels between the knots)."""
        assert self.halfwidth == 0 and K.ns.numel() == self.n_bins
        g = torch.zeros(self.n_bins, 1, self.n_ant, 1, dtype=torch.complex64, device=K.data.device)
        g[..., 0] = 1
        co = self.coarse.solve(K.data, K.model, K.flags, g.clone(), want_residual=False, want_chi2=False)
        fi = self.fine.solve(K.data, K.model, K.flags, g, want_residual=False, want_chi2=False)
        f = wcal.gains_to_bins(co["gains"], 1, 0)
        t = wcal.gains_to_bins(fi["gains"], 1, 0)
        ok = bool(((fi["status"] & wcal.CONVERGED) != 0).all())
        return f, t, ok

    def train(self, X: torch.Tensor, T: torch.Tensor, epochs: int = 30, batch: int = 4096, lr: float = 1e-3,
              seed: int = 0, log=None) -> list:
        g = torch.Generator(device=X.device)
        g.manual_seed(seed)
        n = X.shape[0]
        losses = []
        loss = torch.zeros(1, dtype=torch.float64, device=X.device)
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g, device=X.device)
            acc = torch.zeros((), dtype=torch.float64, device=X.device)
            nb = 0
            for i in range(0, n, batch):
                idx = perm[i:i + batch]
                self.mlp.train_step(X[idx].contiguous(), T[idx].contiguous(), lr, loss)
                acc += loss[0]
                nb += 1
            losses.append(float(acc) / max(nb, 1))
            if log:
                log(f"  epoch {ep}: loss {losses[-1]:.3e}")
        return losses


def evaluate(ws: WarmStart, P: synth.Problem, **kw) -> dict:
    """One held-out observation: unit start, the coarse pass without the network (identity),
    and the trained network; updates per interval (the coarse pass's updates counted at its
    share of the rows) and wall time of each, coarse pass included."""
    res = {}
    coarse_share = ws.coarse.rows / ws.plan.rows
    for name in ("unit", "coarse", "mlp"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if name == "unit":
            out = ws.plan.solve(P.data, P.model, P.flags, P.unit_gains(), want_residual=False, **kw)
            out["n_iter_total"], out["fallback"] = out["n_iter"], 0
            c_it = 0.0
        else:
            f, co = ws.features(P.data, P.model, P.flags)
            y = ws.mlp.forward(f) if name == "mlp" else f
            g = wcal.bins_to_gains(y, ws.n_int, ws.bin_width)
            out = ws.solve_from(ws.plan, P.data, P.model, P.flags, g, want_residual=False, **kw)
            c_it = float(co["n_iter"].float().sum()) * coarse_share / ws.n_bins
        torch.cuda.synchronize()
        it = out["n_iter_total"].float()
        res[name] = dict(ms=1e3 * (time.perf_counter() - t0), mean_iter=float(it.mean()) + c_it,
                         median_iter=float(it.median()), coarse_iter=c_it, fallback=int(out["fallback"]),
                         converged=int(((out["status"] & wcal.CONVERGED) != 0).sum()), gains=out["gains"])
    return res


def main(argv=None):
    import argparse
    import json
    import statistics

    ap = argparse.ArgumentParser(description="Train the warm-start network on device and compare unit, "
                                             "coarse-pass and network starts on held-out observations.")
    ap.add_argument("--n-ant", type=int, default=256)
    ap.add_argument("--n-chan", type=int, default=4096)
    ap.add_argument("--bin-width", type=int, default=64)
    ap.add_argument("--hidden", type=int, default=256)
    ap.add_argument("--halfwidth", type=int, default=0)
    ap.add_argument("--coarse-tol", type=float, default=1e-4)
    ap.add_argument("--n-train", type=int, default=200)
    ap.add_argument("--n-test", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=500)
    ap.add_argument("--knots-only", action="store_true",
                    help="generate the training observations at the knot channels only (the targets are "
                         "the unit-start solutions there, as in a full solve; needs --halfwidth 0)")
    ap.add_argument("--out-json", default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    dev = torch.device("cuda", 0)
    P0 = synth.bandpass_di(a.n_ant, a.n_chan, seed=1000, device=dev)
    plan = wcal.plan_for(P0, tol=a.tol, max_iter=a.max_iter)
    ws = WarmStart(plan, bin_width=a.bin_width, hidden=a.hidden, halfwidth=a.halfwidth,
                   coarse_tol=a.coarse_tol, seed=1, max_batch=max(a.batch, a.n_ant))
    log(f"training set: {a.n_train} observations of one sky, {a.n_ant} antennas x {a.n_chan} channels, "
        f"{ws.n_bins} knots")
    t0 = time.perf_counter()
    X, T = [], []
    n_bl = P0.ant1.numel()
    knots = ws.knots.long().to(dev)
    model_k = P0.model.view(a.n_chan, n_bl, 1, 1)[knots].reshape(-1, 1, 1).contiguous()
    for i in range(a.n_train):
        if a.knots_only:
            P = synth.bandpass_di(a.n_ant, a.n_chan, seed=1000 + i, device=dev, model=model_k,
                                  channels=ws.knots.tolist())
            f, t, ok = ws.make_example_knots(P)
        else:
            P = P0 if i == 0 else synth.bandpass_di(a.n_ant, a.n_chan, seed=1000 + i, device=dev, model=P0.model)
            f, t, ok = ws.make_example(P)
        if ok:
            X.append(f)
            T.append(t)
        del P
        if (i + 1) % max(1, a.n_train // 10) == 0:
            torch.cuda.synchronize()
            log(f"  {i + 1}/{a.n_train} observations ({time.perf_counter() - t0:.1f} s)")
    X, T = torch.cat(X).contiguous(), torch.cat(T).contiguous()
    t_data = time.perf_counter() - t0
    identity_mse = float(((X - T) ** 2).mean())
    t0 = time.perf_counter()
    losses = ws.train(X, T, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=0)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"trained {a.epochs} epochs on {X.shape[0]} antenna examples in {t_train:.1f} s: "
        f"loss {losses[0]:.3e} -> {losses[-1]:.3e} (identity {identity_mse:.3e})")
    rows = {k: [] for k in ("unit", "coarse", "mlp")}
    diff = []
    for j in range(a.n_test):
        P = synth.bandpass_di(a.n_ant, a.n_chan, seed=900000 + j, device=dev, model=P0.model)
        r = evaluate(ws, P)
        for k in rows:
            rows[k].append(r[k])
        log(f"  held-out {j}: " + ", ".join(
            f"{k} {r[k]['mean_iter']:.2f} it {r[k]['ms']:.1f} ms fb {r[k]['fallback']}" for k in rows))
        # warm and unit starts reach the same solution up to one phase per channel
        gw, gu = r["mlp"]["gains"][:, 0, :, 0], r["unit"]["gains"][:, 0, :, 0]
        ph = (gw.conj() * gu).sum(1, keepdim=True)
        gw = gw * ph / ph.abs()
        diff.append(float(((gw - gu).abs().pow(2).sum(1) / gu.abs().pow(2).sum(1)).sqrt().max()))
        for k in r:
            r[k].pop("gains")
        del P
    d_mc = [x["mean_iter"] - y["mean_iter"] for x, y in zip(rows["mlp"], rows["coarse"])]
    summary = dict(workload=f"bandpass_na{a.n_ant}", n_chan=a.n_chan, bin_width=a.bin_width,
                   knots_only=a.knots_only,
                   mlp_minus_coarse_iter=dict(mean=statistics.mean(d_mc),
                                              stdev=statistics.stdev(d_mc) if len(d_mc) > 1 else 0.0,
                                              min=min(d_mc), max=max(d_mc)),
                   n_knots=ws.n_bins, hidden=a.hidden, halfwidth=a.halfwidth, coarse_tol=a.coarse_tol,
                   n_train=a.n_train, n_test=a.n_test, epochs=a.epochs, examples=int(X.shape[0]),
                   data_s=round(t_data, 2), train_s=round(t_train, 2), loss_first=losses[0],
                   loss_last=losses[-1], identity_mse=identity_mse, tol=a.tol,
                   warm_vs_unit_rel_diff_max=max(diff))
    for k, v in rows.items():
        summary[k] = dict(mean_iter=statistics.mean(x["mean_iter"] for x in v),
                          stdev_iter=statistics.stdev(x["mean_iter"] for x in v) if len(v) > 1 else 0.0,
                          median_iter=statistics.median(x["median_iter"] for x in v),
                          coarse_iter=statistics.mean(x["coarse_iter"] for x in v),
                          ms_median=statistics.median(x["ms"] for x in v),
                          fallback_rate=sum(x["fallback"] for x in v) / (len(v) * a.n_chan),
                          converged_rate=sum(x["converged"] for x in v) / (len(v) * a.n_chan))
    log(json.dumps(summary))
    if a.out_json:
        with open(a.out_json, "w") as fh:
            json.dump(summary, fh, indent=1)


if __name__ == "__main__":
    main()
