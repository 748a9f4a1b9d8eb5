"""Seeded synthetic calibration problems (inputs only).

This module draws the inputs of a calibration run: antenna-pair tables, ragged
solution intervals, sky coherencies (model visibilities), true gains, noise,
flags, and the observed data that the measurement equation produces from them
(scalar RIME of Sect. 2.1, polarized RIME of Sect. 4, direction-dependent sum of
Sect. 2.5).  It contains no part of the calibration method itself: no Jacobian
products, no normal equations, no solves.  Both the GPU path and the CPU oracle
take their inputs from here; neither is imported by this module.

Row layout (shared by every consumer):
  interval k owns rows [row_off[k], row_off[k+1]), with n_bl * ns[k] rows,
  ordered sample-major: row = row_off[k] + s * n_bl + b  (s < ns[k], b < n_bl).
  data  : [rows, n_corr]            complex
  model : [rows, n_dir, n_corr]     complex
  flags : [rows] uint8 (nonzero = flagged, all correlations) or None
  gains : [n_int, n_dir, n_ant, n_corr] complex, n_corr = 4 means a 2x2 Jones
          matrix stored row-major (xx, xy, yx, yy).

All random draws come from one torch.Generator seeded per problem, on the
device the problem is built on.  Complex Gaussians CN(0, v) have E|z|^2 = v;
"sigma" is the complex standard deviation (E|n|^2 = sigma^2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

SEED_BASE = 150206974


@dataclass
class Problem:
    n_ant: int
    n_dir: int
    n_corr: int
    ant1: torch.Tensor          # int32 [n_bl]
    ant2: torch.Tensor          # int32 [n_bl]
    ns: torch.Tensor            # int64 [n_int]  samples per baseline per interval
    row_off: torch.Tensor       # int64 [n_int + 1]
    data: torch.Tensor          # complex [rows, n_corr]
    model: torch.Tensor         # complex [rows, n_dir, n_corr]
    flags: Optional[torch.Tensor]  # uint8 [rows] or None
    g_true: torch.Tensor        # complex [n_int, n_dir, n_ant, n_corr]
    meta: dict = field(default_factory=dict)

    @property
    def n_bl(self) -> int:
        return int(self.ant1.numel())

    @property
    def n_int(self) -> int:
        return int(self.ns.numel())

    @property
    def n_rows(self) -> int:
        return int(self.row_off[-1])

    def unit_gains(self) -> torch.Tensor:
        """Unit (identity) starting gains in the gains layout."""
        g = torch.zeros(self.n_int, self.n_dir, self.n_ant, self.n_corr,
                        dtype=self.data.dtype, device=self.data.device)
        if self.n_corr == 1:
            g[..., 0] = 1
        else:
            g[..., 0] = 1
            g[..., 3] = 1
        return g

    def interval(self, k: int) -> dict:
        """Interval k as host numpy complex128 arrays with per-row antenna indices."""
        a, b = int(self.row_off[k]), int(self.row_off[k + 1])
        ns = int(self.ns[k])
        nbl = self.n_bl
        a1 = self.ant1.cpu().numpy().astype(np.int64)
        a2 = self.ant2.cpu().numpy().astype(np.int64)
        p = np.tile(a1, ns)
        q = np.tile(a2, ns)
        d = self.data[a:b].cpu().numpy().astype(np.complex128)
        m = self.model[a:b].cpu().numpy().astype(np.complex128)
        f = (np.zeros(b - a, dtype=bool) if self.flags is None
             else self.flags[a:b].cpu().numpy() != 0)
        assert d.shape[0] == nbl * ns
        return dict(d=d, m=m, p=p, q=q, flags=f, ns=ns,
                    g_true=self.g_true[k].cpu().numpy().astype(np.complex128))


def baselines(n_ant: int, device="cpu"):
    """All pairs p<q in p-major order (12, 13, ..., 1n, 23, ...)."""
    p, q = np.triu_indices(n_ant, k=1)
    return (torch.tensor(p, dtype=torch.int32, device=device),
            torch.tensor(q, dtype=torch.int32, device=device))


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _cn(shape, var, gen, device, dtype):
    """Circular complex Gaussian CN(0, var): E|z|^2 = var."""
    z = torch.randn(*shape, generator=gen, device=device, dtype=dtype)
    return z * math.sqrt(var) if var != 1.0 else z


def _diag_gain(shape, gen, device, dtype, amp_sigma=0.1):
    """amplitude exp(N(0, amp_sigma^2)), phase U(-pi, pi)."""
    rdt = torch.float64 if dtype == torch.complex128 else torch.float32
    amp = torch.exp(amp_sigma * torch.randn(*shape, generator=gen, device=device, dtype=rdt))
    ph = (torch.rand(*shape, generator=gen, device=device, dtype=rdt) * 2 - 1) * math.pi
    return torch.polar(amp, ph).to(dtype)


def _row_offsets(ns: torch.Tensor, n_bl: int) -> torch.Tensor:
    off = torch.zeros(ns.numel() + 1, dtype=torch.int64)
    off[1:] = torch.cumsum(ns.to(torch.int64).cpu() * n_bl, 0)
    return off


def _rows_chunks(ns_cpu: np.ndarray, n_bl: int, max_rows: int):
    """Split the interval list into contiguous chunks of at most ~max_rows rows."""
    start = 0
    acc = 0
    for k, n in enumerate(ns_cpu):
        r = int(n) * n_bl
        if acc and acc + r > max_rows:
            yield start, k
            start, acc = k, 0
        acc += r
    if start < len(ns_cpu):
        yield start, len(ns_cpu)


def _forward(model, gains, ant1, ant2, ns, row_off, n_corr, dtype, max_rows=1 << 25):
    """Observed visibilities from the measurement equation: for every row,
    sum over directions of G_p M G_q^H (scalar: g_p m conj(g_q))."""
    rows = model.shape[0]
    device = model.device
    out = torch.zeros(rows, n_corr, dtype=dtype, device=device)
    n_bl = ant1.numel()
    ns_cpu = ns.cpu().numpy()
    a1 = ant1.long()
    a2 = ant2.long()
    for k0, k1 in _rows_chunks(ns_cpu, n_bl, max_rows):
        r0, r1 = int(row_off[k0]), int(row_off[k1])
        nsk = torch.tensor(ns_cpu[k0:k1], device=device)
        kidx = torch.repeat_interleave(torch.arange(k0, k1, device=device), nsk * n_bl)
        bidx = (torch.arange(r1 - r0, device=device)
                - torch.repeat_interleave(row_off[k0:k1].to(device) - r0, nsk * n_bl)) % n_bl
        p = a1[bidx]
        q = a2[bidx]
        m = model[r0:r1]                                  # [r, nd, nc]
        # per-row gains gains[k, :, ant, :] -> [r, nd, nc]
        g_p = gains[kidx, :, p, :]
        g_q = gains[kidx, :, q, :]
        if n_corr == 1:
            v = (g_p * m * g_q.conj()).sum(1)
        else:
            Gp = g_p.view(-1, gains.shape[1], 2, 2)
            Gq = g_q.view(-1, gains.shape[1], 2, 2)
            M = m.view(-1, gains.shape[1], 2, 2)
            v = torch.matmul(torch.matmul(Gp, M), Gq.conj().transpose(-1, -2).contiguous()).sum(1).reshape(-1, 4)
        out[r0:r1] = v
        del g_p, g_q, m, v, kidx, bidx, p, q
    return out


def _finish(n_ant, n_dir, n_corr, ant1, ant2, ns, model, gains, sigma, flag_frac, gen,
            device, dtype, meta, noise=True):
    n_bl = ant1.numel()
    row_off = _row_offsets(ns, n_bl)
    rows = int(row_off[-1])
    data = _forward(model, gains, ant1, ant2, ns, row_off.to(device), n_corr, dtype)
    if noise and sigma > 0:
        data += _cn((rows, n_corr), sigma * sigma, gen, device, dtype)
    flags = None
    if flag_frac > 0:
        flags = (torch.rand(rows, generator=gen, device=device) < flag_frac).to(torch.uint8)
    return Problem(n_ant=n_ant, n_dir=n_dir, n_corr=n_corr, ant1=ant1, ant2=ant2,
                   ns=ns.cpu().to(torch.int64), row_off=row_off, data=data, model=model,
                   flags=flags, g_true=gains, meta=meta)


def scalar_di(n_ant: int, ns: Sequence[int], sigma: float = 0.01, seed: int = 0,
              flag_frac: float = 0.0, device="cpu", dtype=torch.complex64,
              noise: bool = True) -> Problem:
    """Scalar direction-independent problem: m ~ CN(0,1) i.i.d. per row,
    g = exp(N(0, 0.1^2)) * exp(i U(-pi, pi)) per (interval, antenna),
    d = g_p m conj(g_q) + CN(0, sigma^2)."""
    gen = _gen(SEED_BASE * 16 + 1 + 7919 * seed, device)
    ant1, ant2 = baselines(n_ant, device)
    ns = torch.as_tensor(list(ns), dtype=torch.int64)
    n_int = ns.numel()
    rows = int(ns.sum()) * ant1.numel()
    gains = _diag_gain((n_int, 1, n_ant, 1), gen, device, dtype)
    model = _cn((rows, 1, 1), 1.0, gen, device, dtype)
    return _finish(n_ant, 1, 1, ant1, ant2, ns, model, gains, sigma, flag_frac, gen, device,
                   dtype, dict(kind="scalar_di", sigma=sigma, seed=seed), noise)


def pol_di(n_ant: int, ns: Sequence[int], sigma: float = 0.01, leak: float = 0.1, seed: int = 0,
           flag_frac: float = 0.0, device="cpu", dtype=torch.complex64,
           noise: bool = True) -> Problem:
    """Full-polarization 2x2 problem: G_p = [[g_x, l_xy], [l_yx, g_y]] with g_x, g_y
    drawn as in scalar_di and leakages l ~ CN(0, leak^2); every 2x2 entry of M is
    CN(0,1) i.i.d. (a generic coherency, so the only gauge freedom is one global phase);
    D = G_p M G_q^H + CN(0, sigma^2) per correlation."""
    gen = _gen(SEED_BASE * 16 + 2 + 7919 * seed, device)
    ant1, ant2 = baselines(n_ant, device)
    ns = torch.as_tensor(list(ns), dtype=torch.int64)
    n_int = ns.numel()
    rows = int(ns.sum()) * ant1.numel()
    gains = torch.zeros(n_int, 1, n_ant, 4, dtype=dtype, device=device)
    gains[..., 0] = _diag_gain((n_int, 1, n_ant), gen, device, dtype)
    gains[..., 3] = _diag_gain((n_int, 1, n_ant), gen, device, dtype)
    gains[..., 1] = _cn((n_int, 1, n_ant), leak * leak, gen, device, dtype)
    gains[..., 2] = _cn((n_int, 1, n_ant), leak * leak, gen, device, dtype)
    model = _cn((rows, 1, 4), 1.0, gen, device, dtype)
    return _finish(n_ant, 1, 4, ant1, ant2, ns, model, gains, sigma, flag_frac, gen, device,
                   dtype, dict(kind="pol_di", sigma=sigma, leak=leak, seed=seed), noise)


def pol_dd(n_ant: int, ns: Sequence[int], n_dir: int, sigma: float = 0.03, leak: float = 0.1,
           seed: int = 0, flag_frac: float = 0.0, device="cpu", dtype=torch.complex64,
           noise: bool = True, pairs=None) -> Problem:
    """Polarized direction-dependent problem (Sect. 4.4) with the 2x2 recipe of pol_di per
    direction: G^d_p = [[g_x, l_xy], [l_yx, g_y]], g drawn as in scalar_di, leakages
    CN(0, leak^2); every 2x2 entry of every M^d is CN(0, 1) i.i.d. (generic coherencies,
    so the only gauge is one phase per direction); D = sum_d G^d_p M^d G^{dH}_q plus
    CN(0, sigma^2) per correlation.  pairs = (ant1, ant2) replaces the table of all p < q
    (pairs may repeat)."""
    gen = _gen(SEED_BASE * 16 + 6 + 7919 * seed, device)
    if pairs is None:
        ant1, ant2 = baselines(n_ant, device)
    else:
        ant1 = torch.as_tensor(pairs[0], dtype=torch.int32, device=device)
        ant2 = torch.as_tensor(pairs[1], dtype=torch.int32, device=device)
    ns = torch.as_tensor(list(ns), dtype=torch.int64)
    n_int = ns.numel()
    rows = int(ns.sum()) * ant1.numel()
    gains = torch.zeros(n_int, n_dir, n_ant, 4, dtype=dtype, device=device)
    gains[..., 0] = _diag_gain((n_int, n_dir, n_ant), gen, device, dtype)
    gains[..., 3] = _diag_gain((n_int, n_dir, n_ant), gen, device, dtype)
    gains[..., 1] = _cn((n_int, n_dir, n_ant), leak * leak, gen, device, dtype)
    gains[..., 2] = _cn((n_int, n_dir, n_ant), leak * leak, gen, device, dtype)
    model = _cn((rows, n_dir, 4), 1.0, gen, device, dtype)
    return _finish(n_ant, n_dir, 4, ant1, ant2, ns, model, gains, sigma, flag_frac, gen, device,
                   dtype, dict(kind="pol_dd", sigma=sigma, leak=leak, seed=seed), noise)


def ragged_ns(n_int: int, t_max: int = 30, f_max: int = 16, seed: int = 0) -> list:
    """Interval sizes Ns_k = T_k * F_k with T ~ U{1..t_max}, F ~ U{1..f_max}."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, 1, seed])))
    t = rng.integers(1, t_max + 1, size=n_int)
    f = rng.integers(1, f_max + 1, size=n_int)
    return (t * f).tolist()


def bandpass_di(n_ant: int, n_chan: int, sigma: float = 0.05, seed: int = 0,
                flag_frac: float = 0.0, device="cpu", dtype=torch.complex64,
                nu_lo: float = 100e6, nu_hi: float = 200e6, noise: bool = True,
                model: Optional[torch.Tensor] = None, channels: Optional[Sequence[int]] = None) -> Problem:
    """Scalar problem with one interval per channel (Ns = 1): per antenna, amplitude is a
    cubic polynomial c0 + c1 x + c2 x^2 + c3 x^3 over x in [-1, 1] across the band with
    c0 = exp(N(0, 0.1^2)), c1..c3 ~ N(0, 0.05^2); phase phi0 + 2 pi tau (nu - nu_mid)
    with phi0 ~ U(-pi, pi), tau ~ U(-50, 50) ns.  m ~ CN(0,1), noise CN(0, sigma^2).
    A given `model` [rows, 1, 1] is reused instead of drawing a new one (many observations
    of the same sky with fresh gains and noise).  With `channels`, only those channels of
    the n_chan-channel band are generated (one interval each, in the given order; `model`
    then holds their rows only)."""
    gen = _gen(SEED_BASE * 16 + 3 + 7919 * seed, device)
    ant1, ant2 = baselines(n_ant, device)
    f64 = torch.float64
    nu = nu_lo + (torch.arange(n_chan, device=device, dtype=f64) + 0.5) * (nu_hi - nu_lo) / n_chan
    if channels is not None:
        nu = nu[torch.as_tensor(channels, dtype=torch.int64, device=device)]
    n_chan = nu.numel()
    ns = torch.ones(n_chan, dtype=torch.int64)
    rows = n_chan * ant1.numel()
    nu_mid = 0.5 * (nu_lo + nu_hi)
    x = 2 * (nu - nu_mid) / (nu_hi - nu_lo)
    c0 = torch.exp(0.1 * torch.randn(n_ant, generator=gen, device=device, dtype=f64))
    c = 0.05 * torch.randn(3, n_ant, generator=gen, device=device, dtype=f64)
    phi0 = (torch.rand(n_ant, generator=gen, device=device, dtype=f64) * 2 - 1) * math.pi
    tau = (torch.rand(n_ant, generator=gen, device=device, dtype=f64) * 2 - 1) * 50e-9
    amp = c0[None] + c[0][None] * x[:, None] + c[1][None] * x[:, None] ** 2 + c[2][None] * x[:, None] ** 3
    ph = phi0[None] + 2 * math.pi * tau[None] * (nu[:, None] - nu_mid)
    gains = torch.polar(amp, ph).to(dtype).view(n_chan, 1, n_ant, 1)
    if model is None:
        model = _cn((rows, 1, 1), 1.0, gen, device, dtype)
    else:
        assert tuple(model.shape) == (rows, 1, 1)
    return _finish(n_ant, 1, 1, ant1, ant2, ns, model, gains, sigma, flag_frac, gen, device,
                   dtype, dict(kind="bandpass_di", sigma=sigma, seed=seed, nu=nu.cpu()), noise)


C_LIGHT = 299792458.0


def _array_geometry(n_ant, gen, device, disk_diam, lat_deg):
    """Antennas uniform in a planar disk of diameter disk_diam (east, north), rotated to
    local equatorial XYZ at array latitude lat_deg."""
    f64 = torch.float64
    r = 0.5 * disk_diam * torch.sqrt(torch.rand(n_ant, generator=gen, device=device, dtype=f64))
    th = 2 * math.pi * torch.rand(n_ant, generator=gen, device=device, dtype=f64)
    east, north = r * torch.cos(th), r * torch.sin(th)
    lat = math.radians(lat_deg)
    return (-math.sin(lat) * north, east, math.cos(lat) * north)


def _uvw(geo, ant1, ant2, k, n_time, n_int, dt, dec_deg, device):
    """u, v, w [n_time, n_bl] in metres for interval k: n_time timeslots of dt seconds in a
    contiguous hour-angle block (the textbook XYZ -> uvw rotation at declination dec)."""
    f64 = torch.float64
    X, Y, Z = geo
    dec = math.radians(dec_deg)
    omega = 2 * math.pi / 86164.0905
    H = (k * n_time + torch.arange(n_time, device=device, dtype=f64) - 0.5 * n_int * n_time) * dt * omega
    bx = X[ant2.long()] - X[ant1.long()]
    by = Y[ant2.long()] - Y[ant1.long()]
    bz = Z[ant2.long()] - Z[ant1.long()]
    sH, cH = torch.sin(H)[:, None], torch.cos(H)[:, None]
    u = sH * bx[None] + cH * by[None]
    v = -math.sin(dec) * cH * bx[None] + math.sin(dec) * sH * by[None] + math.cos(dec) * bz[None]
    w = math.cos(dec) * cH * bx[None] - math.cos(dec) * sH * by[None] + math.sin(dec) * bz[None]
    return u, v, w


def _power_law(n, lo, hi, index, gen, device):
    """n fluxes with dN/dS ~ S^index on [lo, hi] (inverse-CDF draw)."""
    a1 = index + 1.0
    uu = torch.rand(n, generator=gen, device=device, dtype=torch.float64)
    return (lo ** a1 + uu * (hi ** a1 - lo ** a1)) ** (1.0 / a1)


def dd_point(n_ant: int = 64, n_dir: int = 10, n_time: int = 30, n_chan: int = 64, n_int: int = 1,
             seed: int = 0, device="cpu", dtype=torch.complex64, noise_frac: float = 0.01,
             dt: float = 10.0, disk_diam: float = 5000.0, lat_deg: float = 52.0, dec_deg: float = 52.0,
             nu_lo: float = 100e6, nu_hi: float = 200e6, fov_deg: float = 1.0,
             flux_lo: float = 0.1, flux_hi: float = 10.0, flux_index: float = -1.5,
             noise: bool = True, smooth_gains: bool = True, flag_frac: float = 0.0) -> Problem:
    """Direction-dependent problem built from point sources (the point-source
    coherency of Sect. 3.2.1): per direction d a source at (l, m) ~ U(+-fov)
    with flux S drawn from a power law dN/dS ~ S^flux_index on [flux_lo, flux_hi];
    m^d_pq(t, nu) = S_d exp(-2 pi i (u l + v m + w (n - 1)) nu / c).
    Antennas are uniform in a planar disk of diameter disk_diam; uvw follow the
    textbook ENU -> (u, v, w) rotation at hour angle H and declination dec, with
    array latitude lat.  Interval k covers n_time timeslots of dt seconds at a
    contiguous hour-angle block and all n_chan channels over [nu_lo, nu_hi].
    Gains per (interval, direction, antenna): amplitude exp(N(0, 0.1^2)) and
    phase U(-pi, pi); with smooth_gains they drift smoothly across intervals.
    Noise is CN(0, (noise_frac * sum_d S_d)^2).  meta holds the inputs of the model: uvw
    [n_int][n_time][n_bl][3] (metres, ant2 - ant1), lmn [n_dir][3] (l, m, n - 1), flux, and the
    channel grid freq0 + f * dfreq."""
    gen = _gen(SEED_BASE * 16 + 4 + 7919 * seed, device)
    f64 = torch.float64
    ant1, ant2 = baselines(n_ant, device)
    n_bl = ant1.numel()
    geo = _array_geometry(n_ant, gen, device, disk_diam, lat_deg)
    # sources
    fov = math.radians(fov_deg)
    l = (torch.rand(n_dir, generator=gen, device=device, dtype=f64) * 2 - 1) * fov
    mm = (torch.rand(n_dir, generator=gen, device=device, dtype=f64) * 2 - 1) * fov
    n = torch.sqrt(1 - l * l - mm * mm)
    flux = _power_law(n_dir, flux_lo, flux_hi, flux_index, gen, device)
    nu = nu_lo + (torch.arange(n_chan, device=device, dtype=f64) + 0.5) * (nu_hi - nu_lo) / n_chan
    ns = torch.full((n_int,), n_time * n_chan, dtype=torch.int64)
    rows = n_int * n_time * n_chan * n_bl
    model = torch.empty(rows, n_dir, 1, dtype=dtype, device=device)
    uvw = torch.empty(n_int, n_time, n_bl, 3, dtype=f64, device=device)
    for k in range(n_int):
        u, v, w = _uvw(geo, ant1, ant2, k, n_time, n_int, dt, dec_deg, device)
        uvw[k, ..., 0], uvw[k, ..., 1], uvw[k, ..., 2] = u, v, w
        # phase[t, b, d] per unit frequency
        ph = (u[..., None] * l + v[..., None] * mm + w[..., None] * (n - 1)) / C_LIGHT
        # rows ordered [s][bl] with s = t * n_chan + f
        arg = -2 * math.pi * ph[:, None, :, :] * nu[None, :, None, None]   # [t, f, b, d]
        mk = flux * torch.polar(torch.ones_like(arg), arg)
        r0 = k * n_time * n_chan * n_bl
        model[r0:r0 + n_time * n_chan * n_bl, :, 0] = mk.reshape(-1, n_dir).to(dtype)
    amp = torch.exp(0.1 * torch.randn(n_dir, n_ant, generator=gen, device=device, dtype=f64))
    ph0 = (torch.rand(n_dir, n_ant, generator=gen, device=device, dtype=f64) * 2 - 1) * math.pi
    if smooth_gains and n_int > 1:
        # slow drift across intervals: a random linear phase rate and amplitude slope
        rate = 0.3 * torch.randn(n_dir, n_ant, generator=gen, device=device, dtype=f64)
        slope = 0.02 * torch.randn(n_dir, n_ant, generator=gen, device=device, dtype=f64)
        x = torch.linspace(-1, 1, n_int, device=device, dtype=f64)[:, None, None]
        gains = torch.polar(amp[None] * (1 + slope[None] * x), ph0[None] + rate[None] * x)
    else:
        gains = torch.polar(amp, ph0)[None].expand(n_int, -1, -1)
    gains = gains.to(dtype).reshape(n_int, n_dir, n_ant, 1).contiguous()
    sigma = noise_frac * float(flux.sum())
    meta = dict(kind="dd_point", seed=seed, l=l.cpu(), m=mm.cpu(), flux=flux.cpu(), sigma=sigma,
                uvw=uvw, lmn=torch.stack([l, mm, n - 1], dim=1), n_time=n_time, n_chan=n_chan,
                freq0=nu_lo + 0.5 * (nu_hi - nu_lo) / n_chan, dfreq=(nu_hi - nu_lo) / n_chan)
    return _finish(n_ant, n_dir, 1, ant1, ant2, ns, model, gains, sigma, flag_frac, gen, device,
                   dtype, meta, noise)


def dd_point_pol(n_ant: int = 64, n_dir: int = 10, n_time: int = 30, n_chan: int = 64, n_int: int = 1,
                 seed: int = 0, device="cpu", dtype=torch.complex64, noise_frac: float = 0.01,
                 dt: float = 10.0, disk_diam: float = 5000.0, lat_deg: float = 52.0, dec_deg: float = 52.0,
                 nu_lo: float = 100e6, nu_hi: float = 200e6, fov_deg: float = 1.0,
                 n_comp: int = 3, cluster_deg: float = 0.05, pol_frac: float = 0.3, leak: float = 0.1,
                 xy_phase: float = 0.2,
                 flux_lo: float = 0.1, flux_hi: float = 10.0, flux_index: float = -1.5,
                 noise: bool = True, smooth_gains: bool = True, flag_frac: float = 0.0) -> Problem:
    """Polarized direction-dependent sky (Sect. 4.4) on the geometry of dd_point.
    Direction d is a cluster of n_comp point sources: centre (l, m) ~ U(+-fov), each
    component offset by U(+-cluster_deg) in l and m, with flux I from the same power
    law and brightness B = [[I + Q, U + iV], [U - iV, I - Q]], (Q, U, V) / I each
    U(+-pol_frac).  M^d_pq(t, nu) = sum_c B_c exp(-2 pi i (u l_c + v m_c + w (n_c - 1)) nu / c),
    stored row-major (xx, xy, yx, yy).  The gauge of G^d -> G^d X is the set of X with
    X B_c X^H = B_c for every component: for one positive-definite B a copy of U(2), for
    two a pair of phases (both forms diagonalise under one congruence), for three or more
    generic components one phase per direction.  Weakly polarized clusters leave those
    directions only weakly determined, and the per-antenna updates then converge slowly.
    Gains per (interval, direction, antenna): a phase screen common to both feeds,
    U(-pi, pi) (drifting smoothly across intervals with smooth_gains), feed amplitudes
    exp(N(0, 0.1^2)), a differential phase N(0, xy_phase^2) split between the feeds and
    off-diagonal leakage CN(0, leak^2).  Noise per correlation CN(0, (noise_frac * sum of
    fluxes)^2)."""
    gen = _gen(SEED_BASE * 16 + 5 + 7919 * seed, device)
    f64 = torch.float64
    ant1, ant2 = baselines(n_ant, device)
    n_bl = ant1.numel()
    geo = _array_geometry(n_ant, gen, device, disk_diam, lat_deg)
    fov, cl = math.radians(fov_deg), math.radians(cluster_deg)
    lc = (torch.rand(n_dir, generator=gen, device=device, dtype=f64) * 2 - 1) * fov
    mc = (torch.rand(n_dir, generator=gen, device=device, dtype=f64) * 2 - 1) * fov
    l = lc[:, None] + (torch.rand(n_dir, n_comp, generator=gen, device=device, dtype=f64) * 2 - 1) * cl
    mm = mc[:, None] + (torch.rand(n_dir, n_comp, generator=gen, device=device, dtype=f64) * 2 - 1) * cl
    n = torch.sqrt(1 - l * l - mm * mm)
    flux = _power_law(n_comp * n_dir, flux_lo, flux_hi, flux_index, gen, device).reshape(n_dir, n_comp)
    qu = (torch.rand(n_dir, n_comp, 3, generator=gen, device=device, dtype=f64) * 2 - 1) * pol_frac * flux[..., None]
    B = torch.empty(n_dir, n_comp, 2, 2, dtype=torch.complex128, device=device)    # [d, c, 2, 2]
    B[..., 0, 0] = flux + qu[..., 0]
    B[..., 1, 1] = flux - qu[..., 0]
    B[..., 0, 1] = torch.complex(qu[..., 1], qu[..., 2])
    B[..., 1, 0] = torch.complex(qu[..., 1], -qu[..., 2])
    nu = nu_lo + (torch.arange(n_chan, device=device, dtype=f64) + 0.5) * (nu_hi - nu_lo) / n_chan
    ns = torch.full((n_int,), n_time * n_chan, dtype=torch.int64)
    rows = n_int * n_time * n_chan * n_bl
    model = torch.empty(rows, n_dir, 4, dtype=dtype, device=device)
    Bf = B.reshape(n_dir, n_comp, 4)
    for k in range(n_int):
        u, v, w = _uvw(geo, ant1, ant2, k, n_time, n_int, dt, dec_deg, device)
        r0 = k * n_time * n_chan * n_bl
        for t in range(n_time):
            # phase [b, d, c] per unit frequency, then [f, b, d, c]
            ph = (u[t, :, None, None] * l + v[t, :, None, None] * mm + w[t, :, None, None] * (n - 1)) / C_LIGHT
            arg = -2 * math.pi * ph[None] * nu[:, None, None, None]
            z = torch.polar(torch.ones_like(arg), arg)                           # [f, b, d, c]
            mk = torch.einsum("fbdc,dce->fbde", z, Bf)                           # [f, b, d, 4]
            a = r0 + t * n_chan * n_bl
            model[a:a + n_chan * n_bl] = mk.reshape(-1, n_dir, 4).to(dtype)
    # a phase common to both feeds (U(-pi, pi) per direction and antenna, drifting smoothly
    # across intervals), feed amplitudes exp(N(0, 0.1^2)), a differential phase N(0, xy^2)
    # between the feeds and leakage CN(0, leak^2)
    amp = torch.exp(0.1 * torch.randn(n_dir, n_ant, 2, generator=gen, device=device, dtype=f64))
    ph0 = (torch.rand(n_dir, n_ant, 1, generator=gen, device=device, dtype=f64) * 2 - 1) * math.pi
    ph0 = ph0 + xy_phase * torch.randn(n_dir, n_ant, 2, generator=gen, device=device, dtype=f64) * \
        torch.tensor([0.5, -0.5], device=device, dtype=f64)
    lk = _cn((n_dir, n_ant, 2), leak * leak, gen, device, torch.complex128)
    if smooth_gains and n_int > 1:
        rate = 0.3 * torch.randn(n_dir, n_ant, 1, generator=gen, device=device, dtype=f64)
        slope = 0.02 * torch.randn(n_dir, n_ant, 2, generator=gen, device=device, dtype=f64)
        x = torch.linspace(-1, 1, n_int, device=device, dtype=f64)[:, None, None, None]
        diag = torch.polar(amp[None] * (1 + slope[None] * x), ph0[None] + rate[None] * x)
    else:
        diag = torch.polar(amp, ph0)[None].expand(n_int, -1, -1, -1)
    gains = torch.empty(n_int, n_dir, n_ant, 4, dtype=torch.complex128, device=device)
    gains[..., 0] = diag[..., 0]
    gains[..., 3] = diag[..., 1]
    gains[..., 1] = lk[None, ..., 0]
    gains[..., 2] = lk[None, ..., 1]
    gains = gains.to(dtype).contiguous()
    sigma = noise_frac * float(flux.sum())
    meta = dict(kind="dd_point_pol", seed=seed, l=l.cpu(), m=mm.cpu(), B=B.cpu(), sigma=sigma)
    return _finish(n_ant, n_dir, 4, ant1, ant2, ns, model, gains, sigma, flag_frac, gen, device,
                   dtype, meta, noise)


# ---------------------------------------------------------------- workload presets
def workload(name: str, device="cpu", dtype=torch.complex64, **kw) -> Problem:
    """Named workloads with the shapes of the measured configurations.

    scalar_na27     : Na=27, 351 baselines, one interval of 60 x 4 samples, sigma 0.01
    pol2x2_na64     : Na=64, 2016 baselines, 1000 ragged intervals (T~U{1..30} x F~U{1..16}),
                      5% flags, 2x2 Jones with 0.1 leakage, sigma 0.01
    cohjones_na64   : Na=64, Nd=10 point-source directions, 30 x 64 samples per interval
    pol_cohjones_na64 : Na=64, Nd=10, 2x2 Jones, 16 intervals of 30 x 64 samples, i.i.d.
                      CN(0,1) coherencies per direction (the 2x2 recipe), sigma 0.03
    bandpass_na256  : Na=256, 32640 baselines, 4096 channels solved independently (Ns=1), sigma 0.05
    """
    if name == "scalar_na27":
        return scalar_di(27, [kw.pop("ns", 240)], sigma=0.01, device=device, dtype=dtype, **kw)
    if name == "pol2x2_na64":
        n_int = kw.pop("n_int", 1000)
        ns = kw.pop("ns", None) or ragged_ns(n_int, seed=kw.get("seed", 0))
        return pol_di(64, ns, sigma=0.01, leak=0.1, flag_frac=kw.pop("flag_frac", 0.05),
                      device=device, dtype=dtype, **kw)
    if name == "cohjones_na64":
        return dd_point(64, 10, device=device, dtype=dtype, **kw)
    if name == "pol_cohjones_na64":
        n_int = kw.pop("n_int", 16)
        return pol_dd(64, kw.pop("ns", None) or [30 * 64] * n_int, 10, device=device, dtype=dtype, **kw)
    if name == "bandpass_na256":
        return bandpass_di(256, kw.pop("n_chan", 4096), sigma=0.05, device=device, dtype=dtype, **kw)
    raise ValueError(name)
