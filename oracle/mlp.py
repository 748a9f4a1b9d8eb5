"""float64 reference of the warm-start network, its coarse pass and its bin <-> channel maps.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The warm start is not part of the paper; it sits in front of the scalar StefCal solve
(Sect. 3.1, Eq. stefcal) of many single-channel intervals and only chooses the starting
gains.  Its pieces:

Knots: channels are grouped in bins of bin_width consecutive intervals (the last bin may
be shorter); bin B = [lo, hi) has the knot channel lo + (hi - lo - 1) // 2.

Coarse pass: StefCal from unit gains on the knot channels only; its gains, referenced
to antenna 0 per channel (times conj(g_0)/|g_0|, the phase gauge), are the features,
laid out [n_ant][2 n_bins] (real parts of the bins, then imaginary parts).

Network: h1 = tanh(x W1 + b1), h2 = tanh(h1 W2 + b2), y = h2 W3 + b3 (+ x with the skip
connection) applied to rows x; loss is the mean squared error over every output of the
batch.  Parameters flat in the order W1 [d_in][d_h], b1, W2 [d_h][d_h], b2, W3 [d_h][d_out],
b3 (row-major).  Optimiser: Adam (Kingma & Ba 2015) with bias correction.

Targets: the solver's gains on every channel, referenced to antenna 0 per channel, averaged
over the channels within halfwidth of each knot.

Interpolation: from knot values to every channel, amplitude and phase linear between
neighbouring knots (the phase step between two knots is the principal argument of
z_{B+1} conj(z_B), so steps must stay below pi), constant beyond the outer knots.
"""
from __future__ import annotations

import numpy as np

from . import calib as oc


def sizes(d_in, d_h, d_out):
    return [(d_in, d_h), (d_h,), (d_h, d_h), (d_h,), (d_h, d_out), (d_out,)]


def unpack(theta, d_in, d_h, d_out):
    out, o = [], 0
    for shp in sizes(d_in, d_h, d_out):
        n = int(np.prod(shp))
        out.append(theta[o:o + n].reshape(shp))
        o += n
    return out


def n_params(d_in, d_h, d_out):
    return sum(int(np.prod(s)) for s in sizes(d_in, d_h, d_out))


def forward(theta, x, d_in, d_h, d_out, skip=False):
    W1, b1, W2, b2, W3, b3 = unpack(theta, d_in, d_h, d_out)
    h1 = np.tanh(x @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    y = h2 @ W3 + b3
    if skip:
        y = y + x
    return y, (h1, h2)


def loss_and_grad(theta, x, t, d_in, d_h, d_out, skip=False):
    """Mean squared error and its gradient by backpropagation (the skip connection adds
    no parameters and so no gradient terms)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, d_in, d_h, d_out)
    y, (h1, h2) = forward(theta, x, d_in, d_h, d_out, skip)
    n = y.size
    loss = np.sum((y - t) ** 2) / n
    dy = 2.0 * (y - t) / n
    dW3 = h2.T @ dy
    db3 = dy.sum(0)
    dh2 = (dy @ W3.T) * (1 - h2 ** 2)
    dW2 = h1.T @ dh2
    db2 = dh2.sum(0)
    dh1 = (dh2 @ W2.T) * (1 - h1 ** 2)
    dW1 = x.T @ dh1
    db1 = dh1.sum(0)
    g = np.concatenate([a.ravel() for a in (dW1, db1, dW2, db2, dW3, db3)])
    return loss, g


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step count t starting at 1); returns new theta, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def knots(n_int, bin_width):
    n_bins = (n_int + bin_width - 1) // bin_width
    lo = np.arange(n_bins) * bin_width
    hi = np.minimum(lo + bin_width, n_int)
    return lo + (hi - lo - 1) // 2


def reference(g):
    """g [n_int][n_ant] -> g times conj(g_0)/|g_0| per channel (unchanged where g_0 = 0)."""
    a0 = np.abs(g[:, 0])
    ph = np.where(a0 > 0, np.conj(g[:, 0]) / np.where(a0 > 0, a0, 1.0), 1.0)
    return g * ph[:, None]


def pack(z):
    """complex [n_bins][n_ant] -> float [n_ant][2 n_bins]."""
    return np.concatenate([z.T.real, z.T.imag], axis=1)


def coarse_features(intervals, n_ant, bin_width, tol, max_iter):
    """intervals: list of dicts (d, m, p, q, flags) of single-channel intervals in channel
    order.  StefCal from unit gains on the knot channels; returns (features
    [n_ant][2 n_bins], per-knot oracle results)."""
    ks = knots(len(intervals), bin_width)
    g = np.zeros((len(ks), n_ant), dtype=np.complex128)
    res = []
    for i, k in enumerate(ks):
        iv = intervals[k]
        o = oc.stefcal_scalar(iv["d"], iv["m"], iv["p"], iv["q"], iv["flags"], np.ones(n_ant, complex),
                              tol=tol, max_iter=max_iter)
        g[i] = o["g"]
        res.append(o)
    return pack(reference(g)), res


def channels_to_bins(g, n_ant, bin_width, halfwidth):
    """Targets: gains [n_int][n_ant] referenced per channel, averaged over the channels
    within halfwidth of each knot; [n_ant][2 n_bins]."""
    n_int = g.shape[0]
    r = reference(g)
    ks = knots(n_int, bin_width)
    z = np.stack([r[max(0, k - halfwidth):min(n_int, k + halfwidth + 1)].mean(axis=0) for k in ks])
    return pack(z)


def bins_to_channels(y, n_ant, bin_width, n_int):
    """Knot values [n_ant][2 n_bins] -> gains [n_int][n_ant]: amplitude and phase linear
    between knots, constant beyond the outer knots."""
    ks = knots(n_int, bin_width)
    n_bins = len(ks)
    z = y[:, :n_bins] + 1j * y[:, n_bins:]
    amp = np.abs(z)
    ph = np.zeros_like(amp)
    ph[:, 0] = np.angle(z[:, 0])
    for B in range(1, n_bins):
        ph[:, B] = ph[:, B - 1] + np.angle(z[:, B] * np.conj(z[:, B - 1]))
    ch = np.arange(n_int)
    out = np.zeros((n_int, n_ant), dtype=np.complex128)
    for a in range(n_ant):
        out[:, a] = np.interp(ch, ks, amp[a]) * np.exp(1j * np.interp(ch, ks, ph[a]))
    return out
