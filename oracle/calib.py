"""Algorithm layer of the oracle: the per-antenna calibration updates.

TEST INFRASTRUCTURE ONLY (see the package docstring).  complex128 NumPy.

Every function takes one solution interval as a flat list of stored rows with
per-row antenna indices p, q (p != q; either orientation), following the
compound row index [pqs] of Sect. 2.3:
  scalar : d [R], m [R], gains g [Na]
  2x2    : D [R, 2, 2], M [R, 2, 2], gains G [Na, 2, 2]        (Sect. 4)
  DD     : d [R], m [R, Nd], gains g [Nd, Na]                  (Sect. 2.5)
  2x2 DD : D [R, 2, 2], M [R, Nd, 2, 2], gains G [Nd, Na, 2, 2] (Sect. 4.4)
flags [R] bool: a flagged row is weight 0 (Sect. 2.4), removed from every sum
by selection, so non-finite values under a flag have no effect.

Each stored row (p, q) enters the normal equations twice (row folding,
Eq. JJ:di): for antenna p with y_pq = m conj(g_q) against d, and for antenna q
with y_qp = conj(m) conj(g_p) against conj(d), because d_qp = conj(d_pq) and
m_qp = conj(m_pq).

Readings taken where the paper is silent or garbled:
  * schedule: updates are counted k = 0, 1, 2, ... from the starting gains; the
    LM lambda=1 average (Eq. stefcal-lambda-average) is used on even k and the
    GN step (Eq. stefcal) on odd k ("avg_first"); "gn_first" swaps the parity
    and "gn_only" never averages (Sect. 3.1).
  * 2x2 update order: G_p = (sum_q D_pq Y_pq^H)(sum_q Y_pq Y_pq^H)^-1, i.e. the
    least-squares solution of D = G_p Y; the printed order Y^H D of
    Eq. (update:DI:diag:pol) does not satisfy the normal equations.
  * convergence: relative parameter change ||g_{k+1} - g_k||_F / ||g_{k+1}||_F
    over all antennas (and directions) of the interval, below tol
    (the parameter-update criterion of the convergence appendix).
  * singular blocks: an antenna whose block is not invertible keeps its gain
    and raises SINGULAR_ANT.  Scalar: A_p <= 0.  2x2: Z_00 <= 0 or
    det Z <= EPS_PIVOT * Z_00 * Z_11.  Nd x Nd: a Cholesky pivot
    <= EPS_PIVOT * H_jj.
  * non-finite sums: the interval stops before applying the update, keeps the
    previous gains and raises NONFINITE.
  * residuals of flagged rows are 0; chi^2 sums |r|^2 over unflagged stored rows.
"""
from __future__ import annotations

import numpy as np

CONVERGED = 1
MAXITER = 2
SINGULAR_ANT = 4
NONFINITE = 8

AVG_FIRST = "avg_first"
GN_FIRST = "gn_first"
GN_ONLY = "gn_only"

EPS_PIVOT = 1e-5


# ------------------------------------------------------------------ helpers
def _keep(flags, n):
    if flags is None:
        return np.ones(n, dtype=bool)
    return ~np.asarray(flags, dtype=bool)


def _scatter(out, idx, vals):
    """out[idx[i]] += vals[i] along the first axis (a bincount per trailing element)."""
    n = out.shape[0]
    flat = vals.reshape(vals.shape[0], -1)
    o = out.reshape(n, -1)
    for j in range(flat.shape[1]):
        col = flat[:, j]
        if np.iscomplexobj(o):
            o[:, j] += (np.bincount(idx, weights=col.real, minlength=n)
                        + 1j * np.bincount(idx, weights=col.imag, minlength=n))
        else:
            o[:, j] += np.bincount(idx, weights=col, minlength=n)
    return out


def _is_average_step(k, schedule):
    """True when update k (0-based) is the lambda=1 average of Eq. (stefcal-lambda-average)."""
    if schedule == GN_ONLY:
        return False
    if schedule == AVG_FIRST:
        return k % 2 == 0
    if schedule == GN_FIRST:
        return k % 2 == 1
    raise ValueError(schedule)


def rel_change(g_new, g_old):
    """||g_new - g_old||_F / ||g_new||_F (the parameter-update convergence test)."""
    num = np.sqrt(np.sum(np.abs(g_new - g_old) ** 2))
    den = np.sqrt(np.sum(np.abs(g_new) ** 2))
    if den == 0:
        return 0.0 if num == 0 else np.inf
    return num / den


def cholesky_solve(H, b, eps=EPS_PIVOT):
    """Solve H x = b for Hermitian positive-definite H by the textbook Cholesky
    factorisation H = L L^H, then forward and back substitution.
    Returns None when a pivot is <= eps * H_jj (the singular-block reading)."""
    n = H.shape[0]
    L = np.zeros_like(H, dtype=np.complex128)
    for j in range(n):
        piv = H[j, j].real - np.sum(np.abs(L[j, :j]) ** 2)
        if not (piv > eps * H[j, j].real) or not np.isfinite(piv):
            return None
        L[j, j] = np.sqrt(piv)
        for i in range(j + 1, n):
            L[i, j] = (H[i, j] - np.sum(L[i, :j] * np.conj(L[j, :j]))) / L[j, j]
    z = np.zeros(n, dtype=np.complex128)
    for i in range(n):
        z[i] = (b[i] - np.sum(L[i, :i] * z[:i])) / L[i, i]
    x = np.zeros(n, dtype=np.complex128)
    for i in reversed(range(n)):
        x[i] = (z[i] - np.sum(np.conj(L[i + 1:, i]) * x[i + 1:])) / np.conj(L[i, i])
    return x


# ------------------------------------------------------------------ scalar DI
def accumulate_scalar(d, m, p, q, flags, g):
    """Diagonal of (J^H W J)_UL and top half of J^H W D, J^H W r for scalar gains
    (Eqs. JHJ:DI:tfw and JHR:DI:tfw; J^H D by Eq. ghat).

    Returns dict(A [Na] real, c [Na] = J^H D, jhr [Na] = J^H r, count [Na] int)."""
    na = g.shape[0]
    k = _keep(flags, d.shape[0])
    d, m, p, q = d[k], m[k], p[k], q[k]
    y_pq = m * np.conj(g[q])
    y_qp = np.conj(m) * np.conj(g[p])
    r = d - g[p] * m * np.conj(g[q])
    A = np.zeros(na)
    c = np.zeros(na, dtype=np.complex128)
    jhr = np.zeros(na, dtype=np.complex128)
    _scatter(A, p, np.abs(y_pq) ** 2)
    _scatter(A, q, np.abs(y_qp) ** 2)
    _scatter(c, p, np.conj(y_pq) * d)
    _scatter(c, q, np.conj(y_qp) * np.conj(d))
    _scatter(jhr, p, np.conj(y_pq) * r)
    _scatter(jhr, q, np.conj(y_qp) * np.conj(r))
    count = np.bincount(p, minlength=na) + np.bincount(q, minlength=na)
    return dict(A=A, c=c, jhr=jhr, count=count)


def gn_scalar(acc, g):
    """GN value of Eq. (stefcal): g_p = c_p / A_p; singular antennas keep g_p."""
    A, c = acc["A"], acc["c"]
    sing = ~(A > 0)
    ghat = np.where(sing, g, c / np.where(sing, 1.0, A))
    return ghat, sing


def residual_scalar(d, m, p, q, flags, g):
    """r = d - g_p m conj(g_q) (Eq. cal:DI); flagged rows 0; chi^2 over unflagged rows."""
    k = _keep(flags, d.shape[0])
    r = np.zeros_like(d, dtype=np.complex128)
    r[k] = d[k] - g[p[k]] * m[k] * np.conj(g[q[k]])
    return r, float(np.sum(np.abs(r[k]) ** 2))


# ------------------------------------------------------------------ 2x2 DI
def _H(X):
    return np.conj(np.swapaxes(X, -1, -2))


def accumulate_2x2(D, M, p, q, flags, G):
    """Operator-diagonal blocks of J^H J and J^H D, J^H r for 2x2 Jones (Sect. 4.2-4.3):
    Z_p = sum Y Y^H and N_p = sum D Y^H with Y_pq = M_pq G_q^H; the folded row qp has
    Y_qp = M_pq^H G_p^H and D_qp = D_pq^H.  J^H r = sum R Y^H."""
    na = G.shape[0]
    k = _keep(flags, D.shape[0])
    D, M, p, q = D[k], M[k], p[k], q[k]
    Y_pq = M @ _H(G[q])
    Y_qp = _H(M) @ _H(G[p])
    R = D - G[p] @ M @ _H(G[q])
    Z = np.zeros((na, 2, 2), dtype=np.complex128)
    N = np.zeros((na, 2, 2), dtype=np.complex128)
    jhr = np.zeros((na, 2, 2), dtype=np.complex128)
    _scatter(Z, p, Y_pq @ _H(Y_pq))
    _scatter(Z, q, Y_qp @ _H(Y_qp))
    _scatter(N, p, D @ _H(Y_pq))
    _scatter(N, q, _H(D) @ _H(Y_qp))
    _scatter(jhr, p, R @ _H(Y_pq))
    _scatter(jhr, q, _H(R) @ _H(Y_qp))
    count = np.bincount(p, minlength=na) + np.bincount(q, minlength=na)
    return dict(Z=Z, N=N, jhr=jhr, count=count)


def gn_2x2(acc, G, eps=EPS_PIVOT):
    """GN value G_p = N_p Z_p^-1 (2x2 inverse by the adjugate); singular antennas keep G_p."""
    Z, N = acc["Z"], acc["N"]
    na = G.shape[0]
    Gh = G.copy()
    sing = np.zeros(na, dtype=bool)
    for a in range(na):
        z00, z11 = Z[a, 0, 0].real, Z[a, 1, 1].real
        det = (Z[a, 0, 0] * Z[a, 1, 1] - Z[a, 0, 1] * Z[a, 1, 0]).real
        if not (z00 > 0) or not (det > eps * z00 * z11):
            sing[a] = True
            continue
        Zinv = np.array([[Z[a, 1, 1], -Z[a, 0, 1]], [-Z[a, 1, 0], Z[a, 0, 0]]]) / det
        Gh[a] = N[a] @ Zinv
    return Gh, sing


def residual_2x2(D, M, p, q, flags, G):
    """R = D - G_p M G_q^H (Eq. cal:DI:pol); flagged rows 0; chi^2 = sum ||R||_F^2."""
    k = _keep(flags, D.shape[0])
    R = np.zeros_like(D, dtype=np.complex128)
    R[k] = D[k] - G[p[k]] @ M[k] @ _H(G[q[k]])
    return R, float(np.sum(np.abs(R[k]) ** 2))


# ------------------------------------------------------------------ DD (CohJones / AllJones)
def accumulate_dd(d, m, p, q, flags, g):
    """Per-antenna Nd x Nd blocks of the CAD-ordered J^H J and the vectors J^H D, J^H r
    (Eqs. JHJ:DD:unpol and JHR:DD:unpol): with y^d_pq = m^d conj(g^d_q),
    H_p[c, d] = sum conj(y^c) y^d, c_p[d] = sum conj(y^d) d."""
    nd, na = g.shape
    k = _keep(flags, d.shape[0])
    d, m, p, q = d[k], m[k], p[k], q[k]
    y_pq = m * np.conj(g[:, q]).T            # [R, Nd]
    y_qp = np.conj(m) * np.conj(g[:, p]).T
    r = d - np.sum(g[:, p].T * m * np.conj(g[:, q]).T, axis=1)
    H = np.zeros((na, nd, nd), dtype=np.complex128)
    c = np.zeros((na, nd), dtype=np.complex128)
    jhr = np.zeros((na, nd), dtype=np.complex128)
    _scatter(H, p, np.conj(y_pq)[:, :, None] * y_pq[:, None, :])
    _scatter(H, q, np.conj(y_qp)[:, :, None] * y_qp[:, None, :])
    _scatter(c, p, np.conj(y_pq) * d[:, None])
    _scatter(c, q, np.conj(y_qp) * np.conj(d)[:, None])
    _scatter(jhr, p, np.conj(y_pq) * r[:, None])
    _scatter(jhr, q, np.conj(y_qp) * np.conj(r)[:, None])
    count = np.bincount(p, minlength=na) + np.bincount(q, minlength=na)
    return dict(H=H, c=c, jhr=jhr, count=count)


def gn_cohjones(acc, g, eps=EPS_PIVOT, form="data", H_used=None):
    """CohJones GN value per antenna (Sect. 3.2.2): g_p = H_p^-1 c_p by Cholesky.
    form="residual" uses g_p + H~_p^-1 J^H r (Eq. ghat:approx) with H~ = H_used."""
    nd, na = g.shape
    H = acc["H"] if H_used is None else H_used
    gh = g.copy()
    sing = np.zeros(na, dtype=bool)
    for a in range(na):
        rhs = acc["c"][a] if form == "data" else acc["jhr"][a]
        x = cholesky_solve(H[a], rhs, eps)
        if x is None:
            sing[a] = True
            continue
        gh[:, a] = x if form == "data" else g[:, a] + x
    return gh, sing


def gn_alljones(acc, g):
    """AllJones GN value (Eq. stefcal:dd:unpol): residual form with the diagonal of H_p,
    g^d_p + (sum |y^d|^2)^-1 sum conj(y^d) r."""
    nd, na = g.shape
    diag = np.real(np.einsum("add->ad", acc["H"]))     # [Na, Nd]
    sing = ~(diag > 0)
    step = np.where(sing, 0, acc["jhr"] / np.where(sing, 1.0, diag))
    return g + step.T, sing.T


def residual_dd(d, m, p, q, flags, g):
    """r = d - sum_d g^d_p m^d conj(g^d_q) (Eq. cal:dd:unpol); flagged rows 0."""
    k = _keep(flags, d.shape[0])
    r = np.zeros_like(d, dtype=np.complex128)
    r[k] = d[k] - np.sum(g[:, p[k]].T * m[k] * np.conj(g[:, q[k]]).T, axis=1)
    return r, float(np.sum(np.abs(r[k]) ** 2))


# ------------------------------------------------------------------ polarized DD
def accumulate_dd_2x2(D, M, p, q, flags, G):
    """Polarized direction-dependent blocks (Sect. 4.4): with Y^d_pq = M^d_pq G^{dH}_q
    stacked over directions into Ys_pq [2Nd, 2] (row 2d + k = row k of Y^d), the
    operator-diagonal block of Eq. JHJ:DD:pol for antenna p acts as G_p -> G_p H_p with
        H_p = sum Ys Ys^H           [2Nd, 2Nd], block (c, e) = sum Y^c Y^{eH},
    and the top half of J^H D (Eq. JHR:DD:pol with D in place of R) is
        N_p = sum D Ys^H            [2, 2Nd],   block e = sum D Y^{eH}
    (least-squares order of the update, as for the 2x2 DI case).  J^H r uses
    R = D - sum_d G^d_p M^d G^{dH}_q.  The folded row qp has Y^d_qp = M^{dH} G^{dH}_p
    and D_qp = D^H.  D [R, 2, 2], M [R, Nd, 2, 2], G [Nd, Na, 2, 2]."""
    nd, na = G.shape[:2]
    k = _keep(flags, D.shape[0])
    D, M, p, q = D[k], M[k], p[k], q[k]
    Gp = np.swapaxes(G[:, p], 0, 1)             # [R, Nd, 2, 2]
    Gq = np.swapaxes(G[:, q], 0, 1)
    Y_pq = (M @ _H(Gq)).reshape(-1, 2 * nd, 2)
    Y_qp = (_H(M) @ _H(Gp)).reshape(-1, 2 * nd, 2)
    R = D - np.sum(Gp @ M @ _H(Gq), axis=1)
    Hm = np.zeros((na, 2 * nd, 2 * nd), dtype=np.complex128)
    N = np.zeros((na, 2, 2 * nd), dtype=np.complex128)
    jhr = np.zeros((na, 2, 2 * nd), dtype=np.complex128)
    _scatter(Hm, p, Y_pq @ _H(Y_pq))
    _scatter(Hm, q, Y_qp @ _H(Y_qp))
    _scatter(N, p, D @ _H(Y_pq))
    _scatter(N, q, _H(D) @ _H(Y_qp))
    _scatter(jhr, p, R @ _H(Y_pq))
    _scatter(jhr, q, _H(R) @ _H(Y_qp))
    count = np.bincount(p, minlength=na) + np.bincount(q, minlength=na)
    return dict(H=Hm, N=N, jhr=jhr, count=count)


def _rows_to_dirs(X, nd):
    """[2, 2Nd] row block -> [Nd, 2, 2] per-direction 2x2 matrices."""
    return np.swapaxes(X.reshape(2, nd, 2), 0, 1)


def gn_cohjones_2x2(acc, G, eps=EPS_PIVOT, form="data"):
    """Polarized CohJones GN value per antenna (Sect. 4.4, separable by antenna only):
    the stacked gains [G^0 .. G^{Nd-1}] (2 x 2Nd) solve G H_p = N_p, i.e. each row x of
    the gains solves H_p x^H = (row of N_p)^H, by Cholesky.  form="residual" gives
    G + (J^H r) H_p^-1 (Eq. ghat:approx).  Singular antennas keep their gains."""
    nd, na = G.shape[:2]
    Gh = G.copy()
    sing = np.zeros(na, dtype=bool)
    for a in range(na):
        rhs = acc["N"][a] if form == "data" else acc["jhr"][a]
        rows = []
        for i in range(2):
            x = cholesky_solve(acc["H"][a], np.conj(rhs[i]), eps)
            if x is None:
                break
            rows.append(np.conj(x))
        if len(rows) < 2:
            sing[a] = True
            continue
        step = _rows_to_dirs(np.stack(rows), nd)
        Gh[:, a] = step if form == "data" else G[:, a] + step
    return Gh, sing


def gn_alljones_2x2(acc, G, eps=EPS_PIVOT):
    """Polarized AllJones GN value (Eq. update:DD:diag:pol, least-squares order; residual
    form): G^d_p + (sum R Y^{dH}) (sum Y^d Y^{dH})^-1 per antenna and direction, the
    2x2 inverse by the adjugate.  A singular 2x2 block keeps its gain."""
    nd, na = G.shape[:2]
    Gh = G.copy()
    sing = np.zeros((nd, na), dtype=bool)
    for a in range(na):
        J = _rows_to_dirs(acc["jhr"][a], nd)
        for d in range(nd):
            Z = acc["H"][a, 2 * d:2 * d + 2, 2 * d:2 * d + 2]
            z00, z11 = Z[0, 0].real, Z[1, 1].real
            det = (Z[0, 0] * Z[1, 1] - Z[0, 1] * Z[1, 0]).real
            if not (z00 > 0) or not (det > eps * z00 * z11):
                sing[d, a] = True
                continue
            Zinv = np.array([[Z[1, 1], -Z[0, 1]], [-Z[1, 0], Z[0, 0]]]) / det
            Gh[d, a] = G[d, a] + J[d] @ Zinv
    return Gh, sing


def residual_dd_2x2(D, M, p, q, flags, G):
    """R = D - sum_d G^d_p M^d G^{dH}_q (the polarized DD measurement equation of
    Sect. 4.4); flagged rows 0; chi^2 = sum ||R||_F^2 over unflagged rows."""
    k = _keep(flags, D.shape[0])
    R = np.zeros_like(D, dtype=np.complex128)
    Gp = np.swapaxes(G[:, p[k]], 0, 1)
    Gq = np.swapaxes(G[:, q[k]], 0, 1)
    R[k] = D[k] - np.sum(Gp @ M[k] @ _H(Gq), axis=1)
    return R, float(np.sum(np.abs(R[k]) ** 2))


# ------------------------------------------------------------------ point-source models
C_LIGHT = 299792458.0


def point_model(uvw, lmn, flux, freq):
    """Point-source model of Sect. 3.2.1: m^d = S_d k^d with the phase rotation
    k^d = exp(-2 pi i (u . sigma_d) nu / c), sigma_d = [l_d, m_d, n_d - 1].
    uvw [R, 3] (metres) and freq [R] (Hz) per row, lmn [Nd, 3], flux [Nd]; returns [R, Nd]."""
    ph = (np.asarray(uvw, dtype=np.float64) @ np.asarray(lmn, dtype=np.float64).T)     # [R, Nd]
    arg = -2.0 * np.pi * ph * np.asarray(freq, dtype=np.float64)[:, None] / C_LIGHT
    return np.asarray(flux, dtype=np.float64)[None, :] * np.exp(1j * arg)


# ------------------------------------------------------------------ iteration driver
def _solve(accumulate, gn, residual, finite, sing_to_ant, d, m, p, q, flags, g0,
           tol, max_iter, schedule):
    g = np.array(g0, dtype=np.complex128, copy=True)
    status = 0
    hist = []
    n_iter = 0
    k_rows = _keep(flags, d.shape[0])
    if not (np.all(np.isfinite(d[k_rows])) and np.all(np.isfinite(m[k_rows]))):
        status |= NONFINITE
    else:
        for k in range(max_iter):
            acc = accumulate(d, m, p, q, flags, g)
            if not finite(acc):
                status |= NONFINITE
                break
            ghat, sing = gn(acc, g)
            if np.any(sing):
                status |= SINGULAR_ANT
            g_new = 0.5 * (g + ghat) if _is_average_step(k, schedule) else ghat
            rel = rel_change(g_new, g)
            hist.append(rel)
            g = g_new
            n_iter = k + 1
            if rel < tol:
                status |= CONVERGED
                break
        else:
            status |= MAXITER
    r, chi2 = residual(d, m, p, q, flags, g)
    return dict(g=g, n_iter=n_iter, status=status, residual=r, chi2=chi2, history=hist)


def stefcal_scalar(d, m, p, q, flags, g0, tol=1e-6, max_iter=100, schedule=AVG_FIRST):
    """Scalar StefCal: diagonal J^H J, GN (Eq. stefcal) alternating with the
    lambda=1 LM average (Eq. stefcal-lambda-average), Jacobi over antennas."""
    fin = lambda a: np.all(np.isfinite(a["A"])) and np.all(np.isfinite(a["c"]))
    return _solve(accumulate_scalar, gn_scalar, residual_scalar, fin, None,
                  d, m, p, q, flags, g0, tol, max_iter, schedule)


def stefcal_2x2(D, M, p, q, flags, G0, tol=1e-6, max_iter=100, schedule=AVG_FIRST):
    """Polarized StefCal (Eq. update:DI:diag:pol, order per the least-squares reading)."""
    fin = lambda a: np.all(np.isfinite(a["Z"])) and np.all(np.isfinite(a["N"]))
    return _solve(accumulate_2x2, gn_2x2, residual_2x2, fin, None,
                  D, M, p, q, flags, G0, tol, max_iter, schedule)


def cohjones(d, m, p, q, flags, g0, tol=1e-6, max_iter=100, schedule=AVG_FIRST,
             form="data", perturb=None):
    """CohJones (Sect. 3.2.2): per-antenna Nd x Nd blocks inverted exactly.
    perturb(H) -> H~ replaces the blocks by an approximation (used with form="residual")."""
    fin = lambda a: np.all(np.isfinite(a["H"])) and np.all(np.isfinite(a["c"]))

    def gn(acc, g):
        Hu = None if perturb is None else perturb(acc["H"])
        return gn_cohjones(acc, g, form=form, H_used=Hu)
    return _solve(accumulate_dd, gn, residual_dd, fin, None,
                  d, m, p, q, flags, g0, tol, max_iter, schedule)


def alljones(d, m, p, q, flags, g0, tol=1e-6, max_iter=200, schedule=AVG_FIRST):
    """AllJones (Sect. 3.2.3): fully diagonal DD update in residual form."""
    fin = lambda a: np.all(np.isfinite(a["H"])) and np.all(np.isfinite(a["jhr"]))
    return _solve(accumulate_dd, gn_alljones, residual_dd, fin, None,
                  d, m, p, q, flags, g0, tol, max_iter, schedule)


def cohjones_2x2(D, M, p, q, flags, G0, tol=1e-6, max_iter=100, schedule=AVG_FIRST,
                 form="data"):
    """Polarized CohJones: per-antenna 2Nd x 2Nd blocks (the 4Nd x 4Nd operator block of
    Eq. JHJ:DD:pol acts on both rows of the gains alike) inverted exactly."""
    fin = lambda a: np.all(np.isfinite(a["H"])) and np.all(np.isfinite(a["N"]))
    gn = lambda acc, g: gn_cohjones_2x2(acc, g, form=form)
    return _solve(accumulate_dd_2x2, gn, residual_dd_2x2, fin, None,
                  D, M, p, q, flags, G0, tol, max_iter, schedule)


def alljones_2x2(D, M, p, q, flags, G0, tol=1e-6, max_iter=200, schedule=AVG_FIRST):
    """Polarized AllJones: separable by antenna and direction, residual form
    (Eq. update:DD:diag:pol)."""
    fin = lambda a: np.all(np.isfinite(a["H"])) and np.all(np.isfinite(a["jhr"]))
    return _solve(accumulate_dd_2x2, gn_alljones_2x2, residual_dd_2x2, fin, None,
                  D, M, p, q, flags, G0, tol, max_iter, schedule)


# ------------------------------------------------------------------ smoothing (Sect. 3.4)
def smoothing_kernel(sigma):
    """1-D taps w(j) = exp(-j^2 / (2 sigma^2)) for |j| <= ceil(3 sigma) (reading: truncated at
    three widths; sigma = 0 is the delta kernel, no smoothing).  Returns (taps, radius)."""
    if sigma <= 0:
        return np.ones(1), 0
    r = int(np.ceil(3.0 * sigma))
    j = np.arange(-r, r + 1)
    return np.exp(-j * j / (2.0 * sigma * sigma)), r


def smooth_grid(x, sigma_t, sigma_f):
    """(w o x)(t0, f0) = sum over grid cells (t, f) of w(t - t0, f - f0) x(t, f) for x
    [n_time, n_chan, ...], w the product of the time and frequency kernels; cells beyond the
    grid edge are absent from the sum (Eq. JHJ:diag:smooth, written as its definition: one
    shifted slice per kernel tap)."""
    kt, rt = smoothing_kernel(sigma_t)
    kf, rf = smoothing_kernel(sigma_f)
    nt, nf = x.shape[:2]
    out = np.zeros_like(x)
    # offsets beyond the grid's extent reach no cell
    for dt in range(-min(rt, nt - 1), min(rt, nt - 1) + 1):
        for df in range(-min(rf, nf - 1), min(rf, nf - 1) + 1):
            w = kt[dt + rt] * kf[df + rf]
            # out[t0, f0] += w * x[t0 + dt, f0 + df] where both are on the grid
            t0a, t0b = max(0, -dt), min(nt, nt - dt)
            f0a, f0b = max(0, -df), min(nf, nf - df)
            if t0a >= t0b or f0a >= f0b:
                continue
            out[t0a:t0b, f0a:f0b] += w * x[t0a + dt:t0b + dt, f0a + df:f0b + df]
    return out


def accumulate_cells(d, m, p, q, cell, flags, g, n_cells):
    """alpha_p(t, nu) = sum_q conj(y) d and beta_p(t, nu) = sum_q |y|^2 per cell (Sect. 3.4: the
    accumulators of Eqs. JHJ:DI:tfw, JHR:DI:tfw without the sum over samples), with
    y_pq = m conj(g_q) at the row's own cell and both sides of every row (Eq. JJ:di).
    g [n_cells, Na]; returns alpha [n_cells, Na] complex, beta [n_cells, Na] real."""
    na = g.shape[1]
    k = _keep(flags, d.shape[0])
    d, m, p, q, cell = d[k], m[k], p[k], q[k], cell[k]
    y_pq = m * np.conj(g[cell, q])
    y_qp = np.conj(m) * np.conj(g[cell, p])
    alpha = np.zeros(n_cells * na, dtype=np.complex128)
    beta = np.zeros(n_cells * na)
    _scatter(alpha, cell * na + p, np.conj(y_pq) * d)
    _scatter(alpha, cell * na + q, np.conj(y_qp) * np.conj(d))
    _scatter(beta, cell * na + p, np.abs(y_pq) ** 2)
    _scatter(beta, cell * na + q, np.abs(y_qp) ** 2)
    return alpha.reshape(n_cells, na), beta.reshape(n_cells, na)


def stefcal_smooth(d, m, p, q, cell, flags, g0, n_time, n_chan, sigma_t, sigma_f, tol=1e-6,
                   max_iter=100, schedule=AVG_FIRST):
    """StefCal with time/frequency smoothing (Sect. 3.4) over one chunk of n_time x n_chan
    cells (cell = t * n_chan + nu of each row): every update takes the per-cell GN value
    g_p(t, nu) = (w o alpha_p) / (w o beta_p) (Eq. JHJ:diag:smooth), then the schedule of
    Sect. 3.1.  Convergence (reading; the paper does not test it): the relative change over
    every cell and antenna of the chunk after removing, per cell, the best phase between the
    two iterates.  Each cell's solution answers its own weighted least-squares problem
    (Eq. cal:DI:smooth), defined up to one phase per cell, and the smoothed update is not
    the step of one objective: with noise its iterates keep turning along these phases
    (rigidly, by one common phase per update, when the gains are constant over the chunk),
    a motion the plain relative change would never see stop.  A cell whose smoothed beta_p
    is not positive keeps its gain (SINGULAR_ANT).  g0 [n_cells, Na]."""
    n_cells = n_time * n_chan
    g = np.array(g0, dtype=np.complex128, copy=True)
    na = g.shape[1]
    status, n_iter, hist = 0, 0, []
    kr = _keep(flags, d.shape[0])
    if not (np.all(np.isfinite(d[kr])) and np.all(np.isfinite(m[kr]))):
        status |= NONFINITE
    else:
        for k in range(max_iter):
            alpha, beta = accumulate_cells(d, m, p, q, cell, flags, g, n_cells)
            sa = smooth_grid(alpha.reshape(n_time, n_chan, na), sigma_t, sigma_f).reshape(n_cells, na)
            sb = smooth_grid(beta.reshape(n_time, n_chan, na), sigma_t, sigma_f).reshape(n_cells, na)
            sing = ~(sb > 0)
            if np.any(sing):
                status |= SINGULAR_ANT
            ghat = np.where(sing, g, sa / np.where(sing, 1.0, sb))
            g_new = 0.5 * (g + ghat) if _is_average_step(k, schedule) else ghat
            rel = cell_rel_change(g_new, g)
            hist.append(rel)
            g = g_new
            n_iter = k + 1
            if rel < tol:
                status |= CONVERGED
                break
        else:
            status |= MAXITER
    r = np.zeros_like(d, dtype=np.complex128)
    r[kr] = d[kr] - g[cell[kr], p[kr]] * m[kr] * np.conj(g[cell[kr], q[kr]])
    return dict(g=g, n_iter=n_iter, status=status, residual=r, chi2=float(np.sum(np.abs(r[kr]) ** 2)),
                history=hist)


def cell_rel_change(g_new, g_old):
    """Convergence measure of the smoothed iteration (a reading; Sect. 3.4 does not test
    convergence): ||g_new' - g_old||_F / ||g_new||_F over every cell and antenna, where g_new'
    is g_new with each cell turned by its own least-squares phase onto g_old.  Each cell's
    weighted problem (Eq. cal:DI:smooth) involves only that cell's gains, so it is defined up
    to one phase per cell.  g [n_cells, Na]."""
    aligned = np.stack([align_phase(g_new[c], g_old[c]) for c in range(g_new.shape[0])])
    return rel_change(aligned, g_old)


# ------------------------------------------------------------------ gauge
def align_phase(g, ref):
    """g * exp(i phi) with phi = arg sum conj(g) ref: the least-squares global phase
    that maps g onto ref (the solution is unique only up to this phase)."""
    s = np.sum(np.conj(g) * ref)
    return g * (s / abs(s) if abs(s) > 0 else 1.0)


def align_phase_per_direction(g, ref):
    """DD gains [Nd, Na]: one phase per direction (the DD model is invariant under
    g^d -> g^d exp(i phi_d))."""
    return np.stack([align_phase(g[i], ref[i]) for i in range(g.shape[0])])


def rel_err(a, b):
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2)) / np.sqrt(np.sum(np.abs(b) ** 2)))
