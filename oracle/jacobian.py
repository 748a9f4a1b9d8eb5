"""Definition layer of the oracle: explicit complex Jacobians, full Gauss-Newton
and Levenberg-Marquardt on tiny arrays.

TEST INFRASTRUCTURE ONLY (see the package docstring).  complex128 NumPy.

The Wirtinger derivatives (Sect. 1) of a model v(z, conj z) are obtained here
numerically from real-coordinate central differences,
    dv/dz = (dv/dx - i dv/dy) / 2,   dv/dconj(z) = (dv/dx + i dv/dy) / 2,
which is exact up to rounding for the bilinear measurement equations used
here (their real-coordinate Hessian is constant).  The full complex Jacobian
is then assembled as in Eq. (JJ) and used by GN (Eq. GN, minimum-norm step
because J^H J is singular along the phase gauge) and by the LM variant of the
optimisation appendix (lambda_0 = 1, K = 10).  Closed-form Jacobians written
from Eqs. (JJ:di), the DD Jacobian of Sect. 2.5 and the operator form
Eq. (JJ:pol) are provided for comparison against the numerical ones.
"""
from __future__ import annotations

import numpy as np


# ------------------------------------------------------------------ models v(z)
def model_scalar(g, m, p, q):
    """v_pq = g_p m_pq conj(g_q) for stored rows (Eq. RIME:unpol)."""
    return g[p] * m * np.conj(g[q])


def model_dd(gflat, m, p, q, nd, na):
    """v_pq = sum_d g^d_p m^d_pq conj(g^d_q) (Eq. cal:dd:unpol); gflat in CAD order
    (antenna major, direction minor: index j * nd + d)."""
    g = gflat.reshape(na, nd).T
    return np.sum(g[:, p].T * m * np.conj(g[:, q]).T, axis=1)


def vec(X):
    """Stacked-columns vectorisation of the trailing 2x2 axes (operator-calculus appendix)."""
    return np.swapaxes(X, -1, -2).reshape(X.shape[:-2] + (4,))


def unvec(x):
    return np.swapaxes(x.reshape(x.shape[:-1] + (2, 2)), -1, -2)


def model_2x2(gflat, M, p, q, na):
    """vec(G_p M_pq G_q^H) for stored rows, stacked; gflat = [vec G_1, ..., vec G_na]."""
    G = unvec(gflat.reshape(na, 4))
    V = G[p] @ M @ np.conj(np.swapaxes(G[q], -1, -2))
    return vec(V).reshape(-1)


def model_dd_2x2(gflat, M, p, q, nd, na):
    """vec(sum_d G^d_p M^d_pq G^{dH}_q) for stored rows, stacked (polarized DD, Sect. 4.4);
    gflat = [vec G^d_a] antenna major, direction minor (index (a * nd + d) * 4 + e)."""
    G = unvec(gflat.reshape(na, nd, 4))                  # [na, nd, 2, 2]
    V = np.sum(G[p] @ M @ np.conj(np.swapaxes(G[q], -1, -2)), axis=1)
    return vec(V).reshape(-1)


# ------------------------------------------------------------------ Jacobians
def wirtinger_jacobian(f, z, h=0.05):
    """(J_k, J_k*) = (dv/dz, dv/dconj z) at z by real-coordinate central differences."""
    z = np.asarray(z, dtype=np.complex128)
    n = z.size
    v0 = f(z)
    Jk = np.zeros((v0.size, n), dtype=np.complex128)
    Jks = np.zeros((v0.size, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = h
        dx = (f(z + e) - f(z - e)) / (2 * h)
        dy = (f(z + 1j * e) - f(z - 1j * e)) / (2 * h)
        Jk[:, j] = 0.5 * (dx - 1j * dy)
        Jks[:, j] = 0.5 * (dx + 1j * dy)
    return Jk, Jks


def full_jacobian(Jk, Jks):
    """The complex Jacobian of Eq. (JJ): [[J_k, J_k*], [conj J_k*, conj J_k]]."""
    return np.block([[Jk, Jks], [np.conj(Jks), np.conj(Jk)]])


def jacobian_scalar_closed(g, m, p, q):
    """Row-folded J of Eq. (JJ:di): rows [pq] then [qp] for every stored row; columns
    j (for g_j) then j (for conj g_j).  Row pq: m conj(g_q) at column p and g_p m at
    conjugate column q."""
    na = g.size
    R = m.size
    J = np.zeros((2 * R, 2 * na), dtype=np.complex128)
    for i in range(R):
        a, b, mm = p[i], q[i], m[i]
        J[i, a] = mm * np.conj(g[b])
        J[i, na + b] = g[a] * mm
        # folded conjugate row qp: m_qp = conj(m_pq)
        J[R + i, b] = np.conj(mm) * np.conj(g[a])
        J[R + i, na + a] = g[b] * np.conj(mm)
    return J


def jacobian_dd_closed(g, m, p, q):
    """Row-folded DD Jacobian (Sect. 2.5), columns in CAD order (antenna major,
    direction minor), then the same for the conjugate parameters."""
    nd, na = g.shape
    R = m.shape[0]
    J = np.zeros((2 * R, 2 * na * nd), dtype=np.complex128)
    for i in range(R):
        a, b = p[i], q[i]
        for d in range(nd):
            mm = m[i, d]
            J[i, a * nd + d] = mm * np.conj(g[d, b])
            J[i, na * nd + b * nd + d] = g[d, a] * mm
            J[R + i, b * nd + d] = np.conj(mm) * np.conj(g[d, a])
            J[R + i, na * nd + a * nd + d] = g[d, b] * np.conj(mm)
    return J


def RA4(A):
    """4x4 matrix of the right-multiply operator X -> X A (Eq. RA4x4)."""
    a11, a12, a21, a22 = A[0, 0], A[0, 1], A[1, 0], A[1, 1]
    return np.array([[a11, 0, a21, 0],
                     [0, a11, 0, a21],
                     [a12, 0, a22, 0],
                     [0, a12, 0, a22]], dtype=np.complex128)


def LA4(A):
    """4x4 matrix of the left-multiply operator X -> A X (Eq. LA4x4)."""
    a11, a12, a21, a22 = A[0, 0], A[0, 1], A[1, 0], A[1, 1]
    return np.array([[a11, a12, 0, 0],
                     [a21, a22, 0, 0],
                     [0, 0, a11, a12],
                     [0, 0, a21, a22]], dtype=np.complex128)


def jacobian_2x2_closed(G, M, p, q):
    """Row-folded polarized Jacobian of Eq. (JJ:pol) in 4x4 blocks: row block [pq]
    holds R_{M_pq G_q^H} at column G_p and L_{G_p M_pq} at column G_q^H; the folded
    row [qp] uses M_qp = M_pq^H.  Parameters are [vec G_1..vec G_na, vec G_1^H..]."""
    na = G.shape[0]
    R = M.shape[0]
    H = lambda X: np.conj(X.T)
    J = np.zeros((8 * R, 8 * na), dtype=np.complex128)
    for i in range(R):
        a, b = p[i], q[i]
        Mi = M[i]
        J[4 * i:4 * i + 4, 4 * a:4 * a + 4] = RA4(Mi @ H(G[b]))
        J[4 * i:4 * i + 4, 4 * na + 4 * b:4 * na + 4 * b + 4] = LA4(G[a] @ Mi)
        o = 4 * (R + i)
        J[o:o + 4, 4 * b:4 * b + 4] = RA4(H(Mi) @ H(G[a]))
        J[o:o + 4, 4 * na + 4 * a:4 * na + 4 * a + 4] = LA4(G[b] @ H(Mi))
    return J


# ------------------------------------------------------------------ optimisers
def gn_full(f, d, z0, n_iter=50, tol=1e-14):
    """Complex Gauss-Newton (Eq. GN): z <- z + (J^H J)^+ J^H r (top half), with the
    minimum-norm least-squares step from lstsq."""
    z = np.array(z0, dtype=np.complex128)
    n = z.size
    for _ in range(n_iter):
        r = d - f(z)
        J = full_jacobian(*wirtinger_jacobian(f, z))
        rr = np.concatenate([r, np.conj(r)])
        dz = np.linalg.lstsq(J, rr, rcond=None)[0]
        z = z + dz[:n]
        if np.linalg.norm(dz[:n]) < tol * np.linalg.norm(z):
            break
    return z


def lm_full(f, d, z0, n_iter=200, lam0=1.0, K=10.0, tol=1e-14):
    """Levenberg-Marquardt of the optimisation appendix: step from
    (J^H J + lambda diag(J^H J))^-1 J^H r; an unsuccessful step (chi^2 not lower)
    is undone and lambda *= K, a successful one divides lambda by K."""
    z = np.array(z0, dtype=np.complex128)
    n = z.size
    lam = lam0
    r = d - f(z)
    chi2 = np.sum(np.abs(r) ** 2)
    for _ in range(n_iter):
        J = full_jacobian(*wirtinger_jacobian(f, z))
        JHJ = J.conj().T @ J
        rr = np.concatenate([r, np.conj(r)])
        rhs = J.conj().T @ rr
        dz = np.linalg.solve(JHJ + lam * np.diag(np.diag(JHJ)), rhs)[:n]
        zt = z + dz
        rt = d - f(zt)
        chi2t = np.sum(np.abs(rt) ** 2)
        if chi2t < chi2:
            z, r, chi2 = zt, rt, chi2t
            lam /= K
            if np.linalg.norm(dz) < tol * np.linalg.norm(z):
                break
        else:
            lam *= K
            if lam > 1e30:      # steps no longer change z: no further progress possible
                break
    return z
