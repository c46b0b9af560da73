"""Extended-precision element Schur complements (test infrastructure).

The same element matrix and local Schur complement as ``element`` and
``hybrid``, carried out in x87 extended precision (numpy.longdouble, 64-bit
significand, unit roundoff 5.4e-20) with a hand-written Cholesky.  The
quadrature points/weights and vertex coordinates are taken as exact inputs.

Two correct FP64 computations of H_T differ from each other by about
cond(M_T) times the FP64 unit roundoff; this reference is accurate to about
cond(M_T) * 5e-20, so it measures each FP64 computation's own error (the
noise floor of the 1e-12 parity target) instead of their mutual gap.
"""
from __future__ import annotations

import numpy as np

from . import hybrid, quadrature, rt_basis

LD = np.longdouble


def _lagrange_ld(z, x):
    z = np.asarray(z, dtype=LD)
    x = np.asarray(x, dtype=LD)
    out = np.ones((len(z), x.size), dtype=LD)
    for i in range(len(z)):
        for j in range(len(z)):
            if j != i:
                out[i] *= (x - z[j]) / (z[i] - z[j])
    return out


def _lagrange_deriv_ld(z, x):
    z = np.asarray(z, dtype=LD)
    x = np.asarray(x, dtype=LD)
    out = np.zeros((len(z), x.size), dtype=LD)
    for i in range(len(z)):
        for m in range(len(z)):
            if m == i:
                continue
            term = np.full(x.size, LD(1) / (z[i] - z[m]), dtype=LD)
            for j in range(len(z)):
                if j != i and j != m:
                    term = term * (x - z[j]) / (z[i] - z[j])
            out[i] += term
    return out


def element_matrix_ld(k: int, xyz_e: np.ndarray, alpha: float, beta: float, f=None):
    """M_T (n, n) in long double for one element (q = k+2 Gauss points); with
    an element load f (3,) also returns f_T (n,)."""
    q = k + 2
    X, W = quadrature.hex_rule(q)
    X = X.astype(LD)
    W = W.astype(LD)
    zc = rt_basis.closed_points(k)
    zo = rt_basis.open_points(k)
    tab = rt_basis.dof_table(k)
    n, P = tab.shape[0], X.shape[0]
    Lc = [_lagrange_ld(zc, X[:, a]) for a in range(3)]
    dLc = [_lagrange_deriv_ld(zc, X[:, a]) for a in range(3)]
    Lo = [_lagrange_ld(zo, X[:, a]) for a in range(3)]
    val = np.zeros((n, P), dtype=LD)
    div = np.zeros((n, P), dtype=LD)
    comp = tab[:, 0]
    for idx, (d, i, j0, j1) in enumerate(tab):
        t0, t1 = rt_basis.tangential_axes(int(d))
        tang = Lo[t0][j0] * Lo[t1][j1]
        val[idx] = Lc[d][i] * tang
        div[idx] = dLc[d][i] * tang
    xe = np.asarray(xyz_e, dtype=LD)
    # trilinear Jacobian
    J = np.zeros((P, 3, 3), dtype=LD)
    for v in range(8):
        bits = [(v >> a) & 1 for a in range(3)]
        fa = [X[:, a] if bits[a] else 1 - X[:, a] for a in range(3)]
        ga = [LD(1) if bits[a] else LD(-1) for a in range(3)]
        dN = [ga[0] * fa[1] * fa[2], fa[0] * ga[1] * fa[2], fa[0] * fa[1] * ga[2]]
        for r in range(3):
            for c in range(3):
                J[:, r, c] += xe[v, r] * dN[c]
    det = (J[:, 0, 0] * (J[:, 1, 1] * J[:, 2, 2] - J[:, 1, 2] * J[:, 2, 1])
           - J[:, 0, 1] * (J[:, 1, 0] * J[:, 2, 2] - J[:, 1, 2] * J[:, 2, 0])
           + J[:, 0, 2] * (J[:, 1, 0] * J[:, 2, 1] - J[:, 1, 1] * J[:, 2, 0]))
    G = np.einsum("prd,pre->pde", J, J)                      # J^T J
    wd = W / det
    M = np.zeros((n, n), dtype=LD)
    for i in range(n):
        gi = G[:, comp[i], :][:, comp]                       # (P, n): G[d_i, d_j]
        M[i] = (LD(alpha) * (wd[:, None] * gi * val[i][:, None] * val.T).sum(axis=0)
                + LD(beta) * (wd[:, None] * div[i][:, None] * div.T).sum(axis=0))
    if f is None:
        return M
    fl = np.asarray(f, dtype=LD)
    Jtf = np.einsum("prd,r->pd", J, fl)                       # (J^T f) per point
    fT = np.array([(W * Jtf[:, comp[i]] * val[i]).sum() for i in range(n)], dtype=LD)
    return M, fT


def cholesky_ld(A: np.ndarray) -> np.ndarray:
    A = np.array(A, dtype=LD)
    n = A.shape[0]
    L = np.zeros_like(A)
    for c in range(n):
        s = A[c, c] - np.dot(L[c, :c], L[c, :c])
        if not s > 0:
            raise np.linalg.LinAlgError("not positive definite")
        L[c, c] = np.sqrt(s)
        if c + 1 < n:
            L[c + 1:, c] = (A[c + 1:, c] - L[c + 1:, :c] @ L[c, :c]) / L[c, c]
    return L


def forward_ld(L, B):
    B = np.array(B, dtype=LD)
    X = np.zeros_like(B)
    for i in range(L.shape[0]):
        X[i] = (B[i] - L[i, :i] @ X[:i]) / L[i, i]
    return X


def local_schur_ld(k: int, M: np.ndarray, code: int) -> np.ndarray:
    """H_T = C_T M_rr^{-1} C_T^T in long double: Cholesky of the kept block,
    then (L^{-1} C^T)^T (L^{-1} C^T)."""
    keep, _, mpos = hybrid._split(k, code)
    ni = rt_basis.n_interior(k)
    Mrr = M[np.ix_(keep, keep)]
    eps = hybrid._face_signs(k)[keep[mpos] - ni]
    CT = np.zeros((mpos.size, keep.size), dtype=LD)
    CT[np.arange(mpos.size), mpos] = eps
    L = cholesky_ld(Mrr)
    Y = forward_ld(L, CT.T)
    return Y.T @ Y


def backward_ld(L, B):
    """Solve L^T X = B."""
    B = np.array(B, dtype=LD)
    X = np.zeros_like(B)
    n = L.shape[0]
    for i in range(n - 1, -1, -1):
        X[i] = (B[i] - L[i + 1:, i] @ X[i + 1:]) / L[i, i]
    return X


def local_rhs_ld(k: int, M: np.ndarray, fT: np.ndarray, code: int) -> np.ndarray:
    """r_T = C_T M_rr^{-1} f_r (zero boundary data) in long double."""
    keep, _, mpos = hybrid._split(k, code)
    ni = rt_basis.n_interior(k)
    eps = hybrid._face_signs(k)[keep[mpos] - ni].astype(LD)
    L = cholesky_ld(M[np.ix_(keep, keep)])
    x = backward_ld(L, forward_ld(L, fT[keep]))
    return eps * x[mpos]


def local_recover_ld(k: int, M: np.ndarray, fT: np.ndarray, code: int, lam_T: np.ndarray) -> np.ndarray:
    """u_T = M_rr^{-1} (f_r - C_T^T lam_T) on the kept dofs, 0 on boundary faces."""
    keep, _, mpos = hybrid._split(k, code)
    ni = rt_basis.n_interior(k)
    eps = hybrid._face_signs(k)[keep[mpos] - ni].astype(LD)
    rhs = np.array(fT[keep], dtype=LD)
    rhs[mpos] -= eps * np.asarray(lam_T, dtype=LD)
    L = cholesky_ld(M[np.ix_(keep, keep)])
    u = np.zeros(M.shape[0], dtype=LD)
    u[keep] = backward_ld(L, forward_ld(L, rhs))
    return u


def hybridize_ld(k: int, xyz, e2v, alpha, beta, f, topo, elements, lam=None):
    """Long-double H (as a dict {(mu, nu): value}), r (dict {mu: value}) and,
    with lam, u for the given elements (dict {e: u_T}).  Rows of H and r are
    complete for every face whose two elements are both in ``elements``."""
    from . import topology as topo_mod
    K2 = rt_basis.n_face(k)
    H, r, U = {}, {}, {}
    for e in np.asarray(elements):
        e = int(e)
        code = int(((topo.elem_face[e] < 0) * (1 << np.arange(6))).sum())
        M, fT = element_matrix_ld(k, xyz[e2v[e]], float(alpha[e]), float(beta[e]), f[e])
        HT = local_schur_ld(k, M, code)
        rT = local_rhs_ld(k, M, fT, code)
        ids = [mu for (_, mu, _) in topo_mod.element_multipliers(topo, k, e) if mu >= 0]
        for a, mu in enumerate(ids):
            r[mu] = r.get(mu, LD(0)) + rT[a]
            for b, nu in enumerate(ids):
                H[(mu, nu)] = H.get((mu, nu), LD(0)) + HT[a, b]
        if lam is not None:
            U[e] = local_recover_ld(k, M, fT, code, np.asarray(lam)[ids])
    return H, r, U
