"""Extended-precision element Schur complements (test infrastructure).

The element matrix M_T, the local Schur complement H_T = C_T M_rr^{-1} C_T^T
(Theorem 2.1, Sec. 3.1), the local load r_T = C_T M_rr^{-1} f_r and the
recovery u_T = M_rr^{-1} (f_r - C_T^T lam_T), carried out in x87 extended
precision (numpy.longdouble: 64-bit significand, unit roundoff 2^-64 ~ 5.4e-20)
with a hand-written Cholesky.

Everything that enters is computed in extended precision here as well: the
Gauss-Legendre quadrature nodes and weights, the Gauss-Legendre (open) and
Gauss-Lobatto (closed) interpolation nodes of the basis (Newton's method on
the Legendre three-term recurrence, started from the double-precision
values), the Jacobians and the sums.  Only the vertex coordinates and the
coefficients are taken as exact double inputs.  The result is therefore the
exact value of the method to about cond(M_T) 2^-64, while two correct FP64
computations of H_T differ from it (and from each other) by about
cond(M_T) 2^-53: it measures each FP64 computation's own error, the noise
floor of the FP64 parity target.

The sign, split and Jacobian conventions are written out here again (small
helpers, no import of the FP64 routines), so that the pins in
``tests/test_oracle_extended.py`` compare two independent codings of them.
"""
from __future__ import annotations

import functools

import numpy as np

from . import element, rt_basis

LD = np.longdouble


# --------------------------------------------------------------- 1D rules
def _legendre_ld(q: int, x):
    """P_q(x) and P_{q-1}(x) by the three-term recurrence, in long double."""
    x = np.asarray(x, dtype=LD)
    p0, p1 = np.ones_like(x), x.copy()
    if q == 0:
        return p0, np.zeros_like(x)
    for j in range(1, q):
        p0, p1 = p1, (LD(2 * j + 1) * x * p1 - LD(j) * p0) / LD(j + 1)
    return p1, p0


@functools.lru_cache(maxsize=None)
def gauss_legendre_ld(q: int):
    """q Gauss-Legendre nodes and weights on [0,1] in long double: Newton on
    P_q started from the double-precision nodes; w = 2 / ((1 - x^2) P_q'(x)^2)
    on [-1,1], halved for [0,1]."""
    x0, _ = np.polynomial.legendre.leggauss(q)
    x = x0.astype(LD)
    for _ in range(6):
        p, pm = _legendre_ld(q, x)
        dp = LD(q) * (x * p - pm) / (x * x - LD(1))
        x = x - p / dp
    p, pm = _legendre_ld(q, x)
    dp = LD(q) * (x * p - pm) / (x * x - LD(1))
    w = LD(2) / ((LD(1) - x * x) * dp * dp)
    return (x + LD(1)) / LD(2), w / LD(2)


@functools.lru_cache(maxsize=None)
def gauss_lobatto_ld(npts: int):
    """npts Gauss-Lobatto nodes on [0,1] in long double: the ends and the
    roots of P'_{npts-1}, by Newton with P'' from Legendre's equation
    (1 - x^2) P'' = 2 x P' - n (n+1) P."""
    n = npts - 1
    if n == 1:
        return np.array([LD(0), LD(1)])
    inner = np.sort(np.polynomial.legendre.Legendre.basis(n).deriv().roots().real).astype(LD)
    for _ in range(6):
        p, pm = _legendre_ld(n, inner)
        dp = LD(n) * (inner * p - pm) / (inner * inner - LD(1))
        d2p = (LD(2) * inner * dp - LD(n * (n + 1)) * p) / (LD(1) - inner * inner)
        inner = inner - dp / d2p
    return np.concatenate(([LD(0)], (inner + LD(1)) / LD(2), [LD(1)]))


def hex_rule_ld(q: int):
    """Tensor Gauss-Legendre rule (axis 0 fastest): points (q^3, 3), weights."""
    x, w = gauss_legendre_ld(q)
    X = np.array([[x[a], x[b], x[c]] for c in range(q) for b in range(q) for a in range(q)], dtype=LD)
    W = np.array([w[a] * w[b] * w[c] for c in range(q) for b in range(q) for a in range(q)], dtype=LD)
    return X, W


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


# ------------------------------------------------- conventions, written again
def _dofs_ld(k: int):
    """(d, i, j0, j1) of every local dof, interior dofs first (by d, j1, j0,
    then i innermost), then face f = 2d + s dofs (j0 fastest, i = s (k+1))."""
    rows = [(d, i, j0, j1) for d in range(3) for j1 in range(k + 1) for j0 in range(k + 1)
            for i in range(1, k + 1)]
    rows += [(f // 2, (f % 2) * (k + 1), j0, j1) for f in range(6) for j1 in range(k + 1) for j0 in range(k + 1)]
    return rows


def _signs_ld(k: int) -> np.ndarray:
    """eps_f = 2 s - 1 of every local face dof, in local face-dof order."""
    K2 = (k + 1) ** 2
    return np.array([LD(2 * (f % 2) - 1) for f in range(6) for _ in range(K2)], dtype=LD)


def _split_ld(k: int, code: int, natural: int = 0):
    """Kept local dofs, essential local dofs, and the kept positions that carry
    a multiplier (face dofs of faces neither essential nor natural)."""
    ni, K2 = 3 * k * (k + 1) ** 2, (k + 1) ** 2
    keep, ess, mult = list(range(ni)), [], []
    for f in range(6):
        dofs = [ni + f * K2 + j for j in range(K2)]
        if (code >> f) & 1:
            ess += dofs
            continue
        if not (natural >> f) & 1:
            mult += [len(keep) + j for j in range(K2)]
        keep += dofs
    return np.array(keep), np.array(ess, dtype=np.int64), np.array(mult, dtype=np.int64)


def _jacobian_ld(xe, X):
    """Trilinear Jacobians J[p, r, c] = d x_r / d xi_c and their determinants
    at the points X (P, 3) for the 8 vertex coordinates xe (vertex a+2b+4c at
    corner (a, b, c))."""
    P = X.shape[0]
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
    return J, det


def _combine_ld(alpha, mass, beta, divdiv):
    """M_T = alpha (mass term) + beta (div-div term)."""
    return LD(alpha) * mass + LD(beta) * divdiv


# ------------------------------------------------------------- element level
def element_matrix_ld(k: int, xyz_e: np.ndarray, alpha: float, beta: float, f=None):
    """M_T (n, n) in long double for one element (q = k+2 Gauss points); with
    an element load f (3,) also returns f_T (n,).

    M_T[i, j] = sum_q w_q / det J ( alpha (J phi_i).(J phi_j) + beta div phi_i
    div phi_j ), f_T[i] = sum_q w_q f . (J phi_i) (contravariant Piola map)."""
    X, W = hex_rule_ld(k + 2)
    zc, zo = gauss_lobatto_ld(k + 2), gauss_legendre_ld(k + 1)[0]
    dofs = _dofs_ld(k)
    n, P = len(dofs), X.shape[0]
    Lc = [_lagrange_ld(zc, X[:, a]) for a in range(3)]
    dLc = [_lagrange_deriv_ld(zc, X[:, a]) for a in range(3)]
    Lo = [_lagrange_ld(zo, X[:, a]) for a in range(3)]
    val = np.zeros((n, P), dtype=LD)
    div = np.zeros((n, P), dtype=LD)
    comp = np.array([d for d, _, _, _ in dofs])
    for idx, (d, i, j0, j1) in enumerate(dofs):
        t0, t1 = [a for a in range(3) if a != d]
        tang = Lo[t0][j0] * Lo[t1][j1]
        val[idx] = Lc[d][i] * tang
        div[idx] = dLc[d][i] * tang
    J, det = _jacobian_ld(np.asarray(xyz_e, dtype=LD), X)
    G = np.einsum("prd,pre->pde", J, J)                      # J^T J
    wd = W / det
    mass = np.zeros((n, n), dtype=LD)
    divdiv = np.zeros((n, n), dtype=LD)
    for i in range(n):
        gi = G[:, comp[i], :][:, comp]                       # (P, n): G[d_i, d_j]
        mass[i] = (wd[:, None] * gi * val[i][:, None] * val.T).sum(axis=0)
        divdiv[i] = (wd[:, None] * div[i][:, None] * div.T).sum(axis=0)
    M = _combine_ld(alpha, mass, beta, divdiv)
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
    """Solve L X = B."""
    B = np.array(B, dtype=LD)
    X = np.zeros_like(B)
    for i in range(L.shape[0]):
        X[i] = (B[i] - L[i, :i] @ X[:i]) / L[i, i]
    return X


def backward_ld(L, B):
    """Solve L^T X = B."""
    B = np.array(B, dtype=LD)
    X = np.zeros_like(B)
    n = L.shape[0]
    for i in range(n - 1, -1, -1):
        X[i] = (B[i] - L[i + 1:, i] @ X[i + 1:]) / L[i, i]
    return X


def _kept_load(k, M, fT, code, natural, g):
    """f_r - M_re g_e (g: the element's boundary face data, (6 (k+1)^2,), or None)."""
    keep, ess, _ = _split_ld(k, code, natural)
    ni = 3 * k * (k + 1) ** 2
    fr = np.array(fT[keep], dtype=LD)
    if g is not None and ess.size:
        fr -= M[np.ix_(keep, ess)] @ np.asarray(g, dtype=LD)[ess - ni]
    return fr


def local_schur_ld(k: int, M: np.ndarray, code: int, natural: int = 0) -> np.ndarray:
    """H_T = C_T M_rr^{-1} C_T^T in long double: Cholesky of the kept block,
    then (L^{-1} C^T)^T (L^{-1} C^T)."""
    keep, _, mpos = _split_ld(k, code, natural)
    ni = 3 * k * (k + 1) ** 2
    eps = _signs_ld(k)[keep[mpos] - ni]
    CT = np.zeros((mpos.size, keep.size), dtype=LD)
    CT[np.arange(mpos.size), mpos] = eps
    L = cholesky_ld(M[np.ix_(keep, keep)])
    Y = forward_ld(L, CT.T)
    return Y.T @ Y


def local_rhs_ld(k: int, M: np.ndarray, fT: np.ndarray, code: int, natural: int = 0, g=None) -> np.ndarray:
    """r_T = C_T M_rr^{-1} (f_r - M_re g_e) in long double."""
    keep, _, mpos = _split_ld(k, code, natural)
    ni = 3 * k * (k + 1) ** 2
    eps = _signs_ld(k)[keep[mpos] - ni]
    L = cholesky_ld(M[np.ix_(keep, keep)])
    x = backward_ld(L, forward_ld(L, _kept_load(k, M, fT, code, natural, g)))
    return eps * x[mpos]


def local_recover_ld(k: int, M: np.ndarray, fT: np.ndarray, code: int, lam_T: np.ndarray, natural: int = 0,
                     g=None) -> np.ndarray:
    """u_T = M_rr^{-1} (f_r - M_re g_e - C_T^T lam_T) on the kept dofs, g (or
    0) on the essential ones."""
    keep, ess, mpos = _split_ld(k, code, natural)
    ni = 3 * k * (k + 1) ** 2
    eps = _signs_ld(k)[keep[mpos] - ni]
    rhs = _kept_load(k, M, fT, code, natural, g)
    rhs[mpos] -= eps * np.asarray(lam_T, dtype=LD)
    L = cholesky_ld(M[np.ix_(keep, keep)])
    u = np.zeros(M.shape[0], dtype=LD)
    u[keep] = backward_ld(L, forward_ld(L, rhs))
    if g is not None and ess.size:
        u[ess] = np.asarray(g, dtype=LD)[ess - ni]
    return u


def _masks(topo, e: int, ess):
    """(essential, natural) 6-bit face masks of element e: a boundary face is
    essential unless ess[e, f] == 0."""
    code = nat = 0
    for f in range(6):
        if topo.elem_face[e, f] < 0:
            if ess is None or ess[e, f]:
                code |= 1 << f
            else:
                nat |= 1 << f
    return code, nat


def hybridize_ld(k: int, xyz, e2v, alpha, beta, f, topo, elements, lam=None, ess=None, g_face=None):
    """Long-double H (as a dict {(mu, nu): value}), r (dict {mu: value}) and,
    with lam, u for the given elements (dict {e: u_T}).  Rows of H and r are
    complete for every face whose two elements are both in ``elements``."""
    from . import topology as topo_mod
    H, r, U = {}, {}, {}
    for e in np.asarray(elements):
        e = int(e)
        code, nat = _masks(topo, e, ess)
        g = None if g_face is None else g_face[e]
        M, fT = element_matrix_ld(k, xyz[e2v[e]], float(alpha[e]), float(beta[e]), f[e])
        HT = local_schur_ld(k, M, code, nat)
        rT = local_rhs_ld(k, M, fT, code, nat, g)
        ids = [mu for (_, mu, _) in topo_mod.element_multipliers(topo, k, e) if mu >= 0]
        for a, mu in enumerate(ids):
            r[mu] = r.get(mu, LD(0)) + rT[a]
            for b, nu in enumerate(ids):
                H[(mu, nu)] = H.get((mu, nu), LD(0)) + HT[a, b]
        if lam is not None:
            U[e] = local_recover_ld(k, M, fT, code, np.asarray(lam)[ids], nat, g)
    return H, r, U


# ------------------------------------------------------------- noise floor
U64 = 2.0 ** -53


def kappa_scaled(k: int, xyz, e2v, alpha, beta, topo, elements, ess=None) -> float:
    """max over the elements of cond_2(D M_rr D), D = diag(M_rr)^{-1/2}: the
    condition number that bounds the relative error of a backward-stable FP64
    Cholesky solve of the kept element block (van der Sluis), so that an FP64
    H_T, r_T or u_T is within a small multiple of kappa_scaled 2^-53 of the
    exact value.  Computed in FP64 from the oracle's element matrices."""
    els = np.asarray(elements, dtype=np.int64)
    worst = 1.0
    for s, t, M, _ in element.element_system_chunked(k, xyz, e2v[els], alpha[els], beta[els], None):
        for i in range(t - s):
            code, nat = _masks(topo, int(els[s + i]), ess)
            keep, _, _ = _split_ld(k, code, nat)
            A = M[i][np.ix_(keep, keep)]
            d = 1.0 / np.sqrt(np.diag(A))
            worst = max(worst, float(np.linalg.cond(A * d[:, None] * d[None, :])))
    return worst
