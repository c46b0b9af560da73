"""The plain definition: conforming assembly and direct solve (test infrastructure).

Sec. 2.2: the conforming system is A x = f with A = P^T A_hat P and
f = P^T f_hat, where P maps global dofs to the local (broken) copies.  For RT
each interior-face dof has two copies; the global value is taken as the
owner's outward flux, so the owner copy is eps_o * x and the neighbour copy is
-eps_n * x (then eps_o u_o + eps_n u_n = 0, i.e. C P = 0, Sec. 2.3).  Interior
dofs map by identity.  Essential (boundary-face) dofs are eliminated first.

Theorem 2.1 says the hybridized broken solution equals P x for the solution x
of this system; the tests check exactly that on small meshes.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import element, hybrid, rt_basis, topology as topo_mod


def kept_layout(k: int, topo):
    """Per element, the kept local dofs; and the offsets of each element's
    block in the stacked broken vector x_hat_r."""
    ne = topo.ne
    keeps, offs = [], [0]
    for e in range(ne):
        code = int(((topo.elem_face[e] < 0) * (1 << np.arange(6))).sum())
        keep, _, _ = hybrid._split(k, code)
        keeps.append(keep)
        offs.append(offs[-1] + keep.size)
    return keeps, np.array(offs)


def build_P(k: int, topo) -> sp.csr_matrix:
    """P (n_hat_r x n): global dofs are the multiplier-numbered face dofs
    (0..m-1) followed by every element's interior dofs."""
    ni, K = rt_basis.n_interior(k), k + 1
    m = topo.nfaces * K * K
    n = m + topo.ne * ni
    keeps, offs = kept_layout(k, topo)
    rows, cols, vals = [], [], []
    for e in range(topo.ne):
        pos = {int(l): offs[e] + j for j, l in enumerate(keeps[e])}
        for li in range(ni):
            rows.append(pos[li]); cols.append(m + e * ni + li); vals.append(1.0)
        for loc, mu, eps in topo_mod.element_multipliers(topo, k, e):
            if mu < 0:
                continue
            f = (loc - ni) // (K * K)
            fid = int(topo.elem_face[e, f])
            owner = tuple(topo.face_owner[fid]) == (e, f)
            rows.append(pos[loc]); cols.append(mu); vals.append(float(eps if owner else -eps))
    return sp.csr_matrix((vals, (rows, cols)), shape=(int(offs[-1]), n))


def build_C(k: int, topo) -> sp.csr_matrix:
    """C (m x n_hat_r): C[mu, copy] = eps_f of the copy's own face."""
    ni, K = rt_basis.n_interior(k), k + 1
    m = topo.nfaces * K * K
    keeps, offs = kept_layout(k, topo)
    rows, cols, vals = [], [], []
    for e in range(topo.ne):
        pos = {int(l): offs[e] + j for j, l in enumerate(keeps[e])}
        for loc, mu, eps in topo_mod.element_multipliers(topo, k, e):
            if mu >= 0:
                rows.append(mu); cols.append(pos[loc]); vals.append(float(eps))
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, int(offs[-1])))


def broken_system(k: int, xyz, e2v, alpha, beta, f, topo, g_face=None, q=None):
    """A_hat_r = blockdiag(M_rr) and f_hat_r = f_r - M_re g_e, stacked."""
    keeps, offs = kept_layout(k, topo)
    ni = rt_basis.n_interior(k)
    blocks, rhs = [], []
    for s, t, M, fT in element.element_system_chunked(k, xyz, e2v, alpha, beta, f, q=q):
        for i in range(t - s):
            e = s + i
            keep = keeps[e]
            code = int(((topo.elem_face[e] < 0) * (1 << np.arange(6))).sum())
            _, ess, _ = hybrid._split(k, code)
            fr = fT[i, keep].copy()
            if g_face is not None and ess.size:
                fr -= M[i][np.ix_(keep, ess)] @ g_face[e, ess - ni]
            blocks.append(M[i][np.ix_(keep, keep)])
            rhs.append(fr)
    return sp.block_diag(blocks, format="csr"), np.concatenate(rhs), keeps, offs


def conforming_solve(k: int, xyz, e2v, alpha, beta, f, g_face=None, q=None):
    """x_hat = P x with P^T A_hat P x = P^T f_hat (dense or sparse direct);
    returns u (ne, n) in local order (essential dofs = g)."""
    topo = topo_mod.build_topology(e2v)
    Ahat, fhat, keeps, offs = broken_system(k, xyz, e2v, alpha, beta, f, topo, g_face, q)
    P = build_P(k, topo)
    A = (P.T @ Ahat @ P).tocsc()
    b = P.T @ fhat
    x = np.linalg.solve(A.toarray(), b) if A.shape[0] <= 3000 else spla.spsolve(A, b)
    xhat = P @ x
    n, ni = rt_basis.ndofs(k), rt_basis.n_interior(k)
    u = np.zeros((topo.ne, n))
    for e in range(topo.ne):
        u[e, keeps[e]] = xhat[offs[e]:offs[e + 1]]
        code = int(((topo.elem_face[e] < 0) * (1 << np.arange(6))).sum())
        _, ess, _ = hybrid._split(k, code)
        if g_face is not None and ess.size:
            u[e, ess] = g_face[e, ess - ni]
    return u
