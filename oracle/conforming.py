"""The plain definition: conforming assembly and direct solve (test infrastructure).

Sec. 2.2: the conforming system is A x = f with A = P^T A_hat P and
f = P^T f_hat, where P maps global dofs to the local (broken) copies.  For RT
each interior-face dof has two copies; the global value is taken as the
owner's outward flux, so the owner copy is eps_o * x and the neighbour copy is
-eps_n * x (then eps_o u_o + eps_n u_n = 0, i.e. C P = 0, Sec. 2.3).  Interior
dofs map by identity.  Essential boundary-face dofs are eliminated first;
the dofs of natural boundary faces are global dofs of their one element.

Theorem 2.1 says the hybridized broken solution equals P x for the solution x
of this system; the tests check exactly that on small meshes.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import element, hybrid, rt_basis, topology as topo_mod


def _codes(topo, e: int, ess):
    code, nat = hybrid.face_codes(topo, np.array([e]), ess)
    return int(code[0]), int(nat[0])


def kept_layout(k: int, topo, ess=None):
    """Per element, the kept local dofs; and the offsets of each element's
    block in the stacked broken vector x_hat_r."""
    ne = topo.ne
    keeps, offs = [], [0]
    for e in range(ne):
        keep, _, _ = hybrid._split(k, *_codes(topo, e, ess))
        keeps.append(keep)
        offs.append(offs[-1] + keep.size)
    return keeps, np.array(offs)


def build_P(k: int, topo, ess=None) -> sp.csr_matrix:
    """P (n_hat_r x n): global dofs are the multiplier-numbered face dofs
    (0..m-1), then the dofs of natural boundary faces (one copy each, in
    element and local order), then every element's interior dofs."""
    ni, K = rt_basis.n_interior(k), k + 1
    K2 = K * K
    m = topo.nfaces * K2
    keeps, offs = kept_layout(k, topo, ess)
    nat_dofs = []
    for e in range(topo.ne):
        _, nat = _codes(topo, e, ess)
        for f in range(6):
            if (nat >> f) & 1:
                nat_dofs.extend((e, ni + f * K2 + j) for j in range(K2))
    nat_id = {key: m + t for t, key in enumerate(nat_dofs)}
    n0 = m + len(nat_dofs)
    n = n0 + topo.ne * ni
    rows, cols, vals = [], [], []
    for e in range(topo.ne):
        pos = {int(l): offs[e] + j for j, l in enumerate(keeps[e])}
        for li in range(ni):
            rows.append(pos[li]); cols.append(n0 + e * ni + li); vals.append(1.0)
        for loc, mu, eps in topo_mod.element_multipliers(topo, k, e):
            if mu < 0:
                if (e, loc) in nat_id:
                    rows.append(pos[loc]); cols.append(nat_id[(e, loc)]); vals.append(1.0)
                continue
            f = (loc - ni) // K2
            fid = int(topo.elem_face[e, f])
            owner = tuple(topo.face_owner[fid]) == (e, f)
            rows.append(pos[loc]); cols.append(mu); vals.append(float(eps if owner else -eps))
    return sp.csr_matrix((vals, (rows, cols)), shape=(int(offs[-1]), n))


def build_C(k: int, topo, ess=None) -> sp.csr_matrix:
    """C (m x n_hat_r): C[mu, copy] = eps_f of the copy's own face."""
    ni, K = rt_basis.n_interior(k), k + 1
    m = topo.nfaces * K * K
    keeps, offs = kept_layout(k, topo, ess)
    rows, cols, vals = [], [], []
    for e in range(topo.ne):
        pos = {int(l): offs[e] + j for j, l in enumerate(keeps[e])}
        for loc, mu, eps in topo_mod.element_multipliers(topo, k, e):
            if mu >= 0:
                rows.append(mu); cols.append(pos[loc]); vals.append(float(eps))
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, int(offs[-1])))


def broken_system(k: int, xyz, e2v, alpha, beta, f, topo, g_face=None, q=None, ess=None):
    """A_hat_r = blockdiag(M_rr) and f_hat_r = f_r - M_re g_e, stacked."""
    keeps, offs = kept_layout(k, topo, ess)
    ni = rt_basis.n_interior(k)
    blocks, rhs = [], []
    for s, t, M, fT in element.element_system_chunked(k, xyz, e2v, alpha, beta, f, q=q):
        for i in range(t - s):
            e = s + i
            keep = keeps[e]
            _, ess_dofs, _ = hybrid._split(k, *_codes(topo, e, ess))
            fr = fT[i, keep].copy()
            if g_face is not None and ess_dofs.size:
                fr -= M[i][np.ix_(keep, ess_dofs)] @ g_face[e, ess_dofs - ni]
            blocks.append(M[i][np.ix_(keep, keep)])
            rhs.append(fr)
    return sp.block_diag(blocks, format="csr"), np.concatenate(rhs), keeps, offs


def conforming_solve(k: int, xyz, e2v, alpha, beta, f, g_face=None, q=None, ess=None):
    """x_hat = P x with P^T A_hat P x = P^T f_hat (dense or sparse direct);
    returns u (ne, n) in local order (essential dofs = g)."""
    topo = topo_mod.build_topology(e2v)
    Ahat, fhat, keeps, offs = broken_system(k, xyz, e2v, alpha, beta, f, topo, g_face, q, ess)
    P = build_P(k, topo, ess)
    A = (P.T @ Ahat @ P).tocsc()
    b = P.T @ fhat
    x = np.linalg.solve(A.toarray(), b) if A.shape[0] <= 3000 else spla.spsolve(A, b)
    xhat = P @ x
    n, ni = rt_basis.ndofs(k), rt_basis.n_interior(k)
    u = np.zeros((topo.ne, n))
    for e in range(topo.ne):
        u[e, keeps[e]] = xhat[offs[e]:offs[e + 1]]
        _, ess_dofs, _ = hybrid._split(k, *_codes(topo, e, ess))
        if g_face is not None and ess_dofs.size:
            u[e, ess_dofs] = g_face[e, ess_dofs - ni]
    return u
