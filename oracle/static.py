"""Static condensation of the H(div) system (test infrastructure).

Sec. 3.1: with the broken matrix split into interior dofs i and interface
copies b, the element Schur complements S_hat_T = A_bb - A_bi A_ii^{-1} A_ib
are assembled (not inverted, as for H) into the static condensation matrix
S = [I; W]^T S_hat [I; W] on one dof per interface dof.  With the interface
copies taken as outward fluxes W = -I; here the global face dof is the
owner's outward flux, so an element's face-dof copy is sigma x with
sigma = eps_f for the face's owner and -eps_f for its neighbour (the
convention of ``conforming.build_P``).  S acts on the multiplier-numbered
face dofs, so it has the sparsity of H.

Two independent routes:
* ``condense``: element by element (the algorithm), dense local solves,
  scipy COO assembly;
* ``condense_plain``: the Schur complement of the assembled conforming
  matrix A = P^T A_hat P onto its face dofs (the definition; small meshes).
Recovery: u_b = sigma x_b, u_i = A_ii^{-1} (f_i - A_ib u_b) per element.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

from . import conforming, element, hybrid, rt_basis, topology as topo_mod


@dataclasses.dataclass
class Condensed:
    k: int
    topo: topo_mod.Topology
    S: sp.csr_matrix
    r: np.ndarray
    mult_id: np.ndarray   # (ne, 6 (k+1)^2) face dof id of every local face dof, -1 on boundary


def face_dof_signs(topo, k: int, e: int) -> np.ndarray:
    """sigma of every local face dof of element e: +eps_f where e owns the
    face, -eps_f where it is the neighbour (0 on boundary faces)."""
    K2 = rt_basis.n_face(k)
    out = np.zeros(6 * K2)
    for f in range(6):
        F = int(topo.elem_face[e, f])
        if F < 0:
            continue
        eps = 2 * (f % 2) - 1
        owner = tuple(topo.face_owner[F]) == (e, f)
        out[f * K2:(f + 1) * K2] = eps if owner else -eps
    return out


def _local(k, M, fT, code, g_face):
    """S_hat_T and the condensed load on the element's interior-face dofs
    (boundary faces eliminated with their data g)."""
    keep, ess, mpos = hybrid._split(k, code)
    ni = rt_basis.n_interior(k)
    Mrr = M[:, keep][:, :, keep]
    fr = fT[:, keep].copy()
    if g_face is not None and ess.size:
        fr -= np.einsum("gij,gj->gi", M[:, keep][:, :, ess], g_face[:, ess - ni])
    ii = np.arange(ni)
    Aii, Aib = Mrr[:, :ni, :ni], Mrr[:, :ni][:, :, mpos]
    Abi, Abb = Mrr[:, mpos][:, :, :ni], Mrr[:, mpos][:, :, mpos]
    if ni:
        X = np.linalg.solve(Aii, np.concatenate([Aib, fr[:, ii, None]], axis=2))
        St = Abb - Abi @ X[:, :, :-1]
        gt = fr[:, mpos] - np.einsum("gbi,gi->gb", Abi, X[:, :, -1])
    else:
        St, gt = Abb, fr[:, mpos]
    return St, gt


def condense(k: int, xyz, e2v, alpha, beta, f, g_face=None, topo=None, q=None) -> Condensed:
    """S = sum_T sigma-scatter of S_hat_T and r = sum_T sigma g_T."""
    topo = topo or topo_mod.build_topology(e2v)
    mid = topo_mod.multiplier_map(topo, k)[0]
    m = topo.nfaces * rt_basis.n_face(k)
    ne = e2v.shape[0]
    rows, cols, vals = [], [], []
    r = np.zeros(m)
    sig_all = np.array([face_dof_signs(topo, k, e) for e in range(ne)])
    for s, t, M, fT in element.element_system_chunked(k, xyz, e2v, alpha, beta, f, q=q):
        ids_el = np.arange(s, t)
        codes = hybrid._ess_code_of(topo, ids_el)
        for code in np.unique(codes):
            sel = np.nonzero(codes == code)[0]
            gsel = None if g_face is None else g_face[ids_el[sel]]
            St, gt = _local(k, M[sel], fT[sel], int(code), gsel)
            ids = mid[ids_el[sel]]
            keepcols = ids[0] >= 0
            ids = ids[:, keepcols]
            sig = sig_all[ids_el[sel]][:, keepcols]
            mT = ids.shape[1]
            rows.append(np.repeat(ids, mT, axis=1).reshape(-1))
            cols.append(np.tile(ids, (1, mT)).reshape(-1))
            vals.append((sig[:, :, None] * St * sig[:, None, :]).reshape(-1))
            np.add.at(r, ids.reshape(-1), (sig * gt).reshape(-1))
    if rows:
        R, Cc, V = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    else:
        R = Cc = np.zeros(0, np.int64)
        V = np.zeros(0)
    S = sp.coo_matrix((V, (R, Cc)), shape=(m, m)).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    return Condensed(k, topo, S, r, mid)


def condense_plain(k: int, xyz, e2v, alpha, beta, f, g_face=None, q=None):
    """(S, r) as the Schur complement of the conforming system onto its face
    dofs: A = P^T A_hat P, b = P^T f_hat, S = A_ff - A_fi A_ii^{-1} A_if,
    r = b_f - A_fi A_ii^{-1} b_i (dense; small meshes)."""
    topo = topo_mod.build_topology(e2v)
    Ahat, fhat, _, _ = conforming.broken_system(k, xyz, e2v, alpha, beta, f, topo, g_face, q)
    P = conforming.build_P(k, topo)
    A = (P.T @ Ahat @ P).toarray()
    b = P.T @ fhat
    m = topo.nfaces * rt_basis.n_face(k)
    Aff, Afi, Aii = A[:m, :m], A[:m, m:], A[m:, m:]
    if Aii.size:
        X = np.linalg.solve(Aii, np.column_stack([Afi.T, b[m:]]))
        return Aff - Afi @ X[:, :-1], b[:m] - Afi @ X[:, -1]
    return Aff, b[:m]


def recover(cond: Condensed, xyz, e2v, alpha, beta, f, x, g_face=None, q=None) -> np.ndarray:
    """u (ne, n) from the face dofs x: u_b = sigma x_b, u_i = A_ii^{-1}
    (f_i - A_ib u_b), essential dofs = g."""
    k, topo = cond.k, cond.topo
    n, ni = rt_basis.ndofs(k), rt_basis.n_interior(k)
    ne = e2v.shape[0]
    u = np.zeros((ne, n))
    for s, t, M, fT in element.element_system_chunked(k, xyz, e2v, alpha, beta, f, q=q):
        for j in range(t - s):
            e = s + j
            code = int(hybrid._ess_code_of(topo, np.array([e]))[0])
            keep, ess, mpos = hybrid._split(k, code)
            ge = np.zeros(ess.size) if g_face is None else g_face[e, ess - ni]
            Mm = M[j]
            ids = cond.mult_id[e]
            sig = face_dof_signs(topo, k, e)
            ub = np.zeros(n - ni)
            live = ids >= 0
            ub[live] = sig[live] * x[ids[live]]
            if ess.size:
                ub[ess - ni] = ge
            fi = fT[j, :ni] - Mm[:ni, ni:] @ ub
            u[e, :ni] = np.linalg.solve(Mm[:ni, :ni], fi) if ni else fi
            u[e, ni:] = ub
    return u
