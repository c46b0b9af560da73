"""Algebraic hybridization, element by element (test infrastructure).

Theorem 2.1: with A_hat = blockdiag(M_T) SPD and C full row rank with
Null(C) = Range(P), the multipliers solve H lam = C A_hat^{-1} f_hat with
H = C A_hat^{-1} C^T (SPD), and the broken solution is
x_hat = A_hat^{-1} (f_hat - C^T lam).  Because A_hat is block diagonal, H is
the sum over elements of H_T = C_T M_T^{-1} C_T^T (Sec. 3.1: H assembles the
inverses of the local Schur complements onto the face dofs).

Essential dofs (by default every face on the domain boundary) are
eliminated from each element matrix first (Sec. 5): only the rows/columns of
the remaining ("r") dofs are kept and the load is corrected by -M_re g_e.
Boundary faces marked natural keep their dofs as unknowns of the element and
carry no multiplier.  C_T is the signed selection of the element's
interior-face dofs: C_T[a, face dof a] = eps_f.

Each local solve here is a plain dense ``numpy.linalg.solve`` on the kept
block; the global matrix is formed by COO triplets summed by scipy.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import element, rt_basis, topology as topo_mod


def _ess_code_of(topo, els: np.ndarray) -> np.ndarray:
    """6-bit mask per element: bit f set when local face f is on the boundary."""
    bnd = topo.elem_face[els] < 0
    return (bnd * (1 << np.arange(6))).sum(axis=1)


def face_codes(topo, els: np.ndarray, ess=None):
    """Per element, the 6-bit masks of its essential and of its natural
    boundary faces.  A boundary face is essential (its normal flux prescribed,
    its dofs eliminated, Sec. 5) unless ``ess`` (ne, 6) is given and holds 0
    for it: then it is natural (its dofs stay unknowns of the element and get
    no multiplier).  ``ess`` entries of interior faces are not read."""
    els = np.asarray(els, dtype=np.int64)
    bnd = topo.elem_face[els] < 0
    esm = bnd if ess is None else bnd & (np.asarray(ess)[els] != 0)
    bits = 1 << np.arange(6)
    return (esm * bits).sum(axis=1), ((bnd & ~esm) * bits).sum(axis=1)


def _split(k: int, code: int, natural: int = 0):
    """Kept local dofs (ascending), essential local dofs, and the positions
    (within the kept list) of the multiplier dofs, for the essential-face mask
    ``code`` and the natural-face mask ``natural`` (kept, no multiplier)."""
    ni, K2 = rt_basis.n_interior(k), rt_basis.n_face(k)
    keep = list(range(ni))
    ess = []
    mult_pos = []
    for f in range(6):
        block = list(range(ni + f * K2, ni + (f + 1) * K2))
        if (code >> f) & 1:
            ess.extend(block)
        else:
            if not (natural >> f) & 1:
                mult_pos.extend(range(len(keep), len(keep) + K2))
            keep.extend(block)
    return np.array(keep), np.array(ess, dtype=np.int64), np.array(mult_pos, dtype=np.int64)


def _face_signs(k: int) -> np.ndarray:
    """eps of every local face dof (6 (k+1)^2,) in local face-dof order."""
    K2 = rt_basis.n_face(k)
    return np.repeat([2 * (f % 2) - 1 for f in range(6)], K2).astype(np.float64)


def local_schur(k: int, M: np.ndarray, fT: np.ndarray, code: int, g_face: np.ndarray | None = None,
                natural: int = 0):
    """H_T = C_T M_rr^{-1} C_T^T and r_T = C_T M_rr^{-1} (f_r - M_re g_e) for a
    batch of elements sharing the boundary mask ``code``.

    M (G, n, n), fT (G, n), g_face (G, 6 (k+1)^2) or None.  Returns
    H_T (G, mT, mT), r_T (G, mT), with rows in the element's local face-dof
    order restricted to interior faces."""
    keep, ess, mpos = _split(k, code, natural)
    ni = rt_basis.n_interior(k)
    Mrr = M[:, keep][:, :, keep]
    fr = fT[:, keep].copy()
    if g_face is not None and ess.size:
        ge = g_face[:, ess - ni]
        fr -= np.einsum("gij,gj->gi", M[:, keep][:, :, ess], ge)
    eps = _face_signs(k)[keep[mpos] - ni]
    G, nr, mT = M.shape[0], keep.size, mpos.size
    CT = np.zeros((mT, nr))
    CT[np.arange(mT), mpos] = eps
    rhs = np.concatenate([np.broadcast_to(CT.T, (G, nr, mT)), fr[:, :, None]], axis=2)
    X = np.linalg.solve(Mrr, rhs)
    HT = np.einsum("an,gnb->gab", CT, X[:, :, :mT])
    rT = np.einsum("an,gn->ga", CT, X[:, :, mT])
    return HT, rT


def local_recover(k: int, M: np.ndarray, fT: np.ndarray, code: int, lam_T: np.ndarray,
                  g_face: np.ndarray | None = None, natural: int = 0) -> np.ndarray:
    """x_hat_T = M_rr^{-1} (f_r - M_re g_e - C_T^T lam_T) on the kept dofs and
    g on the essential ones; returns u (G, n) in local order."""
    keep, ess, mpos = _split(k, code, natural)
    ni = rt_basis.n_interior(k)
    G, n = fT.shape
    Mrr = M[:, keep][:, :, keep]
    fr = fT[:, keep].copy()
    ge = np.zeros((G, ess.size)) if g_face is None else g_face[:, ess - ni]
    if ess.size:
        fr -= np.einsum("gij,gj->gi", M[:, keep][:, :, ess], ge)
    eps = _face_signs(k)[keep[mpos] - ni]
    fr[:, mpos] -= eps[None, :] * lam_T
    u = np.zeros((G, n))
    u[:, keep] = np.linalg.solve(Mrr, fr[:, :, None])[:, :, 0]
    u[:, ess] = ge
    return u


@dataclasses.dataclass
class Hybridized:
    k: int
    topo: topo_mod.Topology
    H: sp.csr_matrix
    r: np.ndarray
    mult_id: np.ndarray   # (ne, 6 (k+1)^2) multiplier id of every local face dof, -1 on boundary
    ess: np.ndarray | None = None   # (ne, 6) essential-face flags of the boundary faces, None = all


def hybridize(k: int, xyz, e2v, alpha, beta, f, g_face=None, topo=None, q=None, elements=None, mult_id=None,
              ess=None):
    """Global H (CSR, sorted, duplicates summed) and r = sum_T C_T^T-scatter of
    r_T.  ``elements`` (index array) restricts the element loop, for sampled
    checks and timing samples: H and r then hold only those elements' terms
    (a row of H is complete when both elements of its face are included).
    ``ess`` (ne, 6): boundary faces with 0 are natural (``face_codes``)."""
    topo = topo or topo_mod.build_topology(e2v)
    mid = topo_mod.multiplier_map(topo, k)[0] if mult_id is None else mult_id
    m = topo.nfaces * rt_basis.n_face(k)
    els = np.arange(e2v.shape[0]) if elements is None else np.asarray(elements, dtype=np.int64)
    rows, cols, vals = [], [], []
    r = np.zeros(m)
    for s, t, M, fT in element.element_system_chunked(k, xyz, e2v[els], alpha[els], beta[els], f[els], q=q):
        ids_el = els[s:t]
        codes, nats = face_codes(topo, ids_el, ess)
        keys = codes + 64 * nats
        for key in np.unique(keys):
            sel = np.nonzero(keys == key)[0]
            gsel = None if g_face is None else g_face[ids_el[sel]]
            HT, rT = local_schur(k, M[sel], fT[sel], int(key % 64), gsel, int(key // 64))
            keep_ids = mid[ids_el[sel]]
            ids = keep_ids[:, keep_ids[0] >= 0]          # same mask -> same kept columns
            mT = ids.shape[1]
            rows.append(np.repeat(ids, mT, axis=1).reshape(-1))
            cols.append(np.tile(ids, (1, mT)).reshape(-1))
            vals.append(HT.reshape(-1))
            np.add.at(r, ids.reshape(-1), rT.reshape(-1))
    if rows:
        R, Cc, V = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    else:
        R = Cc = np.zeros(0, np.int64)
        V = np.zeros(0)
    H = sp.coo_matrix((V, (R, Cc)), shape=(m, m)).tocsr()
    H.sum_duplicates()
    H.sort_indices()
    return Hybridized(k, topo, H, r, mid, None if ess is None else np.asarray(ess))


def solve_reduced(H: sp.csr_matrix, r: np.ndarray, rtol: float = 1e-14) -> np.ndarray:
    """lam = H^{-1} r: dense Cholesky-based solve for small systems, sparse
    direct (SuperLU) otherwise."""
    m = H.shape[0]
    if m == 0:
        return np.zeros(0)
    if m <= 4000:
        return np.linalg.solve(H.toarray(), r)
    return spla.spsolve(H.tocsc(), r)


def recover(hyb: Hybridized, xyz, e2v, alpha, beta, f, lam, g_face=None, q=None, elements=None):
    """Broken solution u (len(elements) or ne, n) from multipliers lam
    (Theorem 2.1 back substitution), element by element."""
    k, topo = hyb.k, hyb.topo
    n = rt_basis.ndofs(k)
    els = np.arange(e2v.shape[0]) if elements is None else np.asarray(elements, dtype=np.int64)
    u = np.zeros((els.size, n))
    for s, t, M, fT in element.element_system_chunked(k, xyz, e2v[els], alpha[els], beta[els], f[els], q=q):
        ids_el = els[s:t]
        codes, nats = face_codes(topo, ids_el, hyb.ess)
        keys = codes + 64 * nats
        for key in np.unique(keys):
            sel = np.nonzero(keys == key)[0]
            ids = hyb.mult_id[ids_el[sel]]
            ids = ids[:, ids[0] >= 0]
            gsel = None if g_face is None else g_face[ids_el[sel]]
            u[s + sel] = local_recover(k, M[sel], fT[sel], int(key % 64), lam[ids], gsel, int(key // 64))
    return u


def equilibrium_residual(k: int, topo, M: np.ndarray, fT: np.ndarray, u: np.ndarray, lam_T_full: np.ndarray):
    """M_T u_T + C_T^T lam_T - f_T on the kept dofs of one element (the local
    equations of the saddle-point system in Theorem 2.1).  ``lam_T_full`` has
    one entry per local face dof (0 on boundary faces)."""
    ni = rt_basis.n_interior(k)
    res = M @ u - fT
    res[ni:] += _face_signs(k) * lam_T_full
    return res
