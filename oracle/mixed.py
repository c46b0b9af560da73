"""Hybridized mixed form, an independent route to H_T (test infrastructure).

Sec. 3.2: with the auxiliary unknown q = div u, the element matrix splits as
A_hat = B^T W^{-1} B + M (eq. (discrete_hdiv)), and the reduced matrix of
the 3x3 block system [[M, B^T, C^T], [B, -W, 0], [C, 0, 0]] equals H,
because the (1,1) block of [[M, B^T], [B, -W]]^{-1} is (M + B^T W^{-1} B)^{-1}.

Here the q-space is Q_k on the reference cube (tensor Lagrange on the open
points) mapped by q = q_hat / det J, so that div u = div_hat u_hat / det J
lies in it.  With mass coefficient alpha and div-div coefficient beta:

  M[i,j] = sum_q w/detJ alpha (J phi_i).(J phi_j)
  B[p,i] = sum_q w/detJ q_hat_p div_hat phi_i
  W[p,p'] = sum_q w/detJ q_hat_p q_hat_p' / beta
"""
from __future__ import annotations

import numpy as np

from . import geometry, hybrid, quadrature, rt_basis


def pressure_basis(k: int, X: np.ndarray) -> np.ndarray:
    """Q_k tensor Lagrange basis on the open points, at X: ((k+1)^3, P)."""
    zo = rt_basis.open_points(k)
    L = [rt_basis.lagrange(zo, X[:, a]) for a in range(3)]
    K = k + 1
    out = np.zeros((K ** 3, X.shape[0]))
    for c in range(K):
        for b in range(K):
            for a in range(K):
                out[a + K * (b + K * c)] = L[0][a] * L[1][b] * L[2][c]
    return out


def mixed_blocks(k: int, xyz_e: np.ndarray, alpha: float, beta: float, q: int | None = None):
    """M (n,n), B ((k+1)^3, n), W ((k+1)^3, (k+1)^3) for one element."""
    q = q or (k + 2)
    X, Wq = quadrature.hex_rule(q)
    val, div = rt_basis.rt_eval(k, X)
    J = geometry.jacobians(xyz_e[None], X)[0]
    detJ = np.linalg.det(J)
    Jphi = np.einsum("prc,npc->npr", J, val)
    wd = Wq / detJ
    qh = pressure_basis(k, X)
    M = alpha * np.einsum("p,npr,mpr->nm", wd, Jphi, Jphi)
    B = np.einsum("p,ap,np->an", wd, qh, div)
    W = np.einsum("p,ap,bp->ab", wd, qh, qh) / beta
    return M, B, W


def mixed_local_schur(k: int, xyz_e: np.ndarray, alpha: float, beta: float, code: int, q=None):
    """H~_T = C_T ([[M, B^T], [B, -W]]^{-1})_{11} C_T^T on the kept dofs."""
    M, B, W = mixed_blocks(k, xyz_e, alpha, beta, q)
    keep, _, mpos = hybrid._split(k, code)
    ni = rt_basis.n_interior(k)
    Mr = M[np.ix_(keep, keep)]
    Br = B[:, keep]
    nr, npr = keep.size, B.shape[0]
    K = np.zeros((nr + npr, nr + npr))
    K[:nr, :nr] = Mr
    K[:nr, nr:] = Br.T
    K[nr:, :nr] = Br
    K[nr:, nr:] = -W
    eps = hybrid._face_signs(k)[keep[mpos] - ni]
    CT = np.zeros((mpos.size, nr))
    CT[np.arange(mpos.size), mpos] = eps
    rhs = np.zeros((nr + npr, mpos.size))
    rhs[:nr] = CT.T
    Y = np.linalg.solve(K, rhs)[:nr]
    return CT @ Y
