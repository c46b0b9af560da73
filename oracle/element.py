"""Element matrices and loads of the H(div) form (test infrastructure).

The bilinear form is (alpha u, v) + (beta div u, div v) and the load is
(f, v) (Sec. 3.2, eq. (weak_hdiv), with the mass coefficient called alpha
here).  Element matrices are the local forms evaluated on the element basis
(Sec. 2.1); they are SPD because of the mass term.

RT functions are carried by the contravariant Piola map
u = J u_hat / det J, so div u = div_hat u_hat / det J and

  M_T[i,j] = sum_q w_q / detJ_q * ( alpha (J phi_i).(J phi_j)
                                    + beta div_hat phi_i div_hat phi_j )
  f_T[i]   = sum_q w_q f . (J phi_i)

with f constant on the element.  A quadrature of q = k+2 Gauss points per
direction is the default.
"""
from __future__ import annotations

import numpy as np

from . import geometry, quadrature, rt_basis


def element_system(k: int, xyz_e: np.ndarray, alpha, beta, f=None, q: int | None = None):
    """M_T (E, n, n) and, if ``f`` (E, 3) is given, f_T (E, n) for a batch of
    elements with coordinates ``xyz_e`` (E, 8, 3) and per-element coefficients
    ``alpha``, ``beta`` (E,)."""
    q = q or (k + 2)
    X, W = quadrature.hex_rule(q)
    val, div = rt_basis.rt_eval(k, X)                       # (n,P,3), (n,P)
    J = geometry.jacobians(xyz_e, X)                         # (E,P,3,3)
    detJ = np.linalg.det(J)                                  # (E,P)
    if np.any(detJ <= 0.0):
        raise ValueError("non-positive Jacobian determinant")
    Jphi = np.einsum("eprc,npc->enpr", J, val)              # (E,n,P,3)
    wdet = W[None, :] / detJ                                 # (E,P)
    alpha = np.asarray(alpha, dtype=np.float64).reshape(-1)
    beta = np.asarray(beta, dtype=np.float64).reshape(-1)
    mass = np.einsum("ep,enpr,empr->enm", wdet, Jphi, Jphi)
    divdiv = np.einsum("ep,np,mp->enm", wdet, div, div)
    M = alpha[:, None, None] * mass + beta[:, None, None] * divdiv
    if f is None:
        return M, None
    fT = np.einsum("p,er,enpr->en", W, np.asarray(f, dtype=np.float64), Jphi)
    return M, fT


def element_system_chunked(k: int, xyz: np.ndarray, e2v: np.ndarray, alpha, beta, f=None,
                           chunk: int | None = None, q: int | None = None):
    """``element_system`` over a whole mesh in chunks; yields
    (start, stop, M, fT)."""
    n = rt_basis.ndofs(k)
    ne = e2v.shape[0]
    if chunk is None:
        chunk = max(1, int(2.0e8 // (n * (q or k + 2) ** 3 * 3 * 8 * 2)))
    for s in range(0, ne, chunk):
        t = min(ne, s + chunk)
        xe = xyz[e2v[s:t]]
        M, fT = element_system(k, xe, alpha[s:t], beta[s:t], None if f is None else f[s:t], q)
        yield s, t, M, fT
