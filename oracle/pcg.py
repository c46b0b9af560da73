"""Jacobi-preconditioned conjugate gradients on H lam = r (test infrastructure).

The paper solves the hybridized system with PCG and stops when the l2 norm of
the residual has dropped by a factor of 1e-12 (Sec. 6.1, the soft-hard weak
scaling runs).  Its preconditioner (BoomerAMG) is out of scope here; the diagonal of H
takes its place.  This is the textbook preconditioned CG (Hestenes-Stiefel with
the preconditioner applied to the residual, as in Saad, Iterative Methods for
Sparse Linear Systems, Sec. 9.2), starting from lam_0 = 0:

    r_0 = b, z_0 = D^{-1} r_0, p_0 = z_0
    alpha_j = (r_j, z_j) / (p_j, H p_j)
    lam_{j+1} = lam_j + alpha_j p_j,  r_{j+1} = r_j - alpha_j H p_j
    z_{j+1} = D^{-1} r_{j+1}
    beta_j = (r_{j+1}, z_{j+1}) / (r_j, z_j),  p_{j+1} = z_{j+1} + beta_j p_j

Plain numpy in FP64, one scipy sparse product per iteration.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def jacobi_pcg(H: sp.csr_matrix, b: np.ndarray, rtol: float = 1e-12, maxit: int = 10000,
               check_every: int = 1):
    """Return (lam, iters, converged, history) where history[j] = ||r_j||_2.

    The stopping test ||r_j|| <= rtol ||r_0|| is evaluated after every
    ``check_every`` iterations (and at j = 0), so a caller can mirror a solver
    that only looks at the residual every few iterations."""
    m = H.shape[0]
    lam = np.zeros(m)
    if m == 0:
        return lam, 0, True, [0.0]
    d = H.diagonal()
    dinv = np.where(d != 0.0, 1.0 / np.where(d != 0.0, d, 1.0), 0.0)
    r = np.array(b, dtype=np.float64)
    z = dinv * r
    p = z.copy()
    rz = r @ z
    rr0 = r @ r
    hist = [float(np.sqrt(rr0))]
    tol2 = rtol * rtol * rr0
    if rr0 == 0.0 or rr0 <= tol2:
        return lam, 0, True, hist
    it = 0
    conv = False
    while it < maxit:
        q = H @ p
        pq = p @ q
        alpha = rz / pq if pq != 0.0 else 0.0
        lam = lam + alpha * p
        r = r - alpha * q
        z = dinv * r
        rz_new = r @ z
        rr = r @ r
        hist.append(float(np.sqrt(rr)))
        beta = rz_new / rz if rz != 0.0 else 0.0
        rz = rz_new
        p = z + beta * p
        it += 1
        if it % check_every == 0 and rr <= tol2:
            conv = True
            break
    return lam, it, conv, hist
