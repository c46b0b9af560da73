"""The M_s-weighted constraint of Example 2.3 (test infrastructure).

Deriving C from the bilinear form c(u, lambda) = integral over the interface
of [[u . n]] lambda, with a multiplier space M on the faces, gives
C' = M_s C, M_s the mass matrix between M and the normal traces of the broken
space (Example 2.3).  Then H' = C' A^{-1} C'^T = M_s H M_s^T, r' = M_s r and
lambda' = M_s^{-T} lambda, while the broken solution is unchanged (Theorem 2.1
holds for any C with the same null space).

Here M on a face is Q_k with the Lagrange basis at the face dofs' tangential
nodes, so M_s is computed per face by quadrature of psi_i (phi_j . e_d) over
the reference face, with a rule exact for the products.  On this basis it
comes out diagonal, w_a w_b with the Gauss-Legendre weights of the open
points (a closed form the pins check), identical on all six faces and
invariant under the face symmetries, so the same block serves the owner and
the neighbour frame.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import legendre as npleg

from . import hybrid, rt_basis


def face_mass(k: int, f: int) -> np.ndarray:
    """M_s of local face f = 2d + s: (K2, K2) with rows the multiplier basis
    psi_(a0, a1) = l_a0(t0) l_a1(t1) and columns the face dofs (j0, j1),
    integral over the reference face of psi (phi . e_d)."""
    d, s = f // 2, f % 2
    t0, t1 = rt_basis.tangential_axes(d)
    q = k + 3                                     # exact well beyond degree 2k per direction
    x, w = npleg.leggauss(q)
    x, w = (x + 1.0) / 2.0, w / 2.0
    X = np.zeros((q * q, 3))
    X[:, d] = float(s)
    X[:, t0] = np.tile(x, q)
    X[:, t1] = np.repeat(x, q)
    W = np.tile(w, q) * np.repeat(w, q)
    val, _ = rt_basis.rt_eval(k, X)               # (n, P, 3)
    K2 = rt_basis.n_face(k)
    ni = rt_basis.n_interior(k)
    z = rt_basis.open_points(k)
    L0 = rt_basis.lagrange(z, X[:, t0])           # (k+1, P)
    L1 = rt_basis.lagrange(z, X[:, t1])
    psi = np.array([L0[a0] * L1[a1] for a1 in range(k + 1) for a0 in range(k + 1)])   # (K2, P)
    trace = val[ni + f * K2: ni + (f + 1) * K2, :, d]                                  # (K2, P)
    return (psi * W) @ trace.T


def weights_vector(k: int, m: int) -> np.ndarray:
    """The diagonal of M_s over all multipliers (m = nfaces (k+1)^2): the
    diagonal of face_mass repeated per face."""
    dg = np.diag(face_mass(k, 1))
    K2 = rt_basis.n_face(k)
    return np.tile(dg, m // K2)


def hybridize_weighted(k: int, xyz, e2v, alpha, beta, f, g_face=None):
    """(H', r', plain hybridization) with C' = M_s C."""
    hy = hybrid.hybridize(k, xyz, e2v, alpha, beta, f, g_face)
    ms = weights_vector(k, hy.r.size)
    D = sp.diags(ms)
    Hw = (D @ hy.H @ D).tocsr()
    Hw.sort_indices()
    return Hw, ms * hy.r, hy
