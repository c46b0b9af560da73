"""RT_k reference basis on the unit cube (test infrastructure, see package doc).

The paper leaves the finite element basis to its library (Sec. 5); this oracle
fixes a standard nodal choice:

* closed 1D points: the k+2 Gauss-Lobatto points on [0,1] (ends included);
* open 1D points:   the k+1 Gauss-Legendre points on [0,1];
* the x_d-component basis function with indices (i, j0, j1) is
  l^c_i(xi_d) l^o_j0(xi_t0) l^o_j1(xi_t1) e_d, where (t0, t1) are the two
  axes other than d in increasing order.  Its degree of freedom is the
  reference normal component u_hat . e_d at the node (z^c_i, z^o_j0, z^o_j1).

Local order ("i-first", the 2x2 interior/boundary split of Sec. 5): the
interior dofs (1 <= i <= k) come first, ordered by d, then j1, then j0, then i
(innermost); then the face dofs, face f = 2d + s (side s: xi_d = s) at index
n_i + f (k+1)^2 + j0 + (k+1) j1, which are the dofs with i = s (k+1).
"""
from __future__ import annotations

import functools

import numpy as np
from numpy.polynomial import legendre as npleg


def tangential_axes(d: int) -> tuple[int, int]:
    """The two axes other than ``d``, in increasing order."""
    t = [a for a in range(3) if a != d]
    return t[0], t[1]


@functools.lru_cache(maxsize=None)
def open_points(k: int) -> np.ndarray:
    """k+1 Gauss-Legendre points on [0,1] (numpy's leggauss, mapped)."""
    x, _ = npleg.leggauss(k + 1)
    return (x + 1.0) / 2.0


@functools.lru_cache(maxsize=None)
def closed_points(k: int) -> np.ndarray:
    """k+2 Gauss-Lobatto points on [0,1]: 0, 1 and the roots of P'_{k+1}."""
    if k == 0:
        inner = np.zeros(0)
    else:
        inner = np.sort(npleg.Legendre.basis(k + 1).deriv().roots().real)
    return np.concatenate(([0.0], (inner + 1.0) / 2.0, [1.0]))


def lagrange(z: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Lagrange polynomials on nodes ``z`` evaluated at ``x``: shape (len(z), len(x))."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones((len(z), x.size))
    for i in range(len(z)):
        for j in range(len(z)):
            if j != i:
                out[i] *= (x - z[j]) / (z[i] - z[j])
    return out


def lagrange_deriv(z: np.ndarray, x: np.ndarray) -> np.ndarray:
    """First derivatives of the Lagrange polynomials on ``z`` at ``x``
    (product rule, one dropped factor at a time)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((len(z), x.size))
    for i in range(len(z)):
        for m in range(len(z)):
            if m == i:
                continue
            term = np.full(x.size, 1.0 / (z[i] - z[m]))
            for j in range(len(z)):
                if j != i and j != m:
                    term = term * (x - z[j]) / (z[i] - z[j])
            out[i] += term
    return out


def ndofs(k: int) -> int:
    """Broken RT_k dofs per hexahedron: 3 (k+1)^2 (k+2)."""
    return 3 * (k + 1) ** 2 * (k + 2)


def n_interior(k: int) -> int:
    return 3 * k * (k + 1) ** 2


def n_face(k: int) -> int:
    """Dofs per face: (k+1)^2."""
    return (k + 1) ** 2


@functools.lru_cache(maxsize=None)
def dof_table(k: int) -> np.ndarray:
    """Rows (d, i, j0, j1) in local (i-first) order."""
    rows = []
    for d in range(3):
        for j1 in range(k + 1):
            for j0 in range(k + 1):
                for i in range(1, k + 1):
                    rows.append((d, i, j0, j1))
    for f in range(6):
        d, s = divmod(f, 2)
        for j1 in range(k + 1):
            for j0 in range(k + 1):
                rows.append((d, s * (k + 1), j0, j1))
    tab = np.array(rows, dtype=np.int64).reshape(-1, 4)
    assert tab.shape[0] == ndofs(k)
    return tab


def face_dof_index(k: int, f: int, j0: int, j1: int) -> int:
    return n_interior(k) + f * n_face(k) + j0 + (k + 1) * j1


def rt_eval(k: int, X: np.ndarray):
    """Reference basis at points X (P, 3).

    Returns ``val`` (n, P, 3), the vector basis functions, and ``div`` (n, P),
    their reference divergence."""
    X = np.asarray(X, dtype=np.float64)
    zc, zo = closed_points(k), open_points(k)
    tab = dof_table(k)
    n, P = tab.shape[0], X.shape[0]
    val = np.zeros((n, P, 3))
    div = np.zeros((n, P))
    Lc = [lagrange(zc, X[:, a]) for a in range(3)]
    dLc = [lagrange_deriv(zc, X[:, a]) for a in range(3)]
    Lo = [lagrange(zo, X[:, a]) for a in range(3)]
    for idx, (d, i, j0, j1) in enumerate(tab):
        t0, t1 = tangential_axes(int(d))
        tang = Lo[t0][j0] * Lo[t1][j1]
        val[idx, :, d] = Lc[d][i] * tang
        div[idx] = dLc[d][i] * tang
    return val, div


def dof_nodes(k: int) -> np.ndarray:
    """Reference node (n, 3) of every dof, and its direction is e_d."""
    zc, zo = closed_points(k), open_points(k)
    tab = dof_table(k)
    X = np.zeros((tab.shape[0], 3))
    for idx, (d, i, j0, j1) in enumerate(tab):
        t0, t1 = tangential_axes(int(d))
        X[idx, d] = zc[i]
        X[idx, t0] = zo[j0]
        X[idx, t1] = zo[j1]
    return X
