"""Trilinear hexahedral geometry (test infrastructure).

Element vertex v = a + 2b + 4c sits at reference corner (a, b, c); the map is
x(xi) = sum_v X_v N_v(xi) with N_v the product of xi_d or 1 - xi_d per axis,
and J = dx/dxi (J[r, c] = d x_r / d xi_c).
"""
from __future__ import annotations

import numpy as np


def shape_functions(X: np.ndarray):
    """Trilinear shape functions N (P, 8) and gradients dN (P, 8, 3) at X (P, 3)."""
    X = np.asarray(X, dtype=np.float64)
    P = X.shape[0]
    N = np.ones((P, 8))
    dN = np.ones((P, 8, 3))
    for v in range(8):
        bits = [(v >> a) & 1 for a in range(3)]
        for a in range(3):
            fa = X[:, a] if bits[a] else 1.0 - X[:, a]
            ga = 1.0 if bits[a] else -1.0
            N[:, v] *= fa
            for c in range(3):
                dN[:, v, c] *= ga if c == a else fa
    return N, dN


def map_points(xyz_e: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Physical points (..., P, 3) of reference points X for element
    coordinates xyz_e (..., 8, 3)."""
    N, _ = shape_functions(X)
    return np.einsum("pv,...vr->...pr", N, xyz_e)


def jacobians(xyz_e: np.ndarray, X: np.ndarray) -> np.ndarray:
    """J (..., P, 3, 3) with J[..., p, r, c] = d x_r / d xi_c."""
    _, dN = shape_functions(X)
    return np.einsum("pvc,...vr->...prc", dN, xyz_e)
