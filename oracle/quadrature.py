"""Tensor Gauss-Legendre rules on [0,1]^3 (test infrastructure).

The paper does not state its quadrature; this oracle uses q = k+2 points per
direction for RT_k, which integrates the affine-element mass and div-div
integrands exactly.  Points are ordered with axis 0 fastest.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_1d(q: int):
    x, w = npleg.leggauss(q)
    return (x + 1.0) / 2.0, w / 2.0


def hex_rule(q: int):
    """Returns points X (q^3, 3) and weights W (q^3,)."""
    x, w = gauss_1d(q)
    X = np.array([[x[a], x[b], x[c]] for c in range(q) for b in range(q) for a in range(q)])
    W = np.array([w[a] * w[b] * w[c] for c in range(q) for b in range(q) for a in range(q)])
    return X, W
