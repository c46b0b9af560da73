"""Exact references for the oracle pins (test helpers, no floating point in
the arithmetic).

* ``c1_exact()``: the whole RT0 4^3 reduced system of the C1 workload in
  rational arithmetic, from the closed-form RT0 element matrix of a cube of
  side h (alpha = beta = 1) and a face numbering written out for the
  structured grid.
* ``box_element_exact(k, ...)``: M_T and f_T of RT_0 / RT_1 on an axis-aligned
  box in exact arithmetic over Q(sqrt 3): the 1D Lagrange polynomials on the
  closed (Gauss-Lobatto) and open (Gauss-Legendre) nodes are multiplied and
  integrated monomial by monomial (no quadrature), so the reference does not
  depend on the quadrature rule.  For k <= 1 the nodes are 0, 1/2, 1 and
  1/2 +- sqrt(3)/6, so every entry lies in Q(sqrt 3).
* ``schur_exact``: H_T = C_T M_rr^{-1} C_T^T, r_T and u_T by exact Gauss-Jordan
  elimination, for given essential / natural face masks.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

LD = np.longdouble


class Q3:
    """a + b sqrt(3), a and b rational."""
    __slots__ = ("a", "b")

    def __init__(self, a=0, b=0):
        self.a = a if isinstance(a, Fraction) else Fraction(a)
        self.b = b if isinstance(b, Fraction) else Fraction(b)

    @staticmethod
    def of(x):
        return x if isinstance(x, Q3) else Q3(x)

    def __add__(self, o):
        o = Q3.of(o)
        return Q3(self.a + o.a, self.b + o.b)

    __radd__ = __add__

    def __sub__(self, o):
        o = Q3.of(o)
        return Q3(self.a - o.a, self.b - o.b)

    def __rsub__(self, o):
        return Q3.of(o) - self

    def __neg__(self):
        return Q3(-self.a, -self.b)

    def __mul__(self, o):
        o = Q3.of(o)
        return Q3(self.a * o.a + 3 * self.b * o.b, self.a * o.b + self.b * o.a)

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = Q3.of(o)
        den = o.a * o.a - 3 * o.b * o.b
        num = self * Q3(o.a, -o.b)
        return Q3(num.a / den, num.b / den)

    def __rtruediv__(self, o):
        return Q3.of(o) / self

    def is_zero(self):
        return self.a == 0 and self.b == 0

    def ld(self):
        """Value in long double (each part converted from its exact ratio)."""
        def fr(x):
            return LD(str(x.numerator)) / LD(str(x.denominator))
        return fr(self.a) + fr(self.b) * np.sqrt(LD(3))


# ------------------------------------------------------------ polynomials
def _pmul(p, q):
    out = [Q3() for _ in range(len(p) + len(q) - 1)]
    for i, x in enumerate(p):
        for j, y in enumerate(q):
            out[i + j] = out[i + j] + x * y
    return out


def _pderiv(p):
    return [p[i] * i for i in range(1, len(p))] or [Q3()]


def _pint01(p):
    """Integral over [0, 1]: sum_i c_i / (i + 1)."""
    s = Q3()
    for i, c in enumerate(p):
        s = s + c * Fraction(1, i + 1)
    return s


def _lagrange(z):
    """Coefficient lists (ascending powers) of the Lagrange polynomials on z."""
    out = []
    for i in range(len(z)):
        p = [Q3(1)]
        for j in range(len(z)):
            if j != i:
                p = _pmul(p, [Q3.of(-z[j]) / (z[i] - z[j]), Q3(1) / (z[i] - z[j])])
        out.append(p)
    return out


def nodes(k: int):
    """Closed (k+2 Gauss-Lobatto) and open (k+1 Gauss-Legendre) nodes on [0,1]."""
    if k == 0:
        return [Q3(0), Q3(1)], [Q3(Fraction(1, 2))]
    if k == 1:
        return ([Q3(0), Q3(Fraction(1, 2)), Q3(1)],
                [Q3(Fraction(1, 2), Fraction(-1, 6)), Q3(Fraction(1, 2), Fraction(1, 6))])
    raise ValueError("exact nodes are in Q(sqrt 3) only for k <= 1")


def dofs(k: int):
    """(d, i, j0, j1) in local order: interior dofs (d, j1, j0, i innermost),
    then face f = 2d + s dofs with i = s (k+1)."""
    rows = [(d, i, j0, j1) for d in range(3) for j1 in range(k + 1) for j0 in range(k + 1)
            for i in range(1, k + 1)]
    rows += [(f // 2, (f % 2) * (k + 1), j0, j1) for f in range(6) for j1 in range(k + 1) for j0 in range(k + 1)]
    return rows


def box_element_exact(k: int, h, alpha, beta, f):
    """M_T (n x n lists of Q3) and f_T for the box [o, o + h] (sides h: three
    Fractions), x = o + h xi, so J = diag(h), det J = h0 h1 h2, and under the
    Piola map u = J u_hat / det J:
      M_T[i,j] = alpha sum_d [d_i = d_j = d] h_d^2 / V int phi_i phi_j
                 + beta / V int div phi_i div phi_j,
      f_T[i] = f_{d_i} h_{d_i} int phi_i     (reference integrals over [0,1]^3)."""
    zc, zo = nodes(k)
    Lc, Lo = _lagrange(zc), _lagrange(zo)
    dLc = [_pderiv(p) for p in Lc]
    V = h[0] * h[1] * h[2]
    al, be = Fraction(alpha), Fraction(beta)
    D = dofs(k)

    def axis_factor(dof, axis, deriv):
        d, i, j0, j1 = dof
        if axis == d:
            return dLc[i] if deriv else Lc[i]
        t0, t1 = [a for a in range(3) if a != d]
        return Lo[j0] if axis == t0 else Lo[j1]

    cache = {}

    def int3(di, dj, deriv):
        key = (di, dj, deriv)
        if key not in cache:
            v = Q3(1)
            for ax in range(3):
                v = v * _pint01(_pmul(axis_factor(di, ax, deriv), axis_factor(dj, ax, deriv)))
            cache[key] = v
        return cache[key]

    n = len(D)
    M = [[Q3() for _ in range(n)] for _ in range(n)]
    for a in range(n):
        for b in range(n):
            v = int3(D[a], D[b], True) * (be / V)
            if D[a][0] == D[b][0]:
                d = D[a][0]
                v = v + int3(D[a], D[b], False) * (al * h[d] * h[d] / V)
            M[a][b] = v
    fT = []
    for a in range(n):
        d = D[a][0]
        v = Q3(1)
        for ax in range(3):
            v = v * _pint01(axis_factor(D[a], ax, False))
        fT.append(v * (Fraction(f[d]) * h[d]))
    return M, fT


def split(k: int, code: int, natural: int = 0):
    """Kept dofs, essential dofs, and the kept positions with a multiplier."""
    ni, K2 = 3 * k * (k + 1) ** 2, (k + 1) ** 2
    keep, ess, mult = list(range(ni)), [], []
    for fa in range(6):
        blk = [ni + fa * K2 + j for j in range(K2)]
        if (code >> fa) & 1:
            ess += blk
        else:
            if not (natural >> fa) & 1:
                mult += [len(keep) + j for j in range(K2)]
            keep += blk
    return keep, ess, mult


def solve_exact(A, B):
    """A^{-1} B by Gauss-Jordan (A: list of rows, B: list of rows)."""
    n = len(A)
    M = [list(A[i]) + list(B[i]) for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if not Q3.of(M[r][c]).is_zero())
        M[c], M[p] = M[p], M[c]
        inv = Q3(1) / M[c][c]
        M[c] = [x * inv for x in M[c]]
        for r in range(n):
            if r != c and not Q3.of(M[r][c]).is_zero():
                fac = M[r][c]
                M[r] = [x - fac * y for x, y in zip(M[r], M[c])]
    return [row[n:] for row in M]


def schur_exact(k: int, M, fT, code: int, natural: int = 0, lam=None):
    """H_T, r_T (multiplier dofs in local order) and, with lam, u_T on the
    kept dofs (0 on essential dofs), all exact.  C_T[a, dof] = eps_f = 2s - 1."""
    keep, ess, mult = split(k, code, natural)
    ni, K2 = 3 * k * (k + 1) ** 2, (k + 1) ** 2
    eps = [2 * (((keep[p] - ni) // K2) % 2) - 1 for p in mult]
    Mrr = [[M[i][j] for j in keep] for i in keep]
    nr, mT = len(keep), len(mult)
    rhs = []
    for p in range(nr):
        row = [Q3(eps[a]) if mult[a] == p else Q3() for a in range(mT)]
        row.append(fT[keep[p]])
        if lam is not None:
            v = fT[keep[p]]
            if p in mult:
                a = mult.index(p)
                v = v - Q3(Fraction(lam[a])) * eps[a]
            row.append(v)
        rhs.append(row)
    X = solve_exact(Mrr, rhs)
    H = [[X[mult[a]][b] * eps[a] for b in range(mT)] for a in range(mT)]
    r = [X[mult[a]][mT] * eps[a] for a in range(mT)]
    u = None
    if lam is not None:
        u = [Q3() for _ in range(len(M))]
        for p, i in enumerate(keep):
            u[i] = X[p][mT + 1]
    return H, r, u


def to_ld(x):
    """Nested lists of Q3 -> long-double array."""
    if isinstance(x, Q3):
        return x.ld()
    return np.array([to_ld(v) for v in x], dtype=LD)


# ------------------------------------------------------------------- C1
def c1_exact(prob):
    """The RT0 4^3 reduced system (alpha = beta = 1, h = 1/4) exactly: returns
    (H as {(mu, nu): Fraction}, r as a list of Fractions, m).

    Closed-form M_T of the cube of side h: (1/h) blockdiag_3([[1/3, 1/6],
    [1/6, 1/3]]) + (1/h^3) d d^T with d = (-1, 1, -1, 1, -1, 1); f_T = (h/2)
    (f_x, f_x, f_y, f_y, f_z, f_z); the face between e and its +d neighbour
    is owned by e as its local face 2d+1; boundary faces are eliminated."""
    N, h = 4, Fraction(1, 4)
    blk = [[Fraction(1, 3), Fraction(1, 6)], [Fraction(1, 6), Fraction(1, 3)]]
    d = [-1, 1, -1, 1, -1, 1]
    M = [[(blk[i % 2][j % 2] / h if i // 2 == j // 2 else Fraction(0)) + d[i] * d[j] / h ** 3
          for j in range(6)] for i in range(6)]
    strides = [1, N, N * N]
    owned = []
    for e in range(N ** 3):
        ijk = [e % N, (e // N) % N, e // (N * N)]
        for dd in range(3):
            if ijk[dd] + 1 < N:
                owned.append((e, 2 * dd + 1))
    owned.sort()
    fid = {}
    for i, (e, lf) in enumerate(owned):
        dd = lf // 2
        fid[(e, lf)] = i
        fid[(e + strides[dd], lf - 1)] = i
    m = len(owned)
    Hx = {}
    rx = [Fraction(0)] * m
    for e in range(N ** 3):
        fe = [Fraction(float(x)) for x in prob.f[e]]
        fhat = [h / 2 * fe[i // 2] for i in range(6)]
        kept = [lf for lf in range(6) if (e, lf) in fid]
        Mrr = [[Q3(M[i][j]) for j in kept] for i in kept]
        rhs = [[Q3(Fraction(int(i == j)) * d[i]) for j in kept] + [Q3(fhat[i])] for i in kept]
        X = solve_exact(Mrr, rhs)
        for a, la in enumerate(kept):
            for b, lb in enumerate(kept):
                key = (fid[(e, la)], fid[(e, lb)])
                Hx[key] = Hx.get(key, Fraction(0)) + d[la] * X[a][b].a
            rx[fid[(e, la)]] += d[la] * X[a][len(kept)].a
    return Hx, rx, m
