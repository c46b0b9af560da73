"""Pins for the extended-precision reference ``oracle/extended.py`` (no GPU).

Every GPU tolerance is measured against this reference, so it is pinned to
things other than itself:

* its quadrature and interpolation nodes: Legendre residuals, exactness of
  the weights on monomials, closed forms of the nodes;
* exact arithmetic: the whole RT0 4^3 system (rationals) and RT0 / RT1 box
  elements (Q(sqrt 3), reference integrals by exact polynomial integration)
  with interior, essential and natural faces: it agrees to ~1e-17, where an
  FP64 computation is ~1e-14 off;
* the FP64 oracle on jittered, rotated elements for k = 0..3: agreement
  within a small multiple of kappa 2^-53 (kappa of the equilibrated kept
  block), which pins the geometry (J, not J^T) and the conventions where no
  exact value exists;
* the backward error of its solves is at long-double level;
* planted mistakes (a flipped face sign, J^T for J, a dropped div-div term,
  a natural face taken as essential) each fail one of these pins.
"""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import element, extended as oext, hybrid as ohyb, topology as otopo
from tests import exact_rt

LD = np.longdouble
U64 = 2.0 ** -53


def _rel(ref, got):
    ref = np.asarray(ref, dtype=LD)
    got = np.asarray(got, dtype=LD)
    return float(np.abs(ref - got).max() / np.abs(ref).max())


# ------------------------------------------------------------------ nodes
@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_gauss_legendre_nodes_weights(q):
    x, w = oext.gauss_legendre_ld(q)
    p, _ = oext._legendre_ld(q, 2 * x - 1)
    assert float(np.abs(p).max()) <= 1e-17
    for deg in range(2 * q):
        assert abs(float((w * x ** deg).sum() - LD(1) / LD(deg + 1))) <= 1e-18   # ~10 ulp of long double
    assert float(w.min()) > 0


def test_node_closed_forms():
    s = np.sqrt
    half = LD(1) / 2
    glo = {1: [half], 2: [half - s(LD(1) / 3) / 2, half + s(LD(1) / 3) / 2],
           3: [half - s(LD(3) / 5) / 2, half, half + s(LD(3) / 5) / 2]}
    for q, ref in glo.items():
        assert float(np.abs(oext.gauss_legendre_ld(q)[0] - np.array(ref, dtype=LD)).max()) <= 2e-19
    gll = {2: [0, 1], 3: [0, half, 1],
           4: [0, half - s(LD(1) / 5) / 2, half + s(LD(1) / 5) / 2, 1],
           5: [0, half - s(LD(3) / 7) / 2, half, half + s(LD(3) / 7) / 2, 1]}
    for npts, ref in gll.items():
        assert float(np.abs(oext.gauss_lobatto_ld(npts) - np.array(ref, dtype=LD)).max()) <= 2e-19


# ------------------------------------------------------------- exact pins
def _pin_c1():
    """Max relative error of the long-double H and r of C1 against the exact
    rational system."""
    prob = synth.config_c1()
    Hx, rx, m = exact_rt.c1_exact(prob)
    topo = otopo.build_topology(prob.mesh.e2v)
    Hld, rld, _ = oext.hybridize_ld(0, prob.mesh.xyz, prob.mesh.e2v, prob.alpha, prob.beta, prob.f, topo,
                                    np.arange(prob.mesh.ne))
    if set(Hld) != set(Hx):
        return np.inf
    sH = max(abs(v) for v in Hx.values())
    eH = max(abs(Fraction(*Hld[key].as_integer_ratio()) - v) for key, v in Hx.items()) / sH
    sr = max(abs(v) for v in rx)
    er = max(abs(Fraction(*rld[mu].as_integer_ratio()) - rx[mu]) for mu in range(m)) / sr
    return float(max(eH, er))


def test_c1_long_double_exact():
    """The whole C1 system: long double within 1e-17 of the exact rationals
    (the FP64 oracle is ~1e-15 off, test_oracle_theorem)."""
    assert _pin_c1() <= 1e-17


BOX_H = (Fraction(1, 4), Fraction(1, 8), Fraction(3, 16))
BOX_O = (Fraction(1, 2), Fraction(0), Fraction(1, 4))
BOX_ALPHA, BOX_BETA = Fraction(3, 2), Fraction(5, 4)
BOX_F = (Fraction(1, 2), Fraction(-3, 4), Fraction(5, 8))
# (essential-face mask, natural-face mask): interior element, a corner with
# three essential faces, essential and natural faces together
BOX_MASKS = [(0, 0), (0b010101, 0), (0b000001, 0b100100)]


def _box_xyz():
    xyz = np.zeros((8, 3))
    for v in range(8):
        bits = [(v >> a) & 1 for a in range(3)]
        xyz[v] = [float(BOX_O[a] + bits[a] * BOX_H[a]) for a in range(3)]
    return xyz


def _pin_box(k, code, nat):
    """Max relative error of the long-double M_T, f_T, H_T, r_T and u_T of a
    box element against exact arithmetic."""
    M, fT = exact_rt.box_element_exact(k, BOX_H, BOX_ALPHA, BOX_BETA, BOX_F)
    n_mult = len(exact_rt.split(k, code, nat)[2])
    lam = [Fraction(j + 1, 8) * (-1) ** j for j in range(n_mult)]    # exact in binary
    H, r, u = exact_rt.schur_exact(k, M, fT, code, nat, lam)
    Ml, fl = oext.element_matrix_ld(k, _box_xyz(), float(BOX_ALPHA), float(BOX_BETA), [float(x) for x in BOX_F])
    Hl = oext.local_schur_ld(k, Ml, code, nat)
    rl = oext.local_rhs_ld(k, Ml, fl, code, nat)
    ul = oext.local_recover_ld(k, Ml, fl, code, np.array([float(x) for x in lam]), nat)
    if Hl.shape != (n_mult, n_mult):
        return np.inf
    kap = np.linalg.cond(np.array(exact_rt.to_ld(M), dtype=np.float64))
    err = max(_rel(exact_rt.to_ld(M), Ml), _rel(exact_rt.to_ld(fT), fl), _rel(exact_rt.to_ld(H), Hl),
              _rel(exact_rt.to_ld(r), rl), _rel(exact_rt.to_ld(u), ul))
    return err / (kap * 2.0 ** -64)


@pytest.mark.parametrize("k", [0, 1])
@pytest.mark.parametrize("code,nat", BOX_MASKS)
def test_box_element_long_double_exact(k, code, nat):
    """RT0 / RT1 box element (sides 1/4, 1/8, 3/16): long double within
    16 kappa 2^-64 of the exact Q(sqrt 3) values (M_T, f_T to a few ulp),
    with interior, essential and natural faces; kappa(M_T) is 1e3 / 1e4 here,
    so an FP64 computation sits 2048 times further off."""
    assert _pin_box(k, code, nat) <= 16.0


# ------------------------------------------------- against the FP64 oracle
def _jittered(k, seed):
    rng = np.random.default_rng(seed)
    mesh = synth.structured_hex(2, jitter=0.25, rng=rng)
    mesh, _ = synth.rotate_connectivity(mesh, rng)
    ne = mesh.ne
    return mesh, synth.lognormal(rng, ne), synth.lognormal(rng, ne, 0.5), synth.element_loads(rng, ne)


def _pin_fp64(k, seed, natural_faces=False):
    """Largest ratio over the elements of |LD - FP64 oracle| / (kappa_s 2^-53)
    for H_T, r_T and u_T (relative to each block's largest entry)."""
    mesh, a, b, f = _jittered(k, seed)
    topo = otopo.build_topology(mesh.e2v)
    ess = None
    if natural_faces:
        ess = np.ones((mesh.ne, 6), np.uint8)
        ess[:, 0] = 0                     # every boundary face at xi_0 = 0 natural
        ess[:, 5] = 0
    M, fT = element.element_system(k, mesh.xyz[mesh.e2v], a, b, f)
    codes, nats = ohyb.face_codes(topo, np.arange(mesh.ne), ess)
    rng = np.random.default_rng(seed + 1)
    worst = 0.0
    for e in range(mesh.ne):
        code, nat = int(codes[e]), int(nats[e])
        kap = oext.kappa_scaled(k, mesh.xyz, mesh.e2v, a, b, topo, [e], ess)
        HT, rT = ohyb.local_schur(k, M[e:e + 1], fT[e:e + 1], code, None, nat)
        lam = rng.standard_normal(HT.shape[1])
        uT = ohyb.local_recover(k, M[e:e + 1], fT[e:e + 1], code, lam[None], None, nat)[0]
        Ml, fl = oext.element_matrix_ld(k, mesh.xyz[mesh.e2v[e]], a[e], b[e], f[e])
        Hl = oext.local_schur_ld(k, Ml, code, nat)
        rl = oext.local_rhs_ld(k, Ml, fl, code, nat)
        ul = oext.local_recover_ld(k, Ml, fl, code, lam, nat)
        if Hl.shape != HT[0].shape:
            return np.inf
        err = max(_rel(Hl, HT[0]), _rel(rl, rT[0]), _rel(ul, uT))
        worst = max(worst, err / (kap * U64))
    return worst


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_long_double_agrees_with_fp64_oracle(k):
    """Jittered (0.25 h), rotated 2^3 meshes, lognormal coefficients: the FP64
    oracle is within 16 kappa_s 2^-53 of the long-double reference for every
    element's H_T, r_T and u_T (about 1 kappa_s 2^-53 is measured)."""
    assert _pin_fp64(k, 60 + k) <= 16.0


@pytest.mark.parametrize("k", [1, 2])
def test_long_double_agrees_with_fp64_oracle_natural_faces(k):
    assert _pin_fp64(k, 70 + k, natural_faces=True) <= 16.0


def test_long_double_backward_error():
    """X = M_rr^{-1} C^T by the long-double Cholesky on an RT3 element:
    ||C^T - M X||_inf <= 4 n 2^-64 ||M||_inf ||X||_inf, i.e. the solve is at
    long-double precision (an FP64 solve gives ~2^-53)."""
    mesh, a, b, f = _jittered(3, 80)
    M = oext.element_matrix_ld(3, mesh.xyz[mesh.e2v[5]], a[5], b[5])
    n = M.shape[0]
    L = oext.cholesky_ld(M)
    ni = oext._split_ld(3, 0)[0].size - 96
    B = np.zeros((n, 96), dtype=LD)
    B[ni + np.arange(96), np.arange(96)] = oext._signs_ld(3)
    X = oext.backward_ld(L, oext.forward_ld(L, B))
    res = np.abs(B - M @ X).sum(axis=1).max()
    bound = 4 * n * LD(2.0) ** -64 * np.abs(M).sum(axis=1).max() * np.abs(X).sum(axis=1).max()
    assert res <= bound


def test_kappa_scaled_is_a_condition_number():
    """kappa_s of an element equals cond_2 of its equilibrated kept block
    (diagonal scaling leaves a diagonal matrix's kappa_s at 1)."""
    mesh, a, b, f = _jittered(1, 81)
    topo = otopo.build_topology(mesh.e2v)
    k_all = oext.kappa_scaled(1, mesh.xyz, mesh.e2v, a, b, topo, np.arange(mesh.ne))
    k_one = [oext.kappa_scaled(1, mesh.xyz, mesh.e2v, a, b, topo, [e]) for e in range(mesh.ne)]
    assert k_all == max(k_one) and min(k_one) > 1.0


# ------------------------------------------------------- planted mistakes
def test_planted_flipped_face_sign(monkeypatch):
    orig = oext._signs_ld

    def flipped(k):
        s = orig(k).copy()
        K2 = (k + 1) ** 2
        s[3 * K2:4 * K2] *= -1            # face 3 with the wrong outward sign
        return s
    monkeypatch.setattr(oext, "_signs_ld", flipped)
    assert _pin_c1() > 1e-3


def test_planted_transposed_jacobian(monkeypatch):
    orig = oext._jacobian_ld

    def transposed(xe, X):
        J, det = orig(xe, X)
        return np.transpose(J, (0, 2, 1)).copy(), det
    monkeypatch.setattr(oext, "_jacobian_ld", transposed)
    assert _pin_fp64(2, 62) > 1e3


def test_planted_dropped_divdiv(monkeypatch):
    monkeypatch.setattr(oext, "_combine_ld", lambda al, mass, be, divdiv: LD(al) * mass)
    assert _pin_c1() > 1e-3


def test_planted_natural_face_taken_as_essential(monkeypatch):
    orig = oext._split_ld
    monkeypatch.setattr(oext, "_split_ld", lambda k, code, natural=0: orig(k, code | natural, 0))
    assert _pin_box(1, 0b000001, 0b100100) > 1e6
