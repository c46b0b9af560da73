"""Pins for the oracle's static condensation (no GPU): the element-by-element
assembly equals the Schur complement of the assembled conforming matrix (two
different routes), S is symmetric positive definite with the sparsity of H,
its solution recovers the conforming / hybridized solution (Theorem 2.1 and
Sec. 3.1), and element by element H_T = D S_hat_T^{-1} D (Sec. 3.1: H
assembles the inverses of the local Schur complements, S the complements)."""
import numpy as np
import pytest

import synth
from oracle import conforming, element, hybrid, static


def _problem(k, N, jitter, seed, rotate=False, with_g=False):
    rng = np.random.default_rng(seed)
    mesh = synth.structured_hex(N, jitter=jitter, rng=rng)
    if rotate:
        mesh, _ = synth.rotate_connectivity(mesh, rng)
    ne = mesh.ne
    a, b, f = synth.lognormal(rng, ne), synth.lognormal(rng, ne), synth.element_loads(rng, ne)
    g = rng.standard_normal((ne, 6 * (k + 1) ** 2)) if with_g else None
    return mesh, a, b, f, g


CASES = [(0, 3, 0.2, True, False), (1, 2, 0.0, False, False), (1, 3, 0.2, True, True), (2, 2, 0.2, True, True),
         (3, 2, 0.2, False, False)]


@pytest.mark.parametrize("k,N,jit,rot,wg", CASES)
def test_elementwise_equals_plain_definition(k, N, jit, rot, wg):
    mesh, a, b, f, g = _problem(k, N, jit, 400 + k, rot, wg)
    c = static.condense(k, mesh.xyz, mesh.e2v, a, b, f, g)
    Sp, rp = static.condense_plain(k, mesh.xyz, mesh.e2v, a, b, f, g)
    S = c.S.toarray()
    assert np.abs(S - Sp).max() <= 1e-11 * np.abs(Sp).max()
    assert np.abs(c.r - rp).max() <= 1e-11 * np.abs(rp).max()
    assert np.abs(S - S.T).max() <= 1e-13 * np.abs(S).max()
    assert np.linalg.eigvalsh(S).min() > 0


@pytest.mark.parametrize("k,N,jit,rot,wg", CASES)
def test_solution_equals_conforming_and_hybridized(k, N, jit, rot, wg):
    mesh, a, b, f, g = _problem(k, N, jit, 500 + k, rot, wg)
    c = static.condense(k, mesh.xyz, mesh.e2v, a, b, f, g)
    x = np.linalg.solve(c.S.toarray(), c.r)
    u = static.recover(c, mesh.xyz, mesh.e2v, a, b, f, x, g)
    uc = conforming.conforming_solve(k, mesh.xyz, mesh.e2v, a, b, f, g)
    hy = hybrid.hybridize(k, mesh.xyz, mesh.e2v, a, b, f, g)
    uh = hybrid.recover(hy, mesh.xyz, mesh.e2v, a, b, f, hybrid.solve_reduced(hy.H, hy.r), g)
    scale = np.abs(uc).max()
    assert np.abs(u - uc).max() <= 1e-10 * scale
    assert np.abs(u - uh).max() <= 1e-10 * scale
    # same sparsity as H
    assert np.array_equal(c.S.indptr, hy.H.indptr) and np.array_equal(c.S.indices, hy.H.indices)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_H_T_is_the_signed_inverse_of_S_hat_T(k):
    """On an interior element (all faces interior): H_T = D S_hat_T^{-1} D."""
    mesh, a, b, f, _ = _problem(k, 3, 0.2, 600 + k)
    e = 13                                   # the centre element of 3^3
    M, fT = element.element_system(k, mesh.xyz[mesh.e2v[[e]]], a[[e]], b[[e]], f[[e]])
    HT, _ = hybrid.local_schur(k, M, fT, 0)
    St, _ = static._local(k, M, fT, 0, None)
    D = np.diag(hybrid._face_signs(k))
    ref = D @ np.linalg.inv(St[0]) @ D
    # two solves of a matrix with cond ~ 1e4: agreement to kappa 2^-53
    assert np.abs(HT[0] - ref).max() <= 1e-10 * np.abs(ref).max()
