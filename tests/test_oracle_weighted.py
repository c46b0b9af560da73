"""Pins for the M_s-weighted constraint (Example 2.3, no GPU): M_s by
quadrature is diagonal with the closed form w_a w_b (Gauss-Legendre weights
of the face nodes), the same on all faces and invariant under the square's
symmetries; H' = M_s H M_s is SPD; the broken solution does not change."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import synth
from oracle import hybrid, topology, weighted


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_face_mass_closed_form(k):
    x, w = npleg.leggauss(k + 1)
    w = w / 2.0
    ref = np.diag(np.outer(w, w).reshape(-1))       # index a0 + (k+1) a1: w[a1] w[a0]
    for f in range(6):
        Ms = weighted.face_mass(k, f)
        assert np.abs(Ms - ref).max() <= 1e-14
    # invariant under the 8 symmetries of the face (frame maps)
    K = k
    dg = np.diag(ref)
    for pi in range(8):
        perm = [0] * len(dg)
        for a1 in range(k + 1):
            for a0 in range(k + 1):
                b0, b1 = topology.apply_symmetry(pi, a0, a1, K)
                perm[a0 + (k + 1) * a1] = b0 + (k + 1) * b1
        assert np.allclose(dg[perm], dg, rtol=0, atol=1e-15)


@pytest.mark.parametrize("k,N", [(0, 3), (1, 3), (2, 2)])
def test_weighted_system_same_solution(k, N):
    rng = np.random.default_rng(20 + k)
    mesh = synth.structured_hex(N, jitter=0.2, rng=rng)
    mesh, _ = synth.rotate_connectivity(mesh, rng)
    ne = mesh.ne
    a, b, f = synth.lognormal(rng, ne), synth.lognormal(rng, ne), synth.element_loads(rng, ne)
    Hw, rw, hy = weighted.hybridize_weighted(k, mesh.xyz, mesh.e2v, a, b, f)
    assert np.linalg.eigvalsh(Hw.toarray()).min() > 0
    lw = hybrid.solve_reduced(Hw, rw)
    l0 = hybrid.solve_reduced(hy.H, hy.r)
    ms = weighted.weights_vector(k, hy.r.size)
    assert np.abs(ms * lw - l0).max() <= 1e-10 * np.abs(l0).max()   # lambda = M_s^T lambda'
    u0 = hybrid.recover(hy, mesh.xyz, mesh.e2v, a, b, f, l0)
    uw = hybrid.recover(hy, mesh.xyz, mesh.e2v, a, b, f, ms * lw)
    assert np.abs(uw - u0).max() <= 1e-10 * np.abs(u0).max()
