"""Pins for the oracle's hybridization against Theorem 2.1 and the structure
of P, C and H (no GPU)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import conforming, element, hybrid, rt_basis, topology


def _problem(k, N, jitter, seed, rotate=False):
    rng = np.random.default_rng(seed)
    mesh = synth.structured_hex(N, jitter=jitter, rng=rng)
    if rotate:
        mesh, _ = synth.rotate_connectivity(mesh, rng)
    ne = mesh.ne
    return mesh, synth.lognormal(rng, ne), synth.lognormal(rng, ne), synth.element_loads(rng, ne)


CASES = [(0, 2, 0.0), (0, 4, 0.2), (1, 2, 0.0), (1, 3, 0.2), (2, 2, 0.2), (3, 2, 0.0), (3, 2, 0.2)]


@pytest.mark.parametrize("k,N,jit", CASES)
@pytest.mark.parametrize("rotate", [False, True])
def test_theorem_2_1_hybridized_equals_conforming(k, N, jit, rotate):
    """x_hat from the multiplier system equals P x of the assembled system."""
    mesh, a, b, f = _problem(k, N, jit, 100 + k, rotate)
    hyb = hybrid.hybridize(k, mesh.xyz, mesh.e2v, a, b, f)
    lam = hybrid.solve_reduced(hyb.H, hyb.r)
    u = hybrid.recover(hyb, mesh.xyz, mesh.e2v, a, b, f, lam)
    uc = conforming.conforming_solve(k, mesh.xyz, mesh.e2v, a, b, f)
    assert np.abs(u - uc).max() <= 1e-10 * np.abs(uc).max()


@pytest.mark.parametrize("k,N,jit", CASES[:5])
def test_P_C_structure(k, N, jit):
    """C P = 0 exactly, P full column rank, C full row rank, n + m = n_hat."""
    mesh, *_ = _problem(k, N, jit, 7, rotate=True)
    topo = topology.build_topology(mesh.e2v)
    P = conforming.build_P(k, topo)
    C = conforming.build_C(k, topo)
    assert (C @ P).count_nonzero() == 0 or np.abs((C @ P).toarray()).max() == 0.0
    n_hat = P.shape[0]
    m, n = C.shape[0], P.shape[1]
    assert n + m == n_hat
    assert np.linalg.matrix_rank(P.toarray()) == n
    assert np.linalg.matrix_rank(C.toarray()) == m


@pytest.mark.parametrize("k,N,jit", CASES)
def test_H_symmetric_positive_definite(k, N, jit):
    mesh, a, b, f = _problem(k, N, jit, 200 + k)
    hyb = hybrid.hybridize(k, mesh.xyz, mesh.e2v, a, b, f)
    H = hyb.H.toarray()
    assert np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()
    assert np.linalg.eigvalsh((H + H.T) / 2).min() > 0
    np.linalg.cholesky((H + H.T) / 2)


@pytest.mark.parametrize("k,N,jit", [(0, 3, 0.2), (1, 2, 0.2), (2, 2, 0.2)])
def test_local_equilibrium_and_constraint(k, N, jit):
    """M_T x_T + C_T^T lam_T = f_T on the kept dofs, and C x_hat = 0."""
    mesh, a, b, f = _problem(k, N, jit, 300 + k, rotate=True)
    hyb = hybrid.hybridize(k, mesh.xyz, mesh.e2v, a, b, f)
    lam = hybrid.solve_reduced(hyb.H, hyb.r)
    u = hybrid.recover(hyb, mesh.xyz, mesh.e2v, a, b, f, lam)
    M, fT = element.element_system(k, mesh.xyz[mesh.e2v], a, b, f)
    ni = rt_basis.n_interior(k)
    for e in range(mesh.ne):
        lam_full = np.where(hyb.mult_id[e] >= 0, lam[np.maximum(hyb.mult_id[e], 0)], 0.0)
        res = hybrid.equilibrium_residual(k, hyb.topo, M[e], fT[e], u[e], lam_full)
        kept = np.concatenate([np.arange(ni), ni + np.nonzero(hyb.mult_id[e] >= 0)[0]])
        assert np.abs(res[kept]).max() <= 1e-11 * (np.abs(M[e]).max() * np.abs(u[e]).max() + 1)
    topo = hyb.topo
    C = conforming.build_C(k, topo)
    keeps, offs = conforming.kept_layout(k, topo)
    xhat = np.concatenate([u[e, keeps[e]] for e in range(mesh.ne)])
    assert np.abs(C @ xhat).max() <= 1e-11 * np.abs(xhat).max()


def test_c1_exact_rational():
    """The whole RT0 4^3 reduced system in exact rational arithmetic
    (``tests/exact_rt.c1_exact``: closed-form M_T and f_T of the cube of side
    h = 1/4, alpha = beta = 1, the structured-grid face numbering written out
    independently, exact elimination of boundary faces and exact local
    inverses) against the FP64 oracle."""
    from tests.exact_rt import c1_exact
    prob = synth.config_c1()
    Hx, rx, m = c1_exact(prob)
    hyb = hybrid.hybridize(0, prob.mesh.xyz, prob.mesh.e2v, prob.alpha, prob.beta, prob.f)
    H = hyb.H.toarray()
    assert hyb.H.nnz == len(Hx) == 1200 and m == 144
    scale = max(abs(float(v)) for v in Hx.values())
    for (i, j), v in Hx.items():
        assert abs(H[i, j] - float(v)) <= 1e-13 * scale  # cond(M_T) ~ 6e2
    rs = max(abs(float(v)) for v in rx)
    assert np.abs(hyb.r - np.array([float(v) for v in rx])).max() <= 1e-13 * rs


def test_pcg_matches_direct_solve():
    """A Jacobi-preconditioned CG on H (scipy) reaches the direct solution."""
    mesh, a, b, f = _problem(1, 3, 0.2, 9)
    hyb = hybrid.hybridize(1, mesh.xyz, mesh.e2v, a, b, f)
    lam = hybrid.solve_reduced(hyb.H, hyb.r)
    Dinv = 1.0 / hyb.H.diagonal()
    lam2, info = spla.cg(hyb.H, hyb.r, rtol=1e-13, M=spla.LinearOperator(hyb.H.shape, lambda x: Dinv * x))
    assert info == 0
    assert np.abs(lam2 - lam).max() <= 1e-9 * np.abs(lam).max()
