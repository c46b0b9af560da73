"""Pins for the oracle's Jacobi-PCG (no GPU): scipy's independent CG iterates,
the finite-termination property of CG, the energy-norm minimisation, and the
direct solution of a hybridized system."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import hybrid
from oracle.pcg import jacobi_pcg


def _hyb(k, N, seed):
    rng = np.random.default_rng(seed)
    mesh = synth.structured_hex(N, jitter=0.2, rng=rng)
    ne = mesh.ne
    a, b, f = synth.lognormal(rng, ne), synth.lognormal(rng, ne), synth.element_loads(rng, ne)
    return hybrid.hybridize(k, mesh.xyz, mesh.e2v, a, b, f)


def test_iterates_match_scipy_cg():
    """The first iterates equal those of scipy's preconditioned CG (a separate
    implementation) with the same diagonal preconditioner and lam_0 = 0."""
    h = _hyb(1, 3, 11)
    H, r = h.H, h.r
    dinv = 1.0 / H.diagonal()
    xs = []
    spla.cg(H, r, x0=np.zeros_like(r), rtol=1e-30, maxiter=10,
            M=spla.LinearOperator(H.shape, lambda x: dinv * x), callback=lambda xk: xs.append(xk.copy()))
    for j, xk in enumerate(xs, start=1):
        lam, it, _, _ = jacobi_pcg(H, r, rtol=1e-30, maxit=j)
        assert it == j
        assert np.abs(lam - xk).max() <= 1e-12 * np.abs(xk).max(), j


def test_diagonal_matrix_one_iteration():
    """With H diagonal the preconditioned operator is the identity: one step."""
    rng = np.random.default_rng(3)
    d = rng.uniform(0.1, 10.0, 50)
    b = rng.standard_normal(50)
    lam, it, conv, _ = jacobi_pcg(sp.diags(d).tocsr(), b, rtol=1e-14)
    assert conv and it == 1
    assert np.abs(lam - b / d).max() <= 1e-15 * np.abs(b / d).max()


def test_three_distinct_eigenvalues_three_iterations():
    """When the Jacobi-preconditioned operator has 3 distinct eigenvalues, CG
    ends in 3 steps (exact arithmetic; here to rounding).  H = S B S with
    B = Q diag(ev) Q^T, Q a normalised Hadamard matrix (so diag(B) is the
    constant mean(ev)) and S a positive diagonal: D^{-1} H is similar to
    B / mean(ev)."""
    import scipy.linalg
    rng = np.random.default_rng(4)
    m = 32
    Q = scipy.linalg.hadamard(m) / np.sqrt(m)
    ev = rng.permutation(np.repeat([1.0, 2.5, 7.0], [11, 11, 10]))
    B = Q @ np.diag(ev) @ Q.T
    assert np.allclose(np.diag(B), ev.mean())
    s = rng.uniform(0.5, 3.0, m)
    H = sp.csr_matrix(s[:, None] * B * s[None, :])
    b = rng.standard_normal(m)
    lam, it, conv, hist = jacobi_pcg(H, b, rtol=1e-11, maxit=50)
    assert conv and it == 3
    assert np.abs(H @ lam - b).max() <= 1e-11 * np.abs(b).max()
    # a steepest-descent slip (beta dropped) or a missing preconditioner
    # would not terminate in 3 steps on this matrix
    assert hist[2] > 1e-6 * hist[0]


def test_hybridized_system_energy_norm_and_direct_solution():
    """On a hybridized H: the energy-norm error decreases monotonically (CG
    minimises it over the Krylov space) and the iterate reaches the direct
    solution; with check_every = 8 the iteration count is the next multiple
    of 8 of the count with per-iteration checks."""
    h = _hyb(2, 3, 12)
    H, r = h.H, h.r
    ref = hybrid.solve_reduced(H, r)
    errs = []
    for j in range(0, 30, 3):
        lam, *_ = jacobi_pcg(H, r, rtol=1e-30, maxit=j)
        e = lam - ref
        errs.append(float(e @ (H @ e)))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    lam, it1, conv, hist = jacobi_pcg(H, r, rtol=1e-12, maxit=5000)
    assert conv and hist[-1] <= 1e-12 * hist[0]
    assert np.abs(lam - ref).max() <= 1e-9 * np.abs(ref).max()
    _, it8, conv8, _ = jacobi_pcg(H, r, rtol=1e-12, maxit=5000, check_every=8)
    assert conv8 and it8 == -(-it1 // 8) * 8


def test_zero_and_empty_right_hand_sides():
    h = _hyb(0, 2, 13)
    lam, it, conv, _ = jacobi_pcg(h.H, np.zeros(h.H.shape[0]))
    assert conv and it == 0 and not lam.any()
    lam, it, conv, _ = jacobi_pcg(sp.csr_matrix((0, 0)), np.zeros(0))
    assert conv and it == 0 and lam.size == 0
