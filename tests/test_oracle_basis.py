"""Pins for the oracle's basis, quadrature and local matrices against closed
forms (no GPU)."""
import numpy as np
import pytest

from oracle import element, quadrature, rt_basis


@pytest.mark.parametrize("k,n", [(0, 6), (1, 36), (2, 108), (3, 240)])
def test_dimensions(k, n):
    assert rt_basis.ndofs(k) == n
    assert rt_basis.dof_table(k).shape == (n, 4)
    assert rt_basis.n_interior(k) + 6 * rt_basis.n_face(k) == n


def test_closed_points_closed_form():
    s5, s37 = 1 / np.sqrt(5), np.sqrt(3 / 7)
    expect = {0: [0, 1], 1: [0, .5, 1], 2: [0, (1 - s5) / 2, (1 + s5) / 2, 1],
              3: [0, (1 - s37) / 2, .5, (1 + s37) / 2, 1]}
    for k, z in expect.items():
        np.testing.assert_allclose(rt_basis.closed_points(k), z, atol=1e-15)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_kronecker_at_nodes(k):
    """phi_i(node_j) . e_{d_j} = delta_ij: the dofs are nodal normal components."""
    X = rt_basis.dof_nodes(k)
    val, _ = rt_basis.rt_eval(k, X)
    d = rt_basis.dof_table(k)[:, 0]
    V = val[:, np.arange(X.shape[0]), d]          # V[i, j] = phi_i(x_j) . e_{d_j}
    np.testing.assert_allclose(V, np.eye(X.shape[0]), atol=1e-13)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_divergence_theorem(k):
    """int div phi_i = boundary flux: eps_f w_j0 w_j1 for face dofs (Gauss
    weights are the integrals of the open-point Lagrange polynomials), 0 for
    interior dofs."""
    X, W = quadrature.hex_rule(k + 1)
    _, div = rt_basis.rt_eval(k, X)
    integ = div @ W
    _, wo = quadrature.gauss_1d(k + 1)
    ni = rt_basis.n_interior(k)
    np.testing.assert_allclose(integ[:ni], 0.0, atol=1e-13)
    for f in range(6):
        eps = 2 * (f % 2) - 1
        for j1 in range(k + 1):
            for j0 in range(k + 1):
                i = rt_basis.face_dof_index(k, f, j0, j1)
                assert abs(integ[i] - eps * wo[j0] * wo[j1]) < 1e-13


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_quadrature_exact_monomials(q):
    X, W = quadrature.hex_rule(q)
    for a in range(2 * q):
        for b in range(2 * q - a):
            c = 2 * q - 1 - a - b
            exact = 1.0 / ((a + 1) * (b + 1) * (c + 1))
            got = np.sum(W * X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** c)
            assert abs(got - exact) < 1e-14


def _cube(h, origin=(0.0, 0.0, 0.0)):
    o = np.asarray(origin)
    return np.array([o + h * np.array([(v >> 0) & 1, (v >> 1) & 1, (v >> 2) & 1]) for v in range(8)], float)


@pytest.mark.parametrize("h,alpha,beta", [(0.25, 1.0, 1.0), (0.5, 2.0, 0.3), (1.0, 0.7, 5.0)])
def test_rt0_cube_closed_form(h, alpha, beta):
    """RT0 on a cube of side h: M = (alpha/h) blockdiag3([[1/3,1/6],[1/6,1/3]])
    + (beta/h^3) d d^T with d = (-1,1,-1,1,-1,1); f_T = (h/2)(fx,fx,fy,fy,fz,fz)."""
    f = np.array([[0.3, -1.2, 2.0]])
    M, fT = element.element_system(0, _cube(h)[None], [alpha], [beta], f)
    blk = np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    d = np.array([-1, 1, -1, 1, -1, 1.0])
    expect = np.kron(np.eye(3), blk) * alpha / h + beta / h ** 3 * np.outer(d, d)
    np.testing.assert_allclose(M[0], expect, rtol=1e-14, atol=1e-14 * np.abs(expect).max())
    np.testing.assert_allclose(fT[0], h / 2 * np.repeat(f[0], 2), rtol=1e-14)


def test_rt0_interior_schur_closed_form():
    """Interior RT0 element, alpha = beta = 1 (Sherman-Morrison):
    H_T = h blockdiag3([[4,2],[2,4]]) - 36h/(h^2+36) 11^T."""
    from oracle import hybrid
    for h in (0.25, 0.5, 0.1):
        M, fT = element.element_system(0, _cube(h)[None], [1.0], [1.0], np.zeros((1, 3)))
        HT, _ = hybrid.local_schur(0, M, fT, 0)
        expect = h * np.kron(np.eye(3), [[4, 2], [2, 4]]) - 36 * h / (h * h + 36) * np.ones((6, 6))
        np.testing.assert_allclose(HT[0], expect, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_affine_quadrature_independence(k):
    """On an affine element the integrands are polynomials of degree <= 2k+2
    per axis, so q = k+2 and q = k+6 give the same matrix."""
    rng = np.random.default_rng(11)
    A = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    ref = _cube(1.0)
    xyz = (ref @ A.T) * 0.3 + 0.1
    M1, f1 = element.element_system(k, xyz[None], [1.7], [0.4], np.array([[1.0, -2.0, 0.5]]))
    M2, f2 = element.element_system(k, xyz[None], [1.7], [0.4], np.array([[1.0, -2.0, 0.5]]), q=k + 6)
    np.testing.assert_allclose(M1, M2, rtol=1e-12, atol=1e-12 * np.abs(M1).max())
    np.testing.assert_allclose(f1, f2, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_element_matrix_spd(k):
    rng = np.random.default_rng(5)
    import synth
    mesh = synth.structured_hex(2, jitter=0.2, rng=rng)
    M, _ = element.element_system(k, mesh.xyz[mesh.e2v], np.ones(8), np.full(8, 1e-2))
    for e in range(8):
        np.testing.assert_allclose(M[e], M[e].T, atol=1e-13 * np.abs(M[e]).max())
        assert np.linalg.eigvalsh(M[e]).min() > 0
