"""Convention-free pins: reproduction of constant fluxes, normal continuity
across faces in physical space, invariance under re-labelled element frames,
and the hybridized mixed form (no GPU)."""
import numpy as np
import pytest

import synth
from oracle import geometry, hybrid, mixed, rt_basis, topology


def field_at(k, xyz_e, u_e, X):
    """Physical flux u = J u_hat / detJ at reference points X (P,3) of one element."""
    val, _ = rt_basis.rt_eval(k, X)
    uh = np.einsum("n,npr->pr", u_e, val)
    J = geometry.jacobians(xyz_e[None], X)[0]
    return np.einsum("prc,pc->pr", J, uh) / np.linalg.det(J)[:, None]


def _affine_mesh(N, seed):
    """Structured mesh under a global affine map (parallelepiped elements)."""
    rng = np.random.default_rng(seed)
    mesh = synth.structured_hex(N)
    A = np.eye(3) + 0.25 * rng.standard_normal((3, 3))
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    mesh.xyz = mesh.xyz @ A.T + rng.standard_normal(3)
    return mesh


def _interp_constant(k, xyz, e2v, c):
    """Nodal dofs of the constant field c on every element: the reference
    normal component of u_hat = detJ J^{-1} c at each node."""
    X = rt_basis.dof_nodes(k)
    d = rt_basis.dof_table(k)[:, 0]
    J = geometry.jacobians(xyz[e2v], X)                     # (E,n,3,3)
    uh = np.linalg.det(J)[..., None] * np.linalg.solve(J, np.broadcast_to(c, J.shape[:-1])[..., None])[..., 0]
    return uh[:, np.arange(X.shape[0]), d]                  # (E,n)


@pytest.mark.parametrize("k", [0, 1, 2])
@pytest.mark.parametrize("affine", [True, False])
def test_constant_flux_reproduced(k, affine):
    """alpha constant, f = alpha c, boundary normal flux of c imposed: the
    discrete solution is the interpolant of c whenever u_hat = detJ J^{-1} c
    lies in the reference RT_k space.  On affine meshes it is constant (any k).
    On trilinear meshes its d-component (the cofactor row J_t0 x J_t1 . c) is
    quadratic in xi_d and linear in the tangential variables: inside RT_k for
    k >= 1, outside RT_0 (the negative control)."""
    rng = np.random.default_rng(40 + k)
    mesh = _affine_mesh(3, 41) if affine else synth.structured_hex(3, jitter=0.2, rng=rng)
    ne = mesh.ne
    c = np.array([0.7, -1.3, 2.1])
    alpha = np.full(ne, 2.5)
    beta = synth.lognormal(rng, ne)
    f = np.tile(2.5 * c, (ne, 1))
    exact = _interp_constant(k, mesh.xyz, mesh.e2v, c)
    ni = rt_basis.n_interior(k)
    g = exact[:, ni:]
    hyb = hybrid.hybridize(k, mesh.xyz, mesh.e2v, alpha, beta, f, g_face=g)
    lam = hybrid.solve_reduced(hyb.H, hyb.r)
    u = hybrid.recover(hyb, mesh.xyz, mesh.e2v, alpha, beta, f, lam, g_face=g)
    err = np.abs(u - exact).max() / np.abs(exact).max()
    if affine or k >= 1:
        assert err < 1e-11
    else:
        assert err > 1e-6


def _face_points(k, f, topo_pi=0):
    """Reference points on local face f at the face-dof nodes, in the face's
    own frame (j0, j1)."""
    d, s = divmod(f, 2)
    t0, t1 = rt_basis.tangential_axes(d)
    zo = rt_basis.open_points(k)
    pts = {}
    for j1 in range(k + 1):
        for j0 in range(k + 1):
            X = np.zeros(3)
            X[d], X[t0], X[t1] = s, zo[j0], zo[j1]
            pts[(j0, j1)] = X
    return pts


def _physical_normal(xyz_e, f, X):
    d, s = divmod(f, 2)
    t0, t1 = rt_basis.tangential_axes(d)
    J = geometry.jacobians(xyz_e[None], X[None])[0, 0]
    n = np.cross(J[:, t0], J[:, t1])
    n = n / np.linalg.norm(n)
    if np.dot(n, J[:, d]) * (2 * s - 1) < 0:
        n = -n
    return n


@pytest.mark.parametrize("k", [0, 1, 2])
@pytest.mark.parametrize("rotate", [False, True])
def test_normal_flux_continuity_physical(k, rotate):
    """At matched physical points of every interior face the two elements'
    fluxes have the same normal component (H(div) conformity)."""
    rng = np.random.default_rng(60 + k)
    mesh = synth.structured_hex(3, jitter=0.2, rng=rng)
    if rotate:
        mesh, _ = synth.rotate_connectivity(mesh, rng)
    ne = mesh.ne
    a, b, f = synth.lognormal(rng, ne), synth.lognormal(rng, ne), synth.element_loads(rng, ne)
    hyb = hybrid.hybridize(k, mesh.xyz, mesh.e2v, a, b, f)
    lam = hybrid.solve_reduced(hyb.H, hyb.r)
    u = hybrid.recover(hyb, mesh.xyz, mesh.e2v, a, b, f, lam)
    topo = hyb.topo
    scale = 0.0
    worst = 0.0
    for fid in range(topo.nfaces):
        eo, fo = topo.face_owner[fid]
        en, fn = topo.face_nbr[fid]
        po, pn = _face_points(k, fo), _face_points(k, fn)
        xo_e, xn_e = mesh.xyz[mesh.e2v[eo]], mesh.xyz[mesh.e2v[en]]
        for key, Xo in po.items():
            xphys = geometry.map_points(xo_e, Xo[None])[0]
            # neighbour point with the same physical location
            cand = [Xn for Xn in pn.values()
                    if np.linalg.norm(geometry.map_points(xn_e, Xn[None])[0] - xphys) < 1e-12]
            assert len(cand) == 1
            nrm = _physical_normal(xo_e, fo, Xo)
            uo = field_at(k, xo_e, u[eo], Xo[None])[0]
            un = field_at(k, xn_e, u[en], cand[0][None])[0]
            worst = max(worst, abs(uo @ nrm - un @ nrm))
            scale = max(scale, abs(uo @ nrm))
    assert worst <= 1e-11 * scale


def _rotation_point_map(perm):
    """Affine map T of the reference cube with corner(v) = T(corner(perm[v]))."""
    corners = np.array([[(v >> 0) & 1, (v >> 1) & 1, (v >> 2) & 1] for v in range(8)], float)
    src = np.hstack([corners[perm], np.ones((8, 1))])
    T, *_ = np.linalg.lstsq(src, corners, rcond=None)
    return lambda X: np.hstack([X, np.ones((X.shape[0], 1))]) @ T


@pytest.mark.parametrize("k", [0, 1, 2])
def test_field_invariant_under_frame_rotation(k):
    """Turning every element's local frame by a random cube rotation changes
    H, lam and the local dofs, but not the physical flux field."""
    rng = np.random.default_rng(80 + k)
    mesh = synth.structured_hex(3, jitter=0.2, rng=rng)
    ne = mesh.ne
    a, b, f = synth.lognormal(rng, ne), synth.lognormal(rng, ne), synth.element_loads(rng, ne)
    rmesh, rot = synth.rotate_connectivity(mesh, rng)
    sols = []
    for m_ in (mesh, rmesh):
        hyb = hybrid.hybridize(k, m_.xyz, m_.e2v, a, b, f)
        lam = hybrid.solve_reduced(hyb.H, hyb.r)
        sols.append(hybrid.recover(hyb, m_.xyz, m_.e2v, a, b, f, lam))
    X = np.random.default_rng(1).uniform(0.05, 0.95, (7, 3))
    worst = scale = 0.0
    for e in range(ne):
        T = _rotation_point_map(synth.CUBE_ROTATIONS[rot[e]])
        Xr = T(X)
        x0 = geometry.map_points(mesh.xyz[mesh.e2v[e]], X)
        x1 = geometry.map_points(rmesh.xyz[rmesh.e2v[e]], Xr)
        assert np.abs(x0 - x1).max() < 1e-13
        u0 = field_at(k, mesh.xyz[mesh.e2v[e]], sols[0][e], X)
        u1 = field_at(k, rmesh.xyz[rmesh.e2v[e]], sols[1][e], Xr)
        worst = max(worst, np.abs(u0 - u1).max())
        scale = max(scale, np.abs(u0).max())
    assert worst <= 1e-10 * scale


@pytest.mark.parametrize("k", [0, 1, 2, 3])
@pytest.mark.parametrize("jit", [0.0, 0.2])
def test_mixed_hybrid_identity(k, jit):
    """H_T from the primal element matrix equals H~_T from the 3x3 mixed block
    system (Sec. 3.2), with the same quadrature, on affine and trilinear
    elements; both boundary and interior elements."""
    rng = np.random.default_rng(90 + k)
    mesh = synth.structured_hex(3, jitter=jit, rng=rng)
    ne = mesh.ne
    a, b = synth.lognormal(rng, ne), synth.lognormal(rng, ne)
    from oracle import element
    topo = topology.build_topology(mesh.e2v)
    for e in (0, 13, 26):
        code = int(((topo.elem_face[e] < 0) * (1 << np.arange(6))).sum())
        M, fT = element.element_system(k, mesh.xyz[mesh.e2v[e]][None], a[e:e + 1], b[e:e + 1],
                                       np.zeros((1, 3)))
        HT, _ = hybrid.local_schur(k, M, fT, code)
        Ht = mixed.mixed_local_schur(k, mesh.xyz[mesh.e2v[e]], a[e], b[e], code)
        # two correct FP64 routes differ by about cond(M_T) * unit roundoff
        tol = max(1e-13, 2e-15 * np.linalg.cond(M[0]))
        assert np.abs(HT[0] - Ht).max() <= tol * np.abs(HT[0]).max()


def test_paper_problem_sizes():
    """Global RT_k dof counts of the paper's soft-hard initial meshes (all
    401,408), from the oracle's face hashing."""
    import json
    import os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_sizes.json")))
    for case in fx["cases"]:
        k, dims = case["k"], tuple(case["dims"])
        mesh = synth.structured_hex(0, dims=dims)
        topo = topology.build_topology(mesh.e2v)
        nf = topo.nfaces + topo.n_boundary_faces
        assert nf * rt_basis.n_face(k) + mesh.ne * rt_basis.n_interior(k) == case["size"], case["cite"]
    for case in fx["closed_form_only"]:
        k, (nx, ny, nz) = case["k"], case["dims"]
        nf = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
        assert nf * rt_basis.n_face(k) + nx * ny * nz * rt_basis.n_interior(k) == case["size"], case["cite"]
