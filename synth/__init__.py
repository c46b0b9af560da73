"""Seeded synthetic inputs for the hybridization path: hexahedral meshes,
per-element coefficients, element loads and request streams.

Both the CPU oracle (through the tests) and the GPU path (through the tests and
the bench) draw their inputs from here, so this module holds no arithmetic of
the method itself: only vertex coordinates, connectivity, and random draws.

Conventions
-----------
* Element vertex ``v = a + 2b + 4c`` sits at reference corner ``(a, b, c)``.
* Structured vertex ``(i, j, l)`` has index ``i + (N+1)(j + (N+1) l)`` and
  coordinates ``(i, j, l) / N``; element ``(i, j, l)`` has index
  ``i + N (j + N l)``.
* Every generator takes a ``numpy.random.Generator`` (PCG64 through
  ``numpy.random.default_rng(seed)``) and documents the order of its draws, so
  the same seed always yields the same arrays.
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np


@dataclasses.dataclass
class Mesh:
    """Hexahedral mesh: ``xyz`` (nv, 3) float64, ``e2v`` (ne, 8) int32."""
    xyz: np.ndarray
    e2v: np.ndarray

    @property
    def ne(self) -> int:
        return int(self.e2v.shape[0])

    @property
    def nv(self) -> int:
        return int(self.xyz.shape[0])


def structured_hex(N: int, jitter: float = 0.0, rng: np.random.Generator | None = None,
                   dims: tuple[int, int, int] | None = None) -> Mesh:
    """Unit cube split into ``N^3`` hexahedra (or ``nx*ny*nz`` with ``dims``).

    With ``jitter > 0`` every interior vertex moves by
    ``rng.uniform(-jitter*h, jitter*h, 3)`` (one draw of shape (nv, 3) for all
    vertices, applied to interior ones only, so the domain stays the cube);
    ``h`` is the spacing along each axis.
    """
    nx, ny, nz = dims if dims is not None else (N, N, N)
    vx, vy, vz = nx + 1, ny + 1, nz + 1
    idx = np.arange(vx * vy * vz, dtype=np.int64)
    i = idx % vx
    j = (idx // vx) % vy
    l = idx // (vx * vy)
    xyz = np.stack([i / nx, j / ny, l / nz], axis=1).astype(np.float64)
    if jitter > 0.0:
        assert rng is not None
        h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
        d = rng.uniform(-1.0, 1.0, size=(xyz.shape[0], 3)) * (jitter * h)
        interior = (i > 0) & (i < nx) & (j > 0) & (j < ny) & (l > 0) & (l < nz)
        xyz[interior] += d[interior]
    e = np.arange(nx * ny * nz, dtype=np.int64)
    ei = e % nx
    ej = (e // nx) % ny
    el = e // (nx * ny)
    e2v = np.empty((e.size, 8), dtype=np.int32)
    for c in range(2):
        for b in range(2):
            for a in range(2):
                e2v[:, a + 2 * b + 4 * c] = (ei + a) + vx * ((ej + b) + vy * (el + c))
    return Mesh(xyz=xyz, e2v=e2v)


def _cube_rotations() -> list[np.ndarray]:
    """The 24 proper rotations of the cube as vertex permutations.

    ``perm[v_new] = v_old``: new local vertex ``v_new`` is the old local vertex
    that the rotation carries onto it.  Corners are centred coordinates
    ``2*(a,b,c) - 1``.
    """
    corners = np.array([[(v >> 0) & 1, (v >> 1) & 1, (v >> 2) & 1] for v in range(8)]) * 2 - 1
    perms = []
    for p in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=int)
            for r in range(3):
                R[r, p[r]] = signs[r]
            if round(np.linalg.det(R)) != 1:
                continue
            perm = np.empty(8, dtype=np.int64)
            for v_new in range(8):
                target = R @ corners[v_new]
                v_old = int(np.nonzero((corners == target).all(axis=1))[0][0])
                perm[v_new] = v_old
            perms.append(perm)
    assert len(perms) == 24
    return perms


CUBE_ROTATIONS = _cube_rotations()


def rotate_connectivity(mesh: Mesh, rng: np.random.Generator) -> tuple[Mesh, np.ndarray]:
    """Same geometry, each element's local frame turned by a random proper
    rotation (one ``rng.integers(0, 24, ne)`` draw).  Returns the new mesh and
    the rotation index per element."""
    rot = rng.integers(0, 24, size=mesh.ne)
    e2v = np.empty_like(mesh.e2v)
    for e in range(mesh.ne):
        e2v[e] = mesh.e2v[e, CUBE_ROTATIONS[rot[e]]]
    return Mesh(xyz=mesh.xyz.copy(), e2v=e2v), rot


def lognormal(rng: np.random.Generator, size, sigma: float = 1.0) -> np.ndarray:
    """``exp(sigma * N(0,1))`` with one ``standard_normal(size)`` draw."""
    return np.exp(sigma * rng.standard_normal(size))


def element_loads(rng: np.random.Generator, ne: int) -> np.ndarray:
    """Element-constant load vectors f_T, one ``standard_normal((ne, 3))`` draw."""
    return rng.standard_normal((ne, 3))


@dataclasses.dataclass
class Problem:
    """One hybridization problem: mesh, order, per-element alpha/beta, loads."""
    name: str
    mesh: Mesh
    k: int
    alpha: np.ndarray
    beta: np.ndarray
    f: np.ndarray


def config_c1() -> Problem:
    """RT0 on the 4^3 unit cube, alpha = beta = 1, f ~ N(0,1) (seed 1)."""
    rng = np.random.default_rng(1)
    mesh = structured_hex(4)
    ne = mesh.ne
    f = element_loads(rng, ne)
    return Problem("rt0_4x4x4", mesh, 0, np.ones(ne), np.ones(ne), f)


def config_c2(N: int = 32) -> Problem:
    """RT1 on the structured N^3 cube (affine), alpha = exp(N(0,1)) per
    element, beta = 1, f ~ N(0,1) (seed 2; draws: alpha, then f)."""
    rng = np.random.default_rng(2)
    mesh = structured_hex(N)
    ne = mesh.ne
    alpha = lognormal(rng, ne, 1.0)
    f = element_loads(rng, ne)
    return Problem(f"rt1_{N}x{N}x{N}", mesh, 1, alpha, np.ones(ne), f)


def config_c3(N: int = 48) -> Problem:
    """RT2 on the N^3 cube with interior vertices jittered by +-0.2h
    (trilinear elements), alpha = exp(N(0,1)) clipped to [1e-2, 1e2]
    (contrast 1e4), beta = 1e-2, f ~ N(0,1) (seed 3; draws: jitter, alpha, f)."""
    rng = np.random.default_rng(3)
    mesh = structured_hex(N, jitter=0.2, rng=rng)
    ne = mesh.ne
    alpha = np.clip(lognormal(rng, ne, 1.0), 1e-2, 1e2)
    f = element_loads(rng, ne)
    return Problem(f"rt2_{N}x{N}x{N}_jitter", mesh, 2, alpha, np.full(ne, 1e-2), f)


def config_c4(nprob: int = 64, nmin: int = 8, nmax: int = 24, seed: int = 4) -> list[Problem]:
    """Uneven batch: ``nprob`` jittered n^3 meshes, n ~ U{nmin..nmax},
    k ~ U{0..3}, one alpha ~ lognormal(sigma=1.5) and one beta ~
    lognormal(sigma=0.5) per problem, f ~ N(0,1).  Draws per problem, in
    order: n, k, jitter, alpha, beta, f."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(nprob):
        n = int(rng.integers(nmin, nmax + 1))
        k = int(rng.integers(0, 4))
        mesh = structured_hex(n, jitter=0.2, rng=rng)
        ne = mesh.ne
        a = float(lognormal(rng, (), 1.5))
        b = float(lognormal(rng, (), 0.5))
        f = element_loads(rng, ne)
        out.append(Problem(f"batch{p}_rt{k}_{n}", mesh, k, np.full(ne, a), np.full(ne, b), f))
    return out


def serving_requests(nreq: int, qps: float, seed: int = 5, nmin: int = 16, nmax: int = 64,
                     kmin: int = 1, kmax: int = 3, rmax: int = 8):
    """Request stream modelling implicit time steps: Poisson arrivals at
    ``qps``; mesh N ~ U{nmin..nmax} jittered, k ~ U{kmin..kmax},
    alpha_T = 1/(c*dt*sigma_T) with c = dt = 1 and sigma_T ~ lognormal(0,1),
    beta = 1, R ~ U{1..rmax} right-hand sides with f ~ N(0,1).  Draws per
    request, in order: inter-arrival gap, N, k, R, jitter, sigma, the R loads.
    Yields ``(arrival_time_s, Problem, [f_1..f_R])``."""
    rng = np.random.default_rng(seed)
    t = 0.0
    for r in range(nreq):
        t += float(rng.exponential(1.0 / qps))
        n = int(rng.integers(nmin, nmax + 1))
        k = int(rng.integers(kmin, kmax + 1))
        R = int(rng.integers(1, rmax + 1))
        mesh = structured_hex(n, jitter=0.2, rng=rng)
        ne = mesh.ne
        sigma = lognormal(rng, ne, 1.0)
        alpha = 1.0 / sigma
        fs = [element_loads(rng, ne) for _ in range(R)]
        yield t, Problem(f"req{r}_rt{k}_{n}", mesh, k, alpha, np.ones(ne), fs[0]), fs


# The paper's soft-hard materials test (Sec. 6.1): the unit cube, the two
# inclusion cubes [1/4,1/2]^3 and [1/2,3/4]^3, and the initial meshes of its
# weak-scaling runs per order (equal problem sizes across orders).
SOFTHARD_MESHES = {0: (64, 64, 32), 1: (32, 32, 16), 3: (16, 16, 8)}
SOFTHARD_EXPONENTS = (-8, -4, 0, 4, 8)


def config_softhard(k: int, p: int, dims: tuple[int, int, int] | None = None) -> Problem:
    """Soft-hard materials: the mass coefficient alpha = 10^p on elements whose
    centroid lies in the inclusions and 1 elsewhere, the div-div coefficient
    beta = 1, the load f = (1, 1, 1) (no random draws); mesh ``dims`` (default
    the paper's initial mesh for order k, structured on the unit cube)."""
    dims = dims or SOFTHARD_MESHES[k]
    mesh = structured_hex(0, dims=dims)
    c = mesh.xyz[mesh.e2v].mean(axis=1)
    inc = np.all((c > 0.25) & (c < 0.5), axis=1) | np.all((c > 0.5) & (c < 0.75), axis=1)
    ne = mesh.ne
    alpha = np.where(inc, 10.0 ** p, 1.0)
    return Problem(f"softhard_rt{k}_{dims[0]}x{dims[1]}x{dims[2]}_p{p}", mesh, k, alpha, np.ones(ne),
                   np.ones((ne, 3)))


SPE10_DIMS = (60, 220, 85)
SPE10_CELL = (20.0, 10.0, 2.0)


def config_spe10_standin(dims: tuple[int, int, int] = SPE10_DIMS, seed: int = 10) -> Problem:
    """A synthetic stand-in for the SPE10 problem of Sec. 6.4 (the SPE10 data
    are not available): RT0 on the 60 x 220 x 85 grid of 20 x 10 x 2 cells
    (``dims`` scales the cell count, not the cell size), beta = 1, and a
    layered heavy-tailed mass coefficient in the spirit of the SPE10
    permeability: per z-layer l a mean m_l ~ N(0, 1), per element
    ln alpha = m_l + s_l N(0, 1) with s_l = 1.0 in the top 35/85 of the layers
    and 2.0 below (a smooth and a channelized formation; about 8 decades
    over the grid), f ~ N(0, 1).
    Draws, in order: the layer means, the element normals, the loads."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    mesh = structured_hex(0, dims=dims)
    mesh.xyz *= np.array([nx * SPE10_CELL[0], ny * SPE10_CELL[1], nz * SPE10_CELL[2]])
    ne = mesh.ne
    layer = np.arange(ne) // (nx * ny)
    means = rng.standard_normal(nz)
    sig = np.where(layer < (35 * nz) // 85, 1.0, 2.0)
    alpha = np.exp(means[layer] + sig * rng.standard_normal(ne))
    f = element_loads(rng, ne)
    return Problem(f"spe10_standin_{nx}x{ny}x{nz}", mesh, 0, alpha, np.ones(ne), f)
