"""Mesh topology, constraint signs and multiplier numbering (test infrastructure).

The constraint matrix C of algebraic hybridization needs Null(C) = Range(P)
(Sec. 2.3).  For RT elements every shared dof is a face dof and each is copied
into exactly two elements, so C can be built face by face: one multiplier per
face dof of every interior face, coupling the two copies of that dof
(Sec. 3.1, W = -I; Example 2.3 with unit weights, i.e. the jump of the normal
component tested against each multiplier node).

Conventions fixed here (the paper leaves them to its library):

* face f = 2d + s of an element is the face xi_d = s; its corner (a, b) along
  the tangential axes (t0, t1) is element vertex s 2^d + a 2^t0 + b 2^t1;
* eps_f = 2s - 1 (reference outward normal is eps_f e_d);
* a face is the set of its four vertex ids; it belongs to one element
  (boundary, all essential) or two (interior); more is an error;
* the owner of an interior face is the element with the smaller index;
  interior faces are numbered in increasing (owner, owner's local face);
* multiplier id = face_id (k+1)^2 + j0 + (k+1) j1 in the owner's face frame;
* the neighbour's face frame maps to the owner's by one of the 8 symmetries of
  the square, code pi: bit 0 swaps the two indices, then bit 1 mirrors the
  first (j -> K - j) and bit 2 mirrors the second; pi is found by matching
  corner vertex ids (K = 1 on corners, K = k on dof indices).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

from . import rt_basis


def face_corner_vertices(f: int) -> list[int]:
    """Element-local vertices of face f, ordered by face corner a + 2b."""
    d, s = divmod(f, 2)
    t0, t1 = rt_basis.tangential_axes(d)
    return [s * (1 << d) + a * (1 << t0) + b * (1 << t1) for b in range(2) for a in range(2)]


def apply_symmetry(pi: int, p0: int, p1: int, K: int) -> tuple[int, int]:
    """Map neighbour-frame indices (p0, p1) to the owner frame."""
    if pi & 1:
        p0, p1 = p1, p0
    if pi & 2:
        p0 = K - p0
    if pi & 4:
        p1 = K - p1
    return p0, p1


@dataclasses.dataclass
class Topology:
    ne: int
    nfaces: int                 # interior faces (the multiplier faces)
    elem_face: np.ndarray       # (ne, 6) int32: interior face id or -1 (boundary)
    elem_pi: np.ndarray         # (ne, 6) uint8: frame code (0 for owner/boundary)
    face_owner: np.ndarray      # (nfaces, 2) int32: (element, local face)
    face_nbr: np.ndarray        # (nfaces, 2) int32: (element, local face)
    face_nbr_pi: np.ndarray     # (nfaces,) uint8
    n_boundary_faces: int


def build_topology(e2v: np.ndarray) -> Topology:
    """Face hashing by sorted vertex 4-tuples (a dictionary)."""
    e2v = np.asarray(e2v)
    ne = e2v.shape[0]
    table: dict[tuple, list[tuple[int, int]]] = {}
    corners = [face_corner_vertices(f) for f in range(6)]
    for e in range(ne):
        for f in range(6):
            key = tuple(sorted(int(v) for v in e2v[e, corners[f]]))
            table.setdefault(key, []).append((e, f))
    interior = []
    nb = 0
    for key, lst in table.items():
        if len(lst) > 2:
            raise ValueError("face shared by more than two elements")
        if len(lst) == 2:
            (e0, f0), (e1, f1) = sorted(lst)
            if e0 == e1:
                raise ValueError("element touches itself")
            interior.append((e0, f0, e1, f1))
        else:
            nb += 1
    interior.sort()
    nf = len(interior)
    elem_face = np.full((ne, 6), -1, dtype=np.int32)
    elem_pi = np.zeros((ne, 6), dtype=np.uint8)
    face_owner = np.zeros((nf, 2), dtype=np.int32)
    face_nbr = np.zeros((nf, 2), dtype=np.int32)
    face_pi = np.zeros(nf, dtype=np.uint8)
    for fid, (eo, fo, en, fn) in enumerate(interior):
        vo = [int(e2v[eo, v]) for v in corners[fo]]
        vn = [int(e2v[en, v]) for v in corners[fn]]
        found = -1
        for pi in range(8):
            ok = True
            for b in range(2):
                for a in range(2):
                    A, B = apply_symmetry(pi, a, b, 1)
                    if vo[A + 2 * B] != vn[a + 2 * b]:
                        ok = False
            if ok:
                found = pi
                break
        if found < 0:
            raise ValueError("faces with the same vertices do not match")
        elem_face[eo, fo] = fid
        elem_face[en, fn] = fid
        elem_pi[en, fn] = found
        face_owner[fid] = (eo, fo)
        face_nbr[fid] = (en, fn)
        face_pi[fid] = found
    return Topology(ne, nf, elem_face, elem_pi, face_owner, face_nbr, face_pi, nb)


def element_multipliers(topo: Topology, k: int, e: int):
    """For element e: list over its local face dofs (in local order) of
    (local dof index, multiplier id or -1, sign eps_f)."""
    K = k + 1
    out = []
    for f in range(6):
        d, s = divmod(f, 2)
        eps = 2 * s - 1
        fid = int(topo.elem_face[e, f])
        pi = int(topo.elem_pi[e, f])
        for j1 in range(K):
            for j0 in range(K):
                loc = rt_basis.face_dof_index(k, f, j0, j1)
                if fid < 0:
                    out.append((loc, -1, eps))
                else:
                    a, b = apply_symmetry(pi, j0, j1, k)
                    out.append((loc, fid * K * K + a + K * b, eps))
    return out


def multiplier_map(topo: Topology, k: int):
    """Arrays (ne, 6(k+1)^2): multiplier id (or -1) and sign of every local
    face dof, in local face-dof order."""
    mf = 6 * (k + 1) ** 2
    mid = np.full((topo.ne, mf), -1, dtype=np.int64)
    sgn = np.zeros((topo.ne, mf), dtype=np.int64)
    for e in range(topo.ne):
        for t, (_, mu, eps) in enumerate(element_multipliers(topo, k, e)):
            mid[e, t] = mu
            sgn[e, t] = eps
    return mid, sgn


def csr_pattern(topo: Topology, k: int):
    """Structural pattern of H: (mu, nu) belongs to H iff both multipliers sit
    on faces of one element.  Returns (row_ptr int64, col int32)."""
    mid, _ = multiplier_map(topo, k)
    m = topo.nfaces * (k + 1) ** 2
    rows, cols = [], []
    for e in range(topo.ne):
        ids = mid[e][mid[e] >= 0]
        rows.append(np.repeat(ids, ids.size))
        cols.append(np.tile(ids, ids.size))
    if rows:
        r = np.concatenate(rows)
        c = np.concatenate(cols)
    else:
        r = np.zeros(0, np.int64)
        c = np.zeros(0, np.int64)
    A = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(m, m)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32)
