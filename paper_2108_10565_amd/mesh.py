"""Periodic tetrahedral mesh of a cube (input geometry of the corrector).

This module holds no arithmetic of the method: it builds the connectivity and
the corner coordinates of a mesh, which both the corrector's tests and its
benchmark take as input.

The cube [-1, 1]^3 (section "Planar wave convergence analysis") is divided
into m^3 equal sub-cubes, each split into 5 tetrahedra: the central one on
four alternate corners and one at each remaining corner.  Neighbouring
sub-cubes use the two alternate corner sets in turn (by the parity of
i + j + k), so the face diagonals match and the mesh is conforming; m must
be even for the periodic wrap to keep that pattern (and at least 4).

Faces follow the ABI convention of the corrector: local face f of an
element is the vertex triple FACE_VERTICES[f] of its corners.  For every
(element, face): the element behind it, and the code 6 j + h, where j is
that element's face and h the vertex correspondence (own face vertex r is the
neighbour face's vertex PERMUTATIONS[h][r]).
"""
from __future__ import annotations

import dataclasses

import numpy as np

FACE_VERTICES = ((0, 2, 1), (0, 1, 3), (0, 3, 2), (1, 2, 3))
PERMUTATIONS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))

_EVEN = ((0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1))
_ODD = ((1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1))


@dataclasses.dataclass
class Mesh:
    m: int                  # sub-cubes per direction
    vertices: np.ndarray    # (n, 4, 3) corner coordinates (unwrapped: inside the element's sub-cube)
    vertex_ids: np.ndarray  # (n, 4) periodic vertex ids
    neighbor: np.ndarray    # (n, 4) int32 element behind each face
    nb_code: np.ndarray     # (n, 4) int32 6 j + h
    shift: np.ndarray       # (n, 4, 3) coordinates of the neighbour minus own, for the shared face

    @property
    def n(self) -> int:
        return self.vertices.shape[0]

    @property
    def h(self) -> float:
        """Edge length of the sub-cubes."""
        return 2.0 / self.m


def _corner_tets(parity):
    centre, other = (_EVEN, _ODD) if parity == 0 else (_ODD, _EVEN)
    tets = [centre]
    for o in other:
        nbrs = [c for c in centre if sum(abs(a - b) for a, b in zip(c, o)) == 1]
        tets.append((o,) + tuple(nbrs))
    return tets


def periodic_cube(m: int) -> Mesh:
    if m < 4 or m % 2:
        # m = 2 would give distinct faces with the same periodic vertex set
        raise ValueError("m must be even and >= 4")
    verts, ids = [], []
    for i in range(m):
        for j in range(m):
            for k in range(m):
                for tet in _corner_tets((i + j + k) % 2):
                    pts = np.array([[i + c[0], j + c[1], k + c[2]] for c in tet], float)
                    d = np.linalg.det(np.stack([pts[1] - pts[0], pts[2] - pts[0], pts[3] - pts[0]], axis=1))
                    order = [0, 1, 2, 3] if d > 0 else [0, 2, 1, 3]
                    pts = pts[order]
                    verts.append(-1.0 + pts * (2.0 / m))
                    ids.append([((int(p[0]) % m) * m + int(p[1]) % m) * m + int(p[2]) % m for p in pts])
    verts = np.array(verts)
    ids = np.array(ids, dtype=np.int64)
    n = len(ids)
    faces = {}
    for e in range(n):
        for f, tri in enumerate(FACE_VERTICES):
            key = frozenset(int(ids[e, v]) for v in tri)
            faces.setdefault(key, []).append((e, f))
    neighbor = np.empty((n, 4), np.int32)
    code = np.empty((n, 4), np.int32)
    shift = np.empty((n, 4, 3))
    for key, pair in faces.items():
        if len(pair) != 2:
            raise RuntimeError("non-conforming mesh")
        for (e, f), (e2, f2) in (pair, pair[::-1]):
            own = [int(ids[e, v]) for v in FACE_VERTICES[f]]
            oth = [int(ids[e2, v]) for v in FACE_VERTICES[f2]]
            perm = tuple(oth.index(g) for g in own)
            neighbor[e, f] = e2
            code[e, f] = 6 * f2 + PERMUTATIONS.index(perm)
            shift[e, f] = verts[e2, FACE_VERTICES[f2][perm[0]]] - verts[e, FACE_VERTICES[f][0]]
    return Mesh(m=m, vertices=verts, vertex_ids=ids, neighbor=neighbor, nb_code=code, shift=shift)
