"""Face table and geometry of a conforming simplex mesh (oracle).

TEST INFRASTRUCTURE ONLY.

The paper stores the mesh connectivity face-wise: each edge (face) points to
the two elements that share it, its left and right element (Section 1 and
Section 5, Table 5a).  The
enumeration below is the reading used by this project (the paper gives
none):

* triangles are counter-clockwise; local edge ``k`` joins local vertices
  ``k`` and ``(k + 1) mod 3``; tetrahedra have positive volume and local
  face ``k`` is opposite local vertex ``k``, its vertices listed in
  ascending local order;
* faces are numbered in order of first visit when scanning elements
  ``0..K-1`` and their local faces ``0..F-1``; the first visitor is the left
  element ``L``, the second the right element ``R``; a third visitor, or a
  non-positive element measure, is an error; faces with one visitor are
  boundary faces (``R = -1``);
* the unit normal points from ``L`` to ``R`` and is computed from ``L``'s
  own (unwrapped) coordinates, which makes periodic seams work;
* each face stores its vertex ids in ``L``'s order; quadrature points are
  placed by barycentric weights on these vertices, and each side maps them
  to its own reference coordinates through the position of the vertex ids
  in its own element (``face_ref``; refined meshes set it directly, with a
  coarse side seeing a half edge).

Pins (``tests/test_oracle_mesh.py``): ``E = 3K/2`` on closed triangle
meshes and ``E = 2K`` on closed tetrahedral ones; Euler's formula on the
torus; every element's outward normals weighted by face measure sum to
zero; the total measure equals the domain measure.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .basis import REF_VERTS


def local_faces(kind):
    """Local vertex lists of the faces of the reference element (``kind`` is
    "tri", "quad" or "tet"; the dimension 2 / 3 stands for tri / tet)."""
    if kind in (2, "tri"):
        return [(0, 1), (1, 2), (2, 0)]
    if kind == "quad":
        return [(0, 1), (1, 2), (2, 3), (3, 0)]
    return [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]


class MeshError(ValueError):
    pass


@dataclass
class Mesh:
    dim: int
    K: int
    E: int
    elem_vert: np.ndarray      # [K, nv] vertex ids
    elem_xyz: np.ndarray       # [K, nv, dim]
    face_elem: np.ndarray      # [E, 2] (L, R), R = -1 on the boundary
    face_local: np.ndarray     # [E, 2] local face index in L and R (-1)
    face_vert: np.ndarray      # [E, nfv] vertex ids in L's order
    elem_face: np.ndarray      # [K, F] face id of each local face
    normal: np.ndarray         # [E, dim] unit normal, L -> R
    measure: np.ndarray        # [E] face length / area
    detJ: np.ndarray           # [K]
    Jinv: np.ndarray           # [K, dim, dim], Jinv[d, e] = d xi_d / d x_e
    elem_measure: np.ndarray   # [K]
    face_ref: np.ndarray = None  # [E, 2, nfv, dim]: reference coordinates, seen from L / R,
    #                              of the face's vertices taken in L's order
    kind: str = ""                 # "tri", "quad", "tet" or "mixed" (default from dim)
    elem_kind: np.ndarray = None   # [K] 0 triangle, 1 quadrilateral (mixed meshes only)

    def __post_init__(self):
        if not self.kind:
            self.kind = "tri" if self.dim == 2 else "tet"

    @property
    def n_boundary(self) -> int:
        return int((self.face_elem[:, 1] < 0).sum())

    def face_ref_points(self, f: int, side: int, bary: np.ndarray) -> np.ndarray:
        """Reference coordinates on side ``side`` (0 = L, 1 = R) of the points with
        barycentric weights ``bary[q, :]`` on the face's vertices (L's order)."""
        e = self.face_elem[f, side]
        verts = list(self.elem_vert[e])
        ref = REF_VERTS[self.kind]
        loc = [verts.index(v) for v in self.face_vert[f]]
        return bary @ ref[loc]


def build_mesh(elem_vert, elem_xyz) -> Mesh:
    ev = np.asarray(elem_vert, dtype=np.int64)
    xyz = np.asarray(elem_xyz, dtype=np.float64)
    K, nv = ev.shape
    dim = xyz.shape[2]
    kinds = {(2, 3): "tri", (2, 4): "quad", (3, 4): "tet"}
    if (dim, nv) not in kinds:
        raise MeshError("only triangles, quadrilaterals and tetrahedra are supported")
    kind = kinds[(dim, nv)]
    # a quadrilateral table whose fourth vertex is -1 lists a triangle: mixed mesh
    ek = None
    if kind == "quad" and (ev[:, 3] < 0).any():
        kind = "mixed"
        ek = (ev[:, 3] >= 0).astype(np.int64)
    is_quad = np.full(K, kind == "quad") if ek is None else ek == 1

    def faces_of(i):
        return local_faces("quad" if is_quad[i] else ("tri" if dim == 2 else "tet"))

    F = 4 if dim == 3 or kind in ("quad", "mixed") else 3

    # Jacobians: columns are the edge vectors from local vertex 0 (to vertices
    # 1 and 2 of a simplex, to vertices 1 and 3 of a quadrilateral)
    if dim == 3:
        J = np.stack([xyz[:, a, :] - xyz[:, 0, :] for a in (1, 2, 3)], axis=2)  # J[k, e, d] = dx_e/dxi_d
    else:
        second = np.where(is_quad, 3, 2)
        J = np.stack([xyz[:, 1, :] - xyz[:, 0, :], xyz[np.arange(K), second, :] - xyz[:, 0, :]], axis=2)
    if is_quad.any():
        # the affine map of the unit square: a parallelogram
        q = np.nonzero(is_quad)[0]
        gap = np.abs(xyz[q, 2] - xyz[q, 1] - xyz[q, 3] + xyz[q, 0]).max(axis=1)
        size = np.abs(J[q]).max(axis=(1, 2))
        if (gap > 1e-12 * size).any():
            raise MeshError("quadrilateral %d is not a parallelogram" % int(q[np.argmax(gap / size)]))
    detJ = np.linalg.det(J)
    if (detJ <= 0).any():
        raise MeshError("element %d has non-positive measure" % int(np.argmin(detJ)))
    Jinv = np.linalg.inv(J)  # Jinv[k, d, e] = dxi_d/dx_e
    elem_measure = detJ * np.where(is_quad, 1.0, 0.5 if dim == 2 else 1.0 / 6.0)

    key_to_face = {}
    face_elem = []
    face_local = []
    face_vert = []
    elem_face = np.full((K, F), -1, dtype=np.int64)
    for i in range(K):
        for k, loc in enumerate(faces_of(i)):
            vids = tuple(int(ev[i, a]) for a in loc)
            key = tuple(sorted(vids))
            f = key_to_face.get(key)
            if f is None:
                f = len(face_elem)
                key_to_face[key] = f
                face_elem.append([i, -1])
                face_local.append([k, -1])
                face_vert.append(vids)
            else:
                if face_elem[f][1] != -1:
                    raise MeshError("face %r has more than two elements" % (key,))
                face_elem[f][1] = i
                face_local[f][1] = k
            elem_face[i, k] = f
    face_elem = np.array(face_elem, dtype=np.int64)
    face_local = np.array(face_local, dtype=np.int64)
    face_vert = np.array(face_vert, dtype=np.int64)
    E = len(face_elem)

    # geometry from L's own coordinates (vectorised over faces)
    L = face_elem[:, 0]
    if dim == 3:
        LFv = np.array(local_faces("tet"), dtype=np.int64)[face_local[:, 0]]
    else:
        lq = np.array(local_faces("quad"), dtype=np.int64)
        lt = np.array(local_faces("tri") + [(0, 0)], dtype=np.int64)   # padded to four rows
        LFv = np.where(is_quad[L][:, None], lq[face_local[:, 0]], lt[face_local[:, 0]])
    P = xyz[L[:, None], LFv, :]                           # [E, nfv, dim]
    if dim == 2:
        t = P[:, 1] - P[:, 0]
        measure = np.hypot(t[:, 0], t[:, 1])
        normal = np.stack([t[:, 1], -t[:, 0]], axis=1) / measure[:, None]
    else:
        c = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
        ar = np.linalg.norm(c, axis=1)
        normal = c / ar[:, None]
        opp = xyz[L].mean(axis=1)
        flip = np.einsum("ij,ij->i", P[:, 0] - opp, normal) < 0
        normal[flip] *= -1.0
        measure = 0.5 * ar
    # reference coordinates of the face vertices (L's order) on each side:
    # the position of each vertex id inside the side's element
    face_ref = np.zeros((E, 2, dim, dim))
    for side in (0, 1):
        e = face_elem[:, side]
        has = e >= 0
        es = np.where(has, e, 0)
        evs = ev[es]
        pos = np.argmax(evs[:, None, :] == face_vert[:, :, None], axis=2)
        if dim == 3:
            refs = REF_VERTS["tet"][pos]
        else:
            # triangles never reach position 3 (their fourth id is -1)
            refs = np.where(is_quad[es][:, None, None], REF_VERTS["quad"][pos],
                            REF_VERTS["tri"][np.minimum(pos, 2)])
        face_ref[:, side] = np.where(has[:, None, None], refs, 0.0)
    return Mesh(dim=dim, K=K, E=E, elem_vert=ev, elem_xyz=xyz, face_elem=face_elem,
                face_local=face_local, face_vert=face_vert, elem_face=elem_face,
                normal=normal, measure=measure, detJ=detJ, Jinv=Jinv, elem_measure=elem_measure,
                face_ref=face_ref, kind=kind, elem_kind=ek)
