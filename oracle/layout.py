"""Color-based element renumbering and face reordering of Section 5 (oracle).

TEST INFRASTRUCTURE ONLY.

The paper's preprocessing (Section 5, Tables 5 and 6):

1. faces are grouped by color (stable: original id order inside a color);
2. the left and right elements of the ``k``-th face of the first color are
   renumbered ``k`` and ``N_1 + k`` (``N_1`` = number of faces of that
   color), so that one thread per face reads consecutive elements;
3. the faces of every later color are reordered by ascending (new) left
   element; left/right roles are not exchanged (Table 6b keeps ``L = 103``,
   ``R = 65``).

Readings where the paper is silent:

* boundary faces of the first color have no right element; they are placed
  after the interior faces of that color (each part in id order), so the
  interior face ``k`` maps to ``(k, N_1 + k)`` and the numbering stays dense
  (``K = N_1 + I_1`` with ``I_1`` interior faces);
* general (nonconforming) meshes, where an element can miss a color: colors
  are processed in order; for color ``c`` the still-unnumbered left elements
  of its faces (in the color's current face order) are numbered first,
  consecutively, then the still-unnumbered right elements; afterwards the
  color's faces are sorted by new left element.  On conforming meshes this
  is exactly steps 2-3 (every element is touched by the first color).

Modes: ``"paper"`` (steps 1-3), ``"renumber"`` (1-2 only, faces of later
colors keep id order), ``"none"`` (1 only, identity element numbering) and
``"paper_sfc"`` -- an extension that is not in the paper: the interior and
the boundary faces of the first color are each put in Morton (Z-curve)
order of their midpoints (ties by id) before step 2.  Midpoints are taken
from the left element's coordinates and quantised to ``2^31`` (2D) or
``2^21`` (3D) cells of their bounding box.  ``"paired"`` -- a second
extension: the first color's interior faces in the same Morton order, cut
into blocks of ``PAIR_BLOCK`` faces (the last one shorter); block ``b`` with
``n`` faces numbers its left elements ``2 PAIR_BLOCK b + i`` and its right
elements ``2 PAIR_BLOCK b + n + i`` (``i < n``), so the two elements of a
face are never more than ``2 PAIR_BLOCK`` ids apart; the left elements of
the boundary faces of that color follow; later colors as in ``"paper"``.

Returns ``elem_new[K]`` (new id of original element ``i``), ``face_order[E]``
(original face id at each layout position) and ``color_off[F + 1]``.

Pins (``tests/test_oracle_layout.py``): bijection; first-color face ``k`` has
``(L, R) = (k, N_1 + k)``; later colors have strictly ascending ``L``;
orientation preserved.
"""

from __future__ import annotations

import numpy as np

PAIR_BLOCK = 16


def morton_order(mesh, faces):
    """``faces`` sorted by the Morton code of their midpoints, ties by id."""
    from .mesh import local_faces

    faces = list(faces)
    if not faces:
        return faces
    dim = mesh.dim

    def faces_of(e):
        if mesh.kind == "mixed":
            return local_faces("quad" if mesh.elem_kind[e] == 1 else "tri")
        return local_faces(mesh.kind)

    bits = 31 if dim == 2 else 21
    scale = float(2 ** bits)
    mids = []
    for f in faces:
        L = mesh.face_elem[f, 0]
        x = mesh.elem_xyz[L]
        verts = faces_of(L)[mesh.face_local[f, 0]]
        m = []
        for d in range(dim):
            s = 0.0
            for a in verts:
                s += float(x[a, d])
            m.append(s / dim)
        mids.append(m)
    mids = np.array(mids)
    lo = mids.min(axis=0)
    hi = mids.max(axis=0)
    codes = []
    for m in mids:
        c = 0
        for d in range(dim):
            ext = hi[d] - lo[d] if hi[d] > lo[d] else 1.0
            t = (m[d] - lo[d]) / ext * scale
            q = int(scale) - 1 if t >= scale else (int(t) if t > 0 else 0)
            for b in range(bits):
                c |= ((q >> b) & 1) << (b * dim + d)
        codes.append(c)
    return [f for _, f in sorted(zip(codes, faces))]


def make_layout(mesh, color, mode: str = "paper"):
    color = np.asarray(color, dtype=np.int64)
    if (color < 0).any():
        raise ValueError("layout needs a complete coloring")
    n_colors = int(color.max()) + 1
    L = mesh.face_elem[:, 0]
    R = mesh.face_elem[:, 1]
    groups = []
    for c in range(n_colors):
        ids = [f for f in range(mesh.E) if color[f] == c]
        if c == 0 and mode in ("paper_sfc", "paired"):
            ids = morton_order(mesh, [f for f in ids if R[f] >= 0]) + morton_order(mesh, [f for f in ids if R[f] < 0])
        elif c == 0 and mode != "none":
            ids = [f for f in ids if R[f] >= 0] + [f for f in ids if R[f] < 0]
        groups.append(ids)

    if mode == "none":
        elem_new = np.arange(mesh.K, dtype=np.int64)
    else:
        elem_new = np.full(mesh.K, -1, dtype=np.int64)
        nxt = 0
        for c, ids in enumerate(groups):
            if c == 0 and mode == "paired":
                interior = [f for f in ids if R[f] >= 0]
                for b0 in range(0, len(interior), PAIR_BLOCK):
                    block = interior[b0:b0 + PAIR_BLOCK]
                    for side in (L, R):
                        for f in block:
                            elem_new[side[f]] = nxt
                            nxt += 1
                for f in ids:
                    if R[f] < 0:
                        elem_new[L[f]] = nxt
                        nxt += 1
                continue
            for side in (L, R):
                for f in ids:
                    e = side[f]
                    if e >= 0 and elem_new[e] < 0:
                        elem_new[e] = nxt
                        nxt += 1
        if nxt != mesh.K:
            raise ValueError("some elements have no face")

    order = []
    off = [0]
    for c, ids in enumerate(groups):
        if mode in ("paper", "paper_sfc", "paired") and c > 0:
            ids = sorted(ids, key=lambda f: elem_new[L[f]])
        order.extend(ids)
        off.append(len(order))
    return elem_new, np.array(order, dtype=np.int64), np.array(off, dtype=np.int64)
