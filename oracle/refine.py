"""Nonconforming 4-way refinement and its six-color edge coloring (oracle).

TEST INFRASTRUCTURE ONLY.

Section 3.2 of the paper: a triangle is refined by joining its edge
midpoints (four children); neighbours may differ by one level, so an edge of
a coarse element can face two finer edges (a hanging node).  The refined
mesh is colored from the conforming base coloring without any search:

* a parent edge of color ``c`` (0-based here) gives its first child edge
  color ``c`` and its second child ``(c + 3) mod 6`` -- the paper's
  ``c_m = [(c + 3m - 4) mod 6] + 1`` in 1-based colors;
* each of the three interior edges takes the color of the parent edge it is
  parallel to;
* coarsening restores the parent colors (the center child carries them).

Readings (the paper's figures are not available):

* children of a parent ``(v0, v1, v2)`` (counter-clockwise) with edge
  midpoints ``m01, m12, m20``: corner children ``(v0, m01, m20)``,
  ``(m01, v1, m12)``, ``(m20, m12, v2)`` and the center child
  ``(m12, m20, m01)``, whose local edge ``k`` is parallel to parent edge
  ``k``; children replace their parent in the leaf list in that order;
* "first child" of an edge: the half containing the edge's *recorded* start
  vertex.  The paper orders child edges counter-clockwise per element, which
  is ambiguous on an edge whose two sides are refined (their
  counter-clockwise orders disagree).  Each edge therefore records its
  orientation once: base edges are oriented counter-clockwise for their left
  element, child edges inherit their parent's orientation, interior edges are
  oriented counter-clockwise for the center child;
* 2:1 closure: before a leaf of level ``l`` is split, every coarser
  edge-neighbour (level ``l - 1``) is split too, recursively; the resulting
  set is the unique smallest balanced superset of the flagged leaves;
* new vertices are numbered in order of first need, splitting leaves in
  ascending id order and their edges ``0, 1, 2``;
* faces of the refined mesh: every unsplit edge node referenced by a leaf.
  Scanning leaves and their local edges creates faces in order of first
  visit; a leaf whose local edge is split visits the two child faces as
  their *coarse* side.  The coarse side of a hanging face is always its
  right element; otherwise the first visitor is the left element.

Pins (``tests/test_oracle_refine.py``): the paper's worked example
(parent colors DB, BA, AD = 2, 1, 3 give BG = 1, GA = 4 and the interior
edge parallel to AD = 3); every refined coloring is valid with at most six
colors; the center child carries the parent colors (coarsening); 2:1 balance;
area conservation; free stream and conservation of the DG operator on the
refined mesh.
"""

from __future__ import annotations

import numpy as np

from .basis import REF_VERTS
from .mesh import Mesh


class Edge:
    __slots__ = ("start", "end", "color", "children", "mid", "parent", "id")

    def __init__(self, start, end, color, parent=None):
        self.start = start
        self.end = end
        self.color = color
        self.children = None
        self.mid = -1
        self.parent = parent
        self.id = -1


class Leaf:
    __slots__ = ("verts", "xyz", "level", "edges", "parent", "child")

    def __init__(self, verts, xyz, level, edges, parent=None, child=-1):
        self.verts = verts      # 3 vertex ids, counter-clockwise
        self.xyz = xyz          # [3, 2] own coordinates
        self.level = level
        self.edges = edges      # 3 Edge nodes; local edge k joins verts[k], verts[k+1]
        self.parent = parent    # the Leaf this one was split from (None on the base mesh)
        self.child = child      # 0..3: corner children at v0, v1, v2, then the center child


class RefineState:
    """Leaves of a (possibly nonconforming) triangle mesh with its edge tree.

    ``origin[i]`` says where leaf ``i`` came from in the previous state:
    ``(0, [j])`` the same leaf ``j``; ``(1 + k, [j])`` child ``k`` of leaf
    ``j``; ``(5, [j0, j1, j2, j3])`` the parent of the four leaves ``j0..j3``
    (children 0..3).  The base state has ``origin = None``."""

    def __init__(self, leaves, n_vert, origin=None):
        self.leaves = leaves
        self.n_vert = n_vert
        self.origin = origin


def from_base(mesh, color) -> RefineState:
    """Edge tree of a colored conforming triangle mesh (one node per face)."""
    if mesh.dim != 2:
        raise ValueError("refinement is defined for triangles")
    color = np.asarray(color)
    nodes = []
    for f in range(mesh.E):
        L = mesh.face_elem[f, 0]
        k = mesh.face_local[f, 0]
        a = int(mesh.elem_vert[L, k])
        b = int(mesh.elem_vert[L, (k + 1) % 3])
        nodes.append(Edge(a, b, int(color[f])))
    leaves = []
    for i in range(mesh.K):
        leaves.append(Leaf([int(v) for v in mesh.elem_vert[i]], mesh.elem_xyz[i].copy(), 0,
                           [nodes[mesh.elem_face[i, k]] for k in range(3)]))
    return RefineState(leaves, int(mesh.elem_vert.max()) + 1)


def child_colors(c: int):
    """Colors of the first and second child of an edge of color ``c``."""
    return c, (c + 3) % 6


def _referencing(state):
    ref = {}
    for i, lf in enumerate(state.leaves):
        for e in lf.edges:
            ref.setdefault(id(e), []).append(i)
    return ref


def closure(state, flags):
    """Smallest superset of the flagged leaves that keeps neighbours within one level."""
    ref = _referencing(state)
    split = {i for i, f in enumerate(flags) if f}
    changed = True
    while changed:
        changed = False
        for i in sorted(split):
            lf = state.leaves[i]
            for e in lf.edges:
                if e.children is None and e.parent is not None:
                    for j in ref.get(id(e.parent), []):
                        if state.leaves[j].level < lf.level and j not in split:
                            split.add(j)
                            changed = True
    return split


def _split_edge(state, e):
    if e.children is None:
        e.mid = state.n_vert
        state.n_vert += 1
        c1, c2 = child_colors(e.color)
        e.children = (Edge(e.start, e.mid, c1, e), Edge(e.mid, e.end, c2, e))


def _half(e, a, b):
    """Child of split edge ``e`` that joins vertices ``a`` and ``b`` (either order)."""
    for ch in e.children:
        if {ch.start, ch.end} == {a, b}:
            return ch
    raise AssertionError("no such half edge")


def refine(state: RefineState, flags):
    """One refinement pass; returns ``(new_state, n_closure)``."""
    split = closure(state, flags)
    n_flag = sum(1 for f in flags if f)
    new_leaves = []
    origin = []
    for i, lf in enumerate(state.leaves):
        if i not in split:
            continue
        for e in lf.edges:
            _split_edge(state, e)
    for i, lf in enumerate(state.leaves):
        if i not in split:
            new_leaves.append(lf)
            origin.append((0, [i]))
            continue
        origin.extend((1 + k, [i]) for k in range(4))
        v0, v1, v2 = lf.verts
        E0, E1, E2 = lf.edges
        m01, m12, m20 = E0.mid, E1.mid, E2.mid
        x = lf.xyz
        x01 = 0.5 * (x[0] + x[1])
        x12 = 0.5 * (x[1] + x[2])
        x20 = 0.5 * (x[2] + x[0])
        # interior edges, oriented counter-clockwise for the center child
        I0 = Edge(m12, m20, E0.color)
        I1 = Edge(m20, m01, E1.color)
        I2 = Edge(m01, m12, E2.color)
        lvl = lf.level + 1
        new_leaves.append(Leaf([v0, m01, m20], np.array([x[0], x01, x20]), lvl,
                               [_half(E0, v0, m01), I1, _half(E2, m20, v0)], lf, 0))
        new_leaves.append(Leaf([m01, v1, m12], np.array([x01, x[1], x12]), lvl,
                               [_half(E0, m01, v1), _half(E1, v1, m12), I2], lf, 1))
        new_leaves.append(Leaf([m20, m12, v2], np.array([x20, x12, x[2]]), lvl,
                               [I0, _half(E1, m12, v2), _half(E2, v2, m20)], lf, 2))
        new_leaves.append(Leaf([m12, m20, m01], np.array([x12, x20, x01]), lvl, [I0, I1, I2], lf, 3))
    return RefineState(new_leaves, state.n_vert, origin), len(split) - n_flag


def coarsen(state: RefineState, flags):
    """One coarsening pass (the inverse of a split, Section 3.2); returns
    ``(new_state, n_merged)``.

    Four leaves merge back into their parent when they are the parent's four
    children, all four are flagged and none of their edges is split (a split
    edge means a neighbour two levels finer than the parent would be).  The
    parent takes the place of its first child.  Its edges are the parent
    edges, which kept their colors: coarsening restores the parent coloring.
    A parent edge whose two halves no leaf references any more is unsplit
    (its midpoint id is not reused)."""
    leaves = state.leaves
    K = len(leaves)
    new_leaves = []
    origin = []
    merged = []
    i = 0
    while i < K:
        lf = leaves[i]
        par = lf.parent
        if (par is not None and lf.child == 0 and i + 3 < K
                and all(leaves[i + k].parent is par and leaves[i + k].child == k for k in range(4))
                and all(flags[i + k] for k in range(4))
                and all(e.children is None for k in range(4) for e in leaves[i + k].edges)):
            new_leaves.append(par)
            origin.append((5, [i, i + 1, i + 2, i + 3]))
            merged.append(par)
            i += 4
            continue
        new_leaves.append(lf)
        origin.append((0, [i]))
        i += 1
    used = {id(e) for lf in new_leaves for e in lf.edges}
    for par in merged:
        for e in par.edges:
            if e.children is not None and not any(id(ch) in used for ch in e.children):
                e.children = None
                e.mid = -1
    return RefineState(new_leaves, state.n_vert, origin), len(merged)


def to_mesh(state: RefineState):
    """Face table, geometry and colors of the leaves (see module header)."""
    leaves = state.leaves
    K = len(leaves)
    faces = {}
    order = []

    def face_of(e):
        rec = faces.get(id(e))
        if rec is None:
            rec = {"edge": e, "fine": [], "coarse": None}
            faces[id(e)] = rec
            order.append(rec)
        return rec

    slots = [[] for _ in range(K)]
    for i, lf in enumerate(leaves):
        for k, e in enumerate(lf.edges):
            if e.children is None:
                rec = face_of(e)
                rec["fine"].append((i, k))
                slots[i].append(rec)
            else:
                w0 = lf.verts[k]
                for ch in e.children:
                    rec = face_of(ch)
                    rec["coarse"] = (i, k, 2 if w0 in (ch.start, ch.end) else 3)
                    slots[i].append(rec)
    E = len(order)
    for f, rec in enumerate(order):
        rec["id"] = f
    face_elem = np.full((E, 2), -1, dtype=np.int64)
    face_local = np.full((E, 2), -1, dtype=np.int64)
    face_orient = np.zeros((E, 2), dtype=np.int64)
    color = np.zeros(E, dtype=np.int64)
    ref = REF_VERTS[2]
    face_ref = np.zeros((E, 2, 2, 2))
    normal = np.zeros((E, 2))
    measure = np.zeros(E)
    for f, rec in enumerate(order):
        color[f] = rec["edge"].color
        fine = rec["fine"]
        if rec["coarse"] is not None:
            assert len(fine) == 1
            (L, kL), (R, kR, o) = fine[0], rec["coarse"]
        else:
            assert 1 <= len(fine) <= 2
            L, kL = fine[0]
            R, kR = fine[1] if len(fine) == 2 else (-1, -1)
            o = 1
        face_elem[f] = (L, R)
        face_local[f] = (kL, kR)
        face_orient[f] = (0, o if R >= 0 else 0)
        A = ref[kL]
        B = ref[(kL + 1) % 3]
        face_ref[f, 0] = (A, B)
        if R >= 0:
            P = ref[kR]
            Qv = ref[(kR + 1) % 3]
            Mv = 0.5 * (P + Qv)
            if o == 1:
                face_ref[f, 1] = (Qv, P)
            elif o == 2:
                face_ref[f, 1] = (Mv, P)
            else:
                face_ref[f, 1] = (Qv, Mv)
        x = leaves[L].xyz
        t = x[(kL + 1) % 3] - x[kL]
        ln = float(np.hypot(t[0], t[1]))
        measure[f] = ln
        normal[f] = (t[1] / ln, -t[0] / ln)
    max_slots = max(len(s) for s in slots)
    elem_face = np.full((K, max_slots), -1, dtype=np.int64)
    for i, s in enumerate(slots):
        for a, rec in enumerate(s):
            elem_face[i, a] = rec["id"]
    xyz = np.array([lf.xyz for lf in leaves])
    ev = np.array([lf.verts for lf in leaves], dtype=np.int64)
    J = np.stack([xyz[:, 1, :] - xyz[:, 0, :], xyz[:, 2, :] - xyz[:, 0, :]], axis=2)
    detJ = np.linalg.det(J)
    mesh = Mesh(dim=2, K=K, E=E, elem_vert=ev, elem_xyz=xyz, face_elem=face_elem, face_local=face_local,
                face_vert=np.zeros((E, 2), dtype=np.int64), elem_face=elem_face, normal=normal,
                measure=measure, detJ=detJ, Jinv=np.linalg.inv(J), elem_measure=detJ / 2.0, face_ref=face_ref)
    levels = np.array([lf.level for lf in leaves], dtype=np.int64)
    return mesh, color, face_orient, levels


def check_balance(state) -> bool:
    """True when no leaf has an edge-neighbour more than one level away."""
    ref = _referencing(state)
    for lf in state.leaves:
        for e in lf.edges:
            if e.children is not None and any(ch.children is not None for ch in e.children):
                return False  # a neighbour two levels finer
            anc = e.parent.parent if e.parent is not None else None
            while anc is not None:
                if id(anc) in ref:
                    return False  # a neighbour two levels coarser
                anc = anc.parent
    return True
