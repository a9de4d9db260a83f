"""Edge (face) coloring heuristic of Section 3 of the paper (oracle).

TEST INFRASTRUCTURE ONLY.

The paper colors the faces with the color set ``C`` of size ``F`` (3 for
triangles, 4 for tetrahedra) in two stages (Section 3.1):

1. a modified greedy pass gives each face, in id order, a color chosen at
   random among the colors that conflict with neither of its elements, or
   leaves it uncolored (a *conflict*) when no such color exists;
2. conflict resolution takes the uncolored faces one at a time and swaps the
   "uncolored" state with a colored face of its left or right element in a
   way that keeps the conflict count, until a conflict-free color is free for
   the face; when the moving conflict returns to a face it already visited
   (a loop), two same-colored faces of its two elements are uncolored and
   the current face takes their color, raising the conflict count by one.

Colors here are 0-based (paper color ``c`` is ``c - 1``).  The paper leaves
the random choices, the swap choice and the loop rule open; the single
specification followed here (and, independently, by the native library) is:

* random numbers: SplitMix64 seeded with ``seed``; ``choose(list)`` returns
  ``list[0]`` for a one-element list, else ``list[next() % len(list)]``;
* ``used(i)`` = colors (>= 0) on element ``i``'s faces;
  ``avail(f) = C - used(L_f) - used(R_f)`` (a boundary face has no ``R``);
* stage 1 visits faces in id order and sets ``color[f] = choose(sorted(avail))``
  when ``avail`` is non-empty;
* stage 2 keeps a FIFO queue initialised with the conflicts in ascending id.
  Popping ``f`` (skipped if already colored) starts a chain with
  ``visited = {f}``, ``cur = f``:

  a. if ``avail(cur)`` is non-empty, ``color[cur] = choose(sorted(avail))``;
     the chain ends;
  b. swap candidates are the faces ``g`` of ``L_cur`` (local order) then of
     ``R_cur`` with ``g != cur``, ``color[g] >= 0`` and ``color[g]`` not used
     by the *other* element of ``cur``;
  c. if some candidates are unvisited, ``g = choose(unvisited)``,
     ``color[cur] = color[g]``, ``color[g] = -1``, ``g`` joins ``visited``,
     ``cur = g``, back to (a) -- one swap;
  d. otherwise (a loop): ``S = sorted(used(L_cur) & used(R_cur))``; if ``S``
     is non-empty, ``x = choose(S)``, ``color[cur] = x``, the ``x``-colored
     face of ``L_cur`` and that of ``R_cur`` are uncolored and appended to
     the queue (L's first) -- one loop break; if ``S`` is empty (possible
     only while another face of ``L_cur`` or ``R_cur`` is still uncolored)
     ``cur`` is appended to the queue to be retried later -- one deferral.
     Either way the chain ends.

* swaps plus loop breaks plus deferrals are capped by ``max_swaps``;
  reaching the cap raises :class:`ColorCapError`.

The standard greedy coloring of Section 1 (smallest color free on both
elements, adding colors as needed) is :func:`greedy_standard`.

Pins: validity and color count are exact (no element has two faces of one
color, every face colored, ``F`` colors); on closed conforming meshes every
color class is a perfect matching, ``N_c = K / 2``, and in general
``2 N_c^int + N_c^bnd = K`` (the identity satisfied by every row of the
paper's Tables 1-3 but one); the fraction of conflicts after stage 1 lies
in a band around the paper's 11-12.6 %.  The order of swaps is **parity
unpinned** by the paper (its worked figures are not available); the native
library is checked bit-exactly against this module under the specification
above.
"""

from __future__ import annotations

from collections import deque

import numpy as np

MASK64 = (1 << 64) - 1


class ColorCapError(RuntimeError):
    pass


class SplitMix64:
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): state += golden gamma, then mix."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def choose(self, items):
        if len(items) == 1:
            return items[0]
        return items[self.next() % len(items)]


def color_faces(mesh, seed: int = 0, max_swaps: int | None = None):
    """Return ``(color[E] int64, stats dict)`` following the specification above."""
    F = mesh.elem_face.shape[1]
    E = mesh.E
    colors = list(range(F))
    # rows of elements with fewer faces (triangles of a mixed mesh) are -1 padded
    elem_face = [[g for g in row if g >= 0] for row in mesh.elem_face.tolist()]
    L = mesh.face_elem[:, 0].tolist()
    R = mesh.face_elem[:, 1].tolist()
    color = [-1] * E
    rng = SplitMix64(seed)
    if max_swaps is None:
        max_swaps = 1000 * E

    def used(e):
        if e < 0:
            return set()
        return {color[g] for g in elem_face[e] if color[g] >= 0}

    def avail(f):
        u = used(L[f]) | used(R[f])
        return [c for c in colors if c not in u]

    # stage 1: modified greedy
    for f in range(E):
        a = avail(f)
        if a:
            color[f] = rng.choose(a)
    conflicts = [f for f in range(E) if color[f] < 0]
    stats = {"conflicts_after_greedy": len(conflicts), "swaps": 0, "loop_breaks": 0,
             "deferrals": 0}

    # stage 2: conflict resolution
    queue = deque(conflicts)
    moves = 0
    while queue:
        f = queue.popleft()
        if color[f] >= 0:
            continue
        visited = {f}
        cur = f
        while True:
            a = avail(cur)
            if a:
                color[cur] = rng.choose(a)
                break
            lc, rc = L[cur], R[cur]
            cand = []
            other_used = used(rc)
            for g in elem_face[lc]:
                if g != cur and color[g] >= 0 and color[g] not in other_used:
                    cand.append(g)
            if rc >= 0:
                other_used = used(lc)
                for g in elem_face[rc]:
                    if g != cur and color[g] >= 0 and color[g] not in other_used:
                        cand.append(g)
            unvisited = [g for g in cand if g not in visited]
            if moves >= max_swaps:
                raise ColorCapError("coloring move cap %d reached" % max_swaps)
            moves += 1
            if unvisited:
                g = rng.choose(unvisited)
                color[cur] = color[g]
                color[g] = -1
                visited.add(g)
                cur = g
                stats["swaps"] += 1
                continue
            S = sorted(used(lc) & used(rc))
            if S:
                x = rng.choose(S)
                gl = next(g for g in elem_face[lc] if color[g] == x)
                gr = next(g for g in elem_face[rc] if color[g] == x)
                color[cur] = x
                color[gl] = -1
                color[gr] = -1
                queue.append(gl)
                if gr != gl:
                    queue.append(gr)
                stats["loop_breaks"] += 1
            else:
                queue.append(cur)
                stats["deferrals"] += 1
            break
    col = np.array(color, dtype=np.int64)
    stats["n_colors"] = F
    stats["count"] = [int((col == c).sum()) for c in range(F)]
    return col, stats


def greedy_standard(mesh):
    """Standard greedy coloring: each face in id order takes the smallest color
    absent from both of its elements (Section 1 of the paper)."""
    E = mesh.E
    elem_face = [[g for g in row if g >= 0] for row in mesh.elem_face.tolist()]
    L = mesh.face_elem[:, 0].tolist()
    R = mesh.face_elem[:, 1].tolist()
    color = [-1] * E
    for f in range(E):
        u = {color[g] for g in elem_face[L[f]] if color[g] >= 0}
        if R[f] >= 0:
            u |= {color[g] for g in elem_face[R[f]] if color[g] >= 0}
        c = 0
        while c in u:
            c += 1
        color[f] = c
    return np.array(color, dtype=np.int64)


def check_coloring(mesh, color, n_colors: int | None = None) -> None:
    """Raise ``AssertionError`` unless every face is colored and no element has
    two faces of the same color (optionally: colors lie in ``0..n_colors-1``)."""
    color = np.asarray(color)
    assert color.shape == (mesh.E,)
    assert (color >= 0).all(), "uncolored faces remain"
    if n_colors is not None:
        assert (color < n_colors).all(), "color out of range"
    ef = mesh.elem_face
    # padding slots (-1, refined meshes) get distinct negative placeholders
    per_elem = np.where(ef >= 0, color[np.where(ef >= 0, ef, 0)], -1 - np.arange(ef.shape[1])[None, :])
    s = np.sort(per_elem, axis=1)
    assert not (s[:, 1:] == s[:, :-1]).any(), "an element has two faces of one color"
