"""Seeded synthetic meshes shaped like the paper's workloads.

Every generator returns a dict with

* ``elem_vert`` -- int32 ``[K, nv]`` vertex ids.  On periodic meshes the
  images of a vertex share one id, so faces across the periodic seam are
  matched by id like any other face.
* ``elem_xyz`` -- float64 ``[K, nv, dim]`` *unwrapped* vertex coordinates
  of each element (an element that straddles the seam keeps its own
  geometric copy of the vertices), ordered counter-clockwise in 2D and
  with positive signed volume in 3D.
* ``n_vert`` -- number of distinct vertex ids.

The meshes stand in for the paper's triangular, tetrahedral and refined
meshes (its Tables 1 and 3), which are not distributed with it.
"""

from __future__ import annotations

import itertools

import numpy as np


def periodic_tri(n: int, jitter: float = 0.1, seed: int = 1, length: float = 1.0):
    """``n x n`` cells on the periodic square, each split along the same diagonal.

    Vertex ``(i, j)`` sits at ``(i h, j h)`` plus a displacement drawn from
    ``U(-jitter h, jitter h)`` per coordinate; the displacement of a vertex is
    shared by all its periodic images.  Every cell is cut from its lower-left
    to its upper-right corner, so the edges fall into three direction classes
    (horizontal, vertical, diagonal) -- on the torus the coloring problem is
    then solvable with three colors.
    Element ``2 (i + n j)`` is the lower-right triangle of cell ``(i, j)`` and
    ``2 (i + n j) + 1`` the upper-left one.
    """
    if n < 3:
        raise ValueError("periodic_tri needs n >= 3")
    h = length / n
    rng = np.random.default_rng(seed)
    disp = rng.uniform(-jitter * h, jitter * h, size=(n, n, 2))
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ii = ii.ravel()
    jj = jj.ravel()

    def vid(a, b):
        return (a % n) + n * (b % n)

    def pos(a, b):
        base = np.stack([a * h, b * h], axis=-1).astype(np.float64)
        return base + disp[a % n, b % n]

    c00 = (ii, jj)
    c10 = (ii + 1, jj)
    c11 = (ii + 1, jj + 1)
    c01 = (ii, jj + 1)
    tri_a = [c00, c10, c11]  # lower-right, counter-clockwise
    tri_b = [c00, c11, c01]  # upper-left, counter-clockwise
    K = 2 * n * n
    ev = np.empty((K, 3), dtype=np.int32)
    xyz = np.empty((K, 3, 2), dtype=np.float64)
    for t, tri in enumerate((tri_a, tri_b)):
        for k, (a, b) in enumerate(tri):
            ev[t::2, k] = vid(a, b)
            xyz[t::2, k, :] = pos(a, b)
    return {"elem_vert": ev, "elem_xyz": xyz, "n_vert": n * n, "h": h, "periodic": True}


def quad_grid(n: int, jitter: float = 0.1, seed: int = 1, length: float = 1.0, periodic: bool = True):
    """``n x n`` parallelogram cells, counter-clockwise ``(i,j), (i+1,j), (i+1,j+1), (i,j+1)``.

    Vertex ``(i, j)`` sits at ``(i h + a_i + t_j, j h + b_j + s_i)``: column
    offsets ``a_i``, row offsets ``b_j`` and shears ``s_i``, ``t_j`` drawn from
    ``U(-jitter h, jitter h)``.  A position that is a sum of a per-column and a
    per-row vector makes every cell a parallelogram (an affine image of the
    unit square) while cells differ in size and shape.  ``periodic``: the
    offsets repeat with period ``n`` and vertex ids wrap (a torus; even ``n``
    admits a 4-edge-coloring: horizontal edges by row parity, vertical ones by
    column parity); otherwise the unit square with walls, no shears and fixed
    boundary lines.  Element ``i + n j`` is cell ``(i, j)``.
    """
    if n < 2:
        raise ValueError("quad_grid needs n >= 2")
    h = length / n
    rng = np.random.default_rng(seed)
    a = rng.uniform(-jitter * h, jitter * h, size=n + 1)
    b = rng.uniform(-jitter * h, jitter * h, size=n + 1)
    s = rng.uniform(-jitter * h, jitter * h, size=n + 1)
    t = rng.uniform(-jitter * h, jitter * h, size=n + 1)
    if periodic:
        a[n], b[n], s[n], t[n] = a[0], b[0], s[0], t[0]
    else:
        a[0] = a[n] = b[0] = b[n] = 0.0
        s[:] = 0.0
        t[:] = 0.0
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ii = ii.ravel()
    jj = jj.ravel()
    nv_side = n if periodic else n + 1

    def vid(i, j):
        return (i % nv_side) + nv_side * (j % nv_side) if periodic else i + nv_side * j

    def pos(i, j):
        return np.stack([i * h + a[i] + t[j], j * h + b[j] + s[i]], axis=-1)

    corners = [(ii, jj), (ii + 1, jj), (ii + 1, jj + 1), (ii, jj + 1)]
    ev = np.stack([vid(i, j) for i, j in corners], axis=1).astype(np.int32)
    xyz = np.stack([pos(i, j) for i, j in corners], axis=1)
    return {"elem_vert": ev, "elem_xyz": xyz, "n_vert": nv_side * nv_side, "h": h, "periodic": periodic}


def hybrid_grid(n: int, jitter: float = 0.1, seed: int = 1, radius: float = 0.25, center=(0.5, 0.5),
                periodic: bool = True):
    """Conforming triangle / quadrilateral mesh: the cells of ``quad_grid`` whose
    center lies within ``radius`` of ``center`` are each split into two
    triangles along the diagonal ``(i, j) - (i+1, j+1)`` (lower-right, then
    upper-left), the others stay parallelograms.  Cells are taken row by row.
    Returns ``elem_vert [K, 4]`` with ``-1`` as the fourth vertex of a
    triangle and ``elem_xyz [K, 4, 2]`` with zeros there."""
    g = quad_grid(n, jitter=jitter, seed=seed, periodic=periodic)
    ev4, x4 = g["elem_vert"], g["elem_xyz"]
    cen = x4.mean(axis=1)                    # cell centers
    split = np.hypot(cen[:, 0] - center[0], cen[:, 1] - center[1]) < radius
    # output rows in cell order: a split cell gives two consecutive rows
    start = np.concatenate([[0], np.cumsum(np.where(split, 2, 1))[:-1]])
    K = int(start[-1] + (2 if split[-1] else 1))
    ev = np.full((K, 4), -1, dtype=np.int32)
    xyz = np.zeros((K, 4, 2))
    q = ~split
    ev[start[q]] = ev4[q]
    xyz[start[q]] = x4[q]
    for r, tri in enumerate(((0, 1, 2), (0, 2, 3))):
        rows = start[split] + r
        ev[rows, :3] = ev4[split][:, list(tri)]
        xyz[rows, :3] = x4[split][:, list(tri)]
    return {"elem_vert": ev, "elem_xyz": xyz, "n_vert": g["n_vert"],
            "h": g["h"], "periodic": periodic, "n_tri": int(2 * split.sum()), "n_quad": int((~split).sum())}


def _poisson_disc(radius: float, seed: int, max_fail: int = 12):
    """Poisson-disc points in the unit square, with boundary points every ``radius``.

    Boundary points (the four corners and equally spaced points, at least
    ``radius`` apart, along each side) are placed first.  Interior points are
    then added by parallel dart throwing on a grid of cells of side
    ``radius / sqrt(2)``, which holds at most one point per cell: in each
    round and for each of the nine phases ``(ix mod 3, iy mod 3)`` every
    still-active empty cell of that phase proposes one uniform point, which
    is accepted when no accepted point lies closer than ``radius``.  Cells
    of one phase are three cells apart, so proposals of a phase never
    conflict with each other.  A cell stops proposing after ``max_fail``
    rejected proposals.
    """
    rng = np.random.default_rng(seed)
    g = radius / np.sqrt(2.0)
    G = int(np.ceil(1.0 / g))
    grid = -np.ones((G + 4, G + 4), dtype=np.int64)  # 2-cell apron on each side

    m = int(np.floor(1.0 / radius))
    side = np.linspace(0.0, 1.0, m + 1)
    bnd = set()
    for t in side:
        for p in ((t, 0.0), (t, 1.0), (0.0, t), (1.0, t)):
            bnd.add((float(p[0]), float(p[1])))
    coords = np.array(sorted(bnd), dtype=np.float64)
    cx = np.minimum((coords[:, 0] / g).astype(np.int64), G - 1) + 2
    cy = np.minimum((coords[:, 1] / g).astype(np.int64), G - 1) + 2
    if len(set(zip(cx.tolist(), cy.tolist()))) != len(coords):
        raise RuntimeError("two boundary points share a grid cell")
    grid[cx, cy] = np.arange(len(coords))
    npts = len(coords)

    offs = [(dx, dy) for dx in range(-2, 3) for dy in range(-2, 3)]
    phases = []
    for px in range(3):
        for py in range(3):
            ax = np.arange(2 + px, G + 2, 3)
            ay = np.arange(2 + py, G + 2, 3)
            AX, AY = np.meshgrid(ax, ay, indexing="ij")
            AX = AX.ravel()
            AY = AY.ravel()
            keep = grid[AX, AY] < 0
            phases.append([AX[keep], AY[keep], np.zeros(keep.sum(), dtype=np.int64)])
    while any(ph[0].size for ph in phases):
        for ph in phases:
            CX, CY, fails = ph
            if CX.size == 0:
                continue
            u = rng.random((CX.size, 2))
            cand = np.stack([(CX - 2 + u[:, 0]) * g, (CY - 2 + u[:, 1]) * g], axis=1)
            ok = (cand[:, 0] < 1.0) & (cand[:, 1] < 1.0) & (cand[:, 0] > 0.0) & (cand[:, 1] > 0.0)
            for dx, dy in offs:
                nb = grid[CX + dx, CY + dy]
                has = nb >= 0
                if not has.any():
                    continue
                q = coords[np.where(has, nb, 0)]
                d2 = ((q - cand) ** 2).sum(axis=1)
                ok &= ~(has & (d2 < radius * radius))
            acc = np.nonzero(ok)[0]
            if acc.size:
                ids = np.arange(npts, npts + acc.size)
                grid[CX[acc], CY[acc]] = ids
                coords = np.concatenate([coords, cand[acc]], axis=0)
                npts += acc.size
            fails = fails + (~ok)
            alive = (~ok) & (fails < max_fail)
            ph[0], ph[1], ph[2] = CX[alive], CY[alive], fails[alive]
    return coords


def poisson_delaunay(n_points: int = 500_000, seed: int = 2, radius: float | None = None):
    """Delaunay triangulation of about ``n_points`` seeded Poisson-disc points.

    The unit square has reflective walls, so the mesh is not periodic and
    ``elem_xyz`` is simply the vertex coordinates.  The disc radius is
    chosen from the measured packing density of the sampler
    (``N ~ 0.645 / r^2``) unless given.  Triangles are ordered as Qhull
    returns them and re-oriented counter-clockwise; zero-area triangles
    (collinear boundary points) are dropped.
    """
    from scipy.spatial import Delaunay  # generator-only dependency

    if radius is None:
        radius = float(np.sqrt(0.6446 / n_points))
    pts = _poisson_disc(radius, seed)
    tri = Delaunay(pts)
    ev = tri.simplices.astype(np.int32).copy()
    xyz = pts[ev]
    area2 = (xyz[:, 1, 0] - xyz[:, 0, 0]) * (xyz[:, 2, 1] - xyz[:, 0, 1]) - (
        xyz[:, 2, 0] - xyz[:, 0, 0]
    ) * (xyz[:, 1, 1] - xyz[:, 0, 1])
    neg = area2 < 0
    ev[neg, 1], ev[neg, 2] = ev[neg, 2].copy(), ev[neg, 1].copy()
    keep = np.abs(area2) > 1e-14 * radius * radius
    ev = np.ascontiguousarray(ev[keep])
    xyz = np.ascontiguousarray(pts[ev])
    return {"elem_vert": ev, "elem_xyz": xyz, "n_vert": len(pts), "h": radius, "periodic": False,
            "points": pts}


def lattice_delaunay(n_points: int, seed: int = 7, jitter: float = 0.3):
    """Delaunay triangulation of about ``n_points`` points of a jittered
    square lattice in the unit square (interior points moved by
    U(-jitter h, jitter h) per coordinate, boundary points on the sides):
    a fast stand-in for the Poisson-disc mesh at sizes where the dart
    throwing would dominate (used for the coloring-time sweep).  Walls, no
    periodicity; counter-clockwise triangles in Qhull's order."""
    from scipy.spatial import Delaunay  # generator-only dependency

    n = max(3, int(round(np.sqrt(n_points))))
    h = 1.0 / (n - 1)
    rng = np.random.default_rng(seed)
    g = np.linspace(0.0, 1.0, n)
    X, Y = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    inner = (pts[:, 0] > 0) & (pts[:, 0] < 1) & (pts[:, 1] > 0) & (pts[:, 1] < 1)
    pts[inner] += rng.uniform(-jitter * h, jitter * h, size=(int(inner.sum()), 2))
    tri = Delaunay(pts)
    ev = tri.simplices.astype(np.int32).copy()
    xyz = pts[ev]
    area2 = (xyz[:, 1, 0] - xyz[:, 0, 0]) * (xyz[:, 2, 1] - xyz[:, 0, 1]) - (
        xyz[:, 2, 0] - xyz[:, 0, 0]
    ) * (xyz[:, 1, 1] - xyz[:, 0, 1])
    neg = area2 < 0
    ev[neg, 1], ev[neg, 2] = ev[neg, 2].copy(), ev[neg, 1].copy()
    keep = np.abs(area2) > 1e-14 * h * h
    ev = np.ascontiguousarray(ev[keep])
    return {"elem_vert": ev, "elem_xyz": np.ascontiguousarray(pts[ev]), "n_vert": len(pts), "h": h,
            "periodic": False}


def kuhn_tets(n: int, jitter: float = 0.05, seed: int = 3, length: float = 1.0, periodic: bool = True):
    """``n^3`` periodic cubes, each split into the six Kuhn tetrahedra.

    Every tetrahedron of cube ``(i, j, k)`` runs from the cube's corner
    ``(0,0,0)`` to its corner ``(1,1,1)`` through one monotone lattice path
    (one per permutation of the axes).  Vertices are displaced by
    ``U(-jitter h, jitter h)`` per coordinate, identically for periodic
    images.  Odd permutations list their vertices with the middle two
    swapped so that every tetrahedron has positive volume.
    Element ``6 (i + n j + n^2 k) + s`` uses the ``s``-th permutation of
    ``itertools.permutations(range(3))``.  With ``periodic=False`` the cube
    is closed by reflective walls: the ``(n+1)^3`` lattice vertices are all
    distinct and only the interior ones are displaced.
    """
    if n < 2:
        raise ValueError("kuhn_tets needs n >= 2")
    h = length / n
    rng = np.random.default_rng(seed)
    nv = n if periodic else n + 1
    disp = rng.uniform(-jitter * h, jitter * h, size=(nv, nv, nv, 3))
    if not periodic:
        disp[[0, -1], :, :] = 0.0
        disp[:, [0, -1], :] = 0.0
        disp[:, :, [0, -1]] = 0.0
    idx = np.arange(n)
    I, J, Kc = np.meshgrid(idx, idx, idx, indexing="ij")
    # cube order: i fastest, then j, then k
    I = I.transpose(2, 1, 0).ravel()
    J = J.transpose(2, 1, 0).ravel()
    Kc = Kc.transpose(2, 1, 0).ravel()
    ncube = n ** 3
    perms = list(itertools.permutations(range(3)))
    ev = np.empty((6 * ncube, 4), dtype=np.int32)
    xyz = np.empty((6 * ncube, 4, 3), dtype=np.float64)

    def vid(a, b, c):
        return (a % nv) + nv * (b % nv) + nv * nv * (c % nv)

    def pos(a, b, c):
        base = np.stack([a * h, b * h, c * h], axis=-1).astype(np.float64)
        return base + disp[a % nv, b % nv, c % nv]

    for s, perm in enumerate(perms):
        corner = [np.zeros(3, dtype=np.int64)]
        for ax in perm:
            nxt = corner[-1].copy()
            nxt[ax] += 1
            corner.append(nxt)
        # parity of the permutation decides the vertex order
        inv = sum(1 for x in range(3) for y in range(x + 1, 3) if perm[x] > perm[y])
        order = [0, 1, 2, 3] if inv % 2 == 0 else [0, 2, 1, 3]
        for slot, c in enumerate(order):
            off = corner[c]
            a, b, cc = I + off[0], J + off[1], Kc + off[2]
            ev[s::6, slot] = vid(a, b, cc)
            xyz[s::6, slot, :] = pos(a, b, cc)
    # orientation check (input sanity, not part of the method)
    vol = element_measure(xyz)
    if (vol <= 0).any():
        flip = vol <= 0
        ev[flip, 1], ev[flip, 2] = ev[flip, 2].copy(), ev[flip, 1].copy()
        xyz[flip, 1], xyz[flip, 2] = xyz[flip, 2].copy(), xyz[flip, 1].copy()
    return {"elem_vert": ev, "elem_xyz": xyz, "n_vert": nv ** 3, "h": h, "periodic": periodic}


def shuffle_elements(mesh: dict, seed: int) -> dict:
    """The same mesh with its elements numbered in a seeded random order.

    A mesh generator hands out element numbers in its own order; structured
    generators (a grid scanned row by row, Qhull's output) number neighbours
    close together, which lets a greedy pass in id order leave fewer
    conflicts than on the paper's unstructured meshes.  A random numbering is
    the stand-in for that order.  Vertex ids and coordinates are unchanged."""
    perm = np.random.default_rng(seed).permutation(len(mesh["elem_vert"]))
    out = dict(mesh)
    out["elem_vert"] = np.ascontiguousarray(np.asarray(mesh["elem_vert"])[perm])
    out["elem_xyz"] = np.ascontiguousarray(np.asarray(mesh["elem_xyz"])[perm])
    out["elem_order"] = perm
    return out


def _tri_rows(elem_xyz, elem_vert):
    """Rows of a 4-slot 2D table that hold triangles (fourth vertex id -1)."""
    if elem_vert is None:
        return np.zeros(len(elem_xyz), dtype=bool)
    return np.asarray(elem_vert)[:, 3] < 0


def element_measure(elem_xyz: np.ndarray, elem_vert=None) -> np.ndarray:
    """Signed area (triangles, parallelograms) or volume (tetrahedra) of each
    element; for a 4-slot 2D table pass ``elem_vert`` so that the rows with a
    -1 fourth vertex are taken as triangles."""
    x = np.asarray(elem_xyz, dtype=np.float64)
    if x.shape[2] == 2 and x.shape[1] in (3, 4):
        a = x[:, 1] - x[:, 0]
        if x.shape[1] == 3:
            b = x[:, 2] - x[:, 0]
            return 0.5 * (a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0])
        tri = _tri_rows(x, elem_vert)
        b = np.where(tri[:, None], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0])
        return np.where(tri, 0.5, 1.0) * (a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0])
    if x.shape[1] == 4 and x.shape[2] == 3:
        a = x[:, 1] - x[:, 0]
        b = x[:, 2] - x[:, 0]
        c = x[:, 3] - x[:, 0]
        return np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0
    raise ValueError("unsupported element shape %r" % (x.shape,))


def element_centroid(elem_xyz: np.ndarray, elem_vert=None) -> np.ndarray:
    """Vertex average of each element (a 4-slot 2D table with ``elem_vert``:
    the triangles' first three vertices)."""
    x = np.asarray(elem_xyz, dtype=np.float64)
    c = x.mean(axis=1)
    if x.shape[1] == 4 and x.shape[2] == 2 and elem_vert is not None:
        tri = _tri_rows(x, elem_vert)
        c[tri] = x[tri, :3].mean(axis=1)
    return c


def refine_flags(elem_xyz: np.ndarray, levels: np.ndarray, level: int, center=(0.5, 0.5),
                 radius: float = 0.15) -> np.ndarray:
    """Refinement criterion of the adaptive workload: leaves of ``level`` whose
    centroid lies within ``radius`` of ``center``."""
    c = np.asarray(elem_xyz, dtype=np.float64).mean(axis=1)
    d = np.hypot(c[:, 0] - center[0], c[:, 1] - center[1])
    return (np.asarray(levels) == level) & (d < radius)


def adapt_flags(elem_xyz: np.ndarray, levels: np.ndarray, center, r_refine: float, r_coarsen: float,
                max_level: int, period: float = 1.0):
    """Criteria of the moving-feature workload on a periodic square: refine
    leaves below ``max_level`` whose centroid lies within ``r_refine`` of
    ``center`` (distance to the nearest periodic image), coarsen leaves above
    level 0 farther than ``r_coarsen``.  Returns ``(refine, coarsen)`` flags."""
    c = np.asarray(elem_xyz, dtype=np.float64).mean(axis=1)
    d = c - np.asarray(center, dtype=np.float64)[None, :]
    d -= period * np.round(d / period)
    r = np.hypot(d[:, 0], d[:, 1])
    lev = np.asarray(levels)
    return (lev < max_level) & (r < r_refine), (lev > 0) & (r > r_coarsen)
