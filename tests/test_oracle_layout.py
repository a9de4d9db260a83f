"""Pins of the oracle layout against the properties of the paper's Tables 5 and 6."""
import numpy as np
import pytest

import synth
from oracle.coloring import color_faces
from oracle.layout import make_layout
from oracle.mesh import build_mesh


@pytest.mark.parametrize("kind", ["periodic", "delaunay"])
def test_paper_layout_properties(kind):
    if kind == "periodic":
        m = synth.periodic_tri(12, seed=2)
    else:
        m = synth.poisson_delaunay(2000, seed=4)
    M = build_mesh(m["elem_vert"], m["elem_xyz"])
    color, _ = color_faces(M, seed=1)
    new, order, off = make_layout(M, color, "paper")
    assert np.array_equal(np.sort(new), np.arange(M.K))          # bijection
    assert np.array_equal(np.sort(order), np.arange(M.E))
    assert off[0] == 0 and off[-1] == M.E
    L = new[M.face_elem[order, 0]]
    Rraw = M.face_elem[order, 1]
    R = np.where(Rraw >= 0, new[np.where(Rraw >= 0, Rraw, 0)], -1)
    c0 = slice(off[0], off[1])
    N1 = off[1] - off[0]
    k = np.arange(N1)
    assert np.array_equal(L[c0], k)                               # Table 5b: L = k
    interior = R[c0] >= 0
    assert np.array_equal(R[c0][interior], N1 + k[interior])      # Table 5b: R = N_1 + k
    assert interior[: interior.sum()].all()                       # interior faces first
    for c in range(1, len(off) - 1):                              # Table 6b: ascending L
        Lc = L[off[c]:off[c + 1]]
        assert (np.diff(Lc) > 0).all()
    # left/right roles are never exchanged
    assert np.array_equal(color[order], np.repeat(np.arange(len(off) - 1), np.diff(off)))


def test_layout_modes():
    m = synth.periodic_tri(8, seed=5)
    M = build_mesh(m["elem_vert"], m["elem_xyz"])
    color, _ = color_faces(M, seed=1)
    new, order, off = make_layout(M, color, "none")
    assert np.array_equal(new, np.arange(M.K))
    new_r, order_r, _ = make_layout(M, color, "renumber")
    new_p, order_p, _ = make_layout(M, color, "paper")
    assert np.array_equal(new_r, new_p)
    assert np.array_equal(order_r[: off[1]], order_p[: off[1]])
    # renumber-only keeps id order inside later colors
    for c in range(1, 3):
        assert (np.diff(order_r[off[c]:off[c + 1]]) > 0).all()


@pytest.mark.parametrize("kind", ["periodic", "delaunay"])
def test_paired_layout_properties(kind):
    """The paired extension: the interior faces of the first color in blocks of
    16, block b of n faces joining left elements 32 b + i to right elements
    32 b + n + i; its boundary faces' left elements follow; the first color's
    face order is the Morton order of the paper_sfc mode; later colors are
    sorted by left element."""
    if kind == "periodic":
        m = synth.periodic_tri(11, seed=2)
    else:
        m = synth.poisson_delaunay(2000, seed=4)
    M = build_mesh(m["elem_vert"], m["elem_xyz"])
    color, _ = color_faces(M, seed=1)
    new, order, off = make_layout(M, color, "paired")
    _, order_sfc, off_sfc = make_layout(M, color, "paper_sfc")
    assert np.array_equal(off, off_sfc)
    assert np.array_equal(order[: off[1]], order_sfc[: off[1]])
    assert np.array_equal(np.sort(new), np.arange(M.K))
    L = new[M.face_elem[order, 0]]
    Rraw = M.face_elem[order, 1]
    R = np.where(Rraw >= 0, new[np.where(Rraw >= 0, Rraw, 0)], -1)
    n_in = int((R[: off[1]] >= 0).sum())
    k = np.arange(n_in)
    b, i = k // 16, k % 16
    n = np.minimum(16, n_in - 16 * b)
    assert np.array_equal(L[:n_in], 32 * b + i) and np.array_equal(R[:n_in], 32 * b + n + i)
    assert n_in % 16 != 0                                         # the short last block is exercised
    n_bd = off[1] - n_in
    assert np.array_equal(L[n_in: off[1]], 2 * n_in + np.arange(n_bd))
    assert (R[n_in: off[1]] < 0).all()
    for c in range(1, len(off) - 1):
        assert (np.diff(L[off[c]:off[c + 1]]) > 0).all()
