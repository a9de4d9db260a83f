"""Pins of the oracle coloring: RNG vector, validity, counts, paper statistics."""
import json
import os

import numpy as np
import pytest

import synth
from oracle.coloring import ColorCapError, SplitMix64, check_coloring, color_faces, greedy_standard
from oracle.mesh import build_mesh

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def test_splitmix64_published_vector():
    # reference output of SplitMix64 for seed 1234567 (Vigna's splitmix64.c)
    r = SplitMix64(1234567)
    assert [r.next() for _ in range(5)] == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                            4593380528125082431, 16408922859458223821]


def _count_identity(M, color):
    # 2 N_c^interior + N_c^boundary = K for every color of a complete coloring
    inter = M.face_elem[:, 1] >= 0
    for c in range(int(color.max()) + 1):
        sel = color == c
        assert 2 * (sel & inter).sum() + (sel & ~inter).sum() == M.K


@pytest.mark.parametrize("n,seed", [(8, 0), (16, 1), (24, 7)])
def test_periodic_triangles_three_colors_perfect_matchings(n, seed):
    m = synth.periodic_tri(n, seed=seed)
    M = build_mesh(m["elem_vert"], m["elem_xyz"])
    color, st = color_faces(M, seed=seed)
    check_coloring(M, color, 3)
    assert st["count"] == [M.K // 2] * 3  # closed mesh: each color is a perfect matching
    _count_identity(M, color)


def test_delaunay_three_colors_and_conflict_band():
    d = synth.poisson_delaunay(6000, seed=3)
    M = build_mesh(d["elem_vert"], d["elem_xyz"])
    color, st = color_faces(M, seed=2)
    check_coloring(M, color, 3)
    _count_identity(M, color)
    frac = st["conflicts_after_greedy"] / M.E
    # the paper reports 11.0-11.5 % on its triangle meshes (Figure 9, left)
    assert 0.05 < frac < 0.2


def test_tets_four_colors():
    t = synth.kuhn_tets(4, seed=2)
    M = build_mesh(t["elem_vert"], t["elem_xyz"])
    color, st = color_faces(M, seed=5)
    check_coloring(M, color, 4)
    assert st["count"] == [M.K // 2] * 4
    assert 0.05 < st["conflicts_after_greedy"] / M.E < 0.2


def test_standard_greedy_bounds():
    d = synth.poisson_delaunay(3000, seed=1)
    M = build_mesh(d["elem_vert"], d["elem_xyz"])
    g = greedy_standard(M)
    check_coloring(M, g)
    assert g.max() + 1 <= 5
    t = synth.kuhn_tets(3)
    T = build_mesh(t["elem_vert"], t["elem_xyz"])
    g = greedy_standard(T)
    check_coloring(T, g)
    assert g.max() + 1 <= 7


def test_cap_raises():
    m = synth.periodic_tri(10, seed=3)
    M = build_mesh(m["elem_vert"], m["elem_xyz"])
    with pytest.raises(ColorCapError):
        color_faces(M, seed=0, max_swaps=0)


def test_check_coloring_rejects_conflict():
    m = synth.periodic_tri(6)
    M = build_mesh(m["elem_vert"], m["elem_xyz"])
    color, _ = color_faces(M, seed=0)
    bad = color.copy()
    f0, f1 = M.elem_face[0, 0], M.elem_face[0, 1]
    bad[f1] = bad[f0]
    with pytest.raises(AssertionError):
        check_coloring(M, bad, 3)


def test_golden_tables_transcription():
    """Checks the stored fixture, not the oracle: every transcribed row of
    Tables 1 and 3 (tet B excepted: its counts do not add up to its side
    count) distributes all sides over the colors, and the closed sphere rows
    are perfect matchings.  A typo in the fixture fails here."""
    for row in GOLDEN["table1_triangles"]:
        assert sum(row["counts"]) == row["sides"]
        if row.get("closed"):
            assert row["counts"] == [row["elements"] // 2] * 3
    for row in GOLDEN["table3_tetrahedra"]:
        assert sum(row["counts"]) == row["sides"]


def _figure9_fraction(family, sides):
    # the paper's conflicts / sides at the mesh closest in size (Figure 9, left)
    pts = GOLDEN["figure9_conflicts"][family]
    s, c = min(pts, key=lambda sc: abs(np.log(sc[0] / sides)))
    return c / s


@pytest.mark.parametrize("family", ["triangles", "quadrilaterals", "tetrahedra"])
def test_conflicts_after_greedy_match_figure9(family):
    """Conflicts left by the modified greedy stage on unstructured numbering
    (Section 3.1, Figure 9 left): the paper measures 11.0-11.5 % of the sides
    for triangles, 11.2-11.6 % for quadrilaterals and 11.3-12.6 % for
    tetrahedra.  The oracle's stage 1 on meshes of the size of the paper's
    mesh A, numbered in a seeded random order, lands within 2 percentage
    points of the paper's figure for the nearest mesh (measured: 12.6 %,
    11.5 %, 12.0 %).  This is a statistical band: it catches a stage that
    colors far too greedily or too rarely, not the choice among the
    available colors (taking the lowest one moves the three fractions by
    0.6-1.3 points only)."""
    if family == "triangles":
        m = synth.shuffle_elements(synth.poisson_delaunay(5000, seed=3), seed=1)
        F = 3
    elif family == "quadrilaterals":
        m = synth.shuffle_elements(synth.quad_grid(66, seed=1, periodic=False), seed=1)
        F = 4
    else:
        m = synth.shuffle_elements(synth.kuhn_tets(12, seed=2), seed=1)
        F = 4
    M = build_mesh(m["elem_vert"], m["elem_xyz"])
    color, st = color_faces(M, seed=2)
    check_coloring(M, color, F)
    frac = st["conflicts_after_greedy"] / M.E
    want = _figure9_fraction(family, M.E)
    assert abs(frac - want) < 0.02, (family, M.E, frac, want)
