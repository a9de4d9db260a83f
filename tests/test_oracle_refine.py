"""Pins of the oracle refinement and six-color map (Section 3.2)."""
import numpy as np
import pytest

import synth
from oracle import dg, refine as R
from oracle.coloring import check_coloring, color_faces
from oracle.mesh import build_mesh


def _single(colors_1based):
    # triangle DBA, counter-clockwise; edges DB, BA, AD with the given colors
    D, B, A = 0, 1, 2
    xyz = np.array([[0.0, 0.0], [1.0, 0.0], [0.3, 0.9]])
    edges = [R.Edge(D, B, colors_1based[0] - 1), R.Edge(B, A, colors_1based[1] - 1),
             R.Edge(A, D, colors_1based[2] - 1)]
    return R.RefineState([R.Leaf([D, B, A], xyz, 0, edges)], 3)


def test_paper_worked_example():
    """Parent colors (DB, BA, AD) = (2, 1, 3): BA splits into BG (1) and GA (4);
    the interior edge parallel to AD gets 3 (1-based, as printed)."""
    st, ncl = R.refine(_single((2, 1, 3)), [True])
    assert ncl == 0 and len(st.leaves) == 4
    parent_edges = {}
    for lf in st.leaves:
        for e in lf.edges:
            if e.parent is not None:
                parent_edges[(e.parent.start, e.parent.end)] = e.parent
    BA = parent_edges[(1, 2)]
    BG, GA = BA.children
    assert (BG.start, GA.end) == (1, 2)          # BG contains B, GA contains A
    assert BG.color + 1 == 1 and GA.color + 1 == 4
    center = st.leaves[3]
    # center child's local edge 2 is parallel to parent edge 2 (AD)
    assert center.edges[2].color + 1 == 3
    assert [e.color + 1 for e in center.edges] == [2, 1, 3]   # coarsening recovers the parent colors
    # the printed map c_m = [(c + 3m - 4) mod 6] + 1
    for c in range(1, 4):
        for mch in (1, 2):
            assert R.child_colors(c - 1)[mch - 1] + 1 == ((c + 3 * mch - 4) % 6) + 1


def _c3_like(n=24, levels=3, radius=0.15, seed=0):
    m = synth.periodic_tri(n, jitter=0.0, seed=4)
    M = build_mesh(m["elem_vert"], m["elem_xyz"])
    col, _ = color_faces(M, seed=seed)
    st = R.from_base(M, col)
    for lvl in range(1, levels + 1):
        cen = np.array([lf.xyz.mean(axis=0) for lf in st.leaves])
        lev = np.array([lf.level for lf in st.leaves])
        flags = (lev == lvl - 1) & (np.hypot(cen[:, 0] - 0.5, cen[:, 1] - 0.5) < radius)
        st, _ = R.refine(st, flags)
    return st


def test_refined_coloring_valid_six_colors_balanced():
    st = _c3_like()
    assert R.check_balance(st)
    mesh, color, orient, levels = R.to_mesh(st)
    check_coloring(mesh, color, 6)
    assert set(np.unique(color)) == set(range(6))
    assert levels.max() == 3
    assert abs(mesh.elem_measure.sum() - 1.0) < 1e-13
    assert (orient[:, 1] >= 2).sum() > 0          # hanging faces exist
    # every parent's center child carries the parent colors (coarsening)
    # and every leaf's edges have distinct residues mod 3
    for lf in st.leaves:
        assert len({e.color % 3 for e in lf.edges}) == 3


def test_worst_case_coarse_element_needs_six_colors():
    """A coarse triangle whose three neighbours are refined has six faces,
    one of each color (the paper's Figure 7 bound)."""
    m = synth.periodic_tri(6, jitter=0.0, seed=4)
    M = build_mesh(m["elem_vert"], m["elem_xyz"])
    col, _ = color_faces(M, seed=1)
    st = R.from_base(M, col)
    target = 14
    nbrs = set(M.face_elem[M.elem_face[target]].ravel()) - {target}
    flags = np.zeros(M.K, dtype=bool)
    flags[list(nbrs)] = True
    st, ncl = R.refine(st, flags)
    assert ncl == 0
    mesh, color, orient, levels = R.to_mesh(st)
    new_id = [i for i, lf in enumerate(st.leaves) if lf.level == 0 and lf.verts == [int(v) for v in M.elem_vert[target]]]
    assert len(new_id) == 1
    f = mesh.elem_face[new_id[0]]
    f = f[f >= 0]
    assert len(f) == 6 and sorted(color[f]) == list(range(6))


def test_closure_restores_balance():
    st = _c3_like(n=12, levels=1, radius=0.2)
    # flag one level-1 leaf next to a level-0 leaf: its coarse neighbour must be split too
    lev = np.array([lf.level for lf in st.leaves])
    flags = np.zeros(len(st.leaves), dtype=bool)
    ref = R._referencing(st)
    for i, lf in enumerate(st.leaves):
        if lf.level == 1 and any(e.parent is not None and id(e.parent) in ref for e in lf.edges):
            flags[i] = True
            break
    st2, ncl = R.refine(st, flags)
    assert ncl >= 1 and R.check_balance(st2)


@pytest.mark.parametrize("p", [1, 2])
def test_dg_free_stream_and_conservation_on_refined_mesh(p):
    st = _c3_like(n=16, levels=2, radius=0.2)
    mesh, color, orient, levels = R.to_mesh(st)
    d = dg.Discretization(mesh, p)
    U = synth.perturbed_dofs(mesh.elem_measure, synth.uniform_states(mesh.K, vel=(0.6, 0.3)), d.n_p, eps=0.0)
    scale = np.abs(dg.surface_abs(d, U)).max()
    assert np.abs(dg.rhs(d, U)).max() < 1e-13 * scale
    U = synth.perturbed_dofs(mesh.elem_measure, synth.uniform_states(mesh.K), d.n_p, eps=0.05, seed=2)
    r = dg.rhs(d, U)
    total = (r[:, :, 0] * np.sqrt(mesh.detJ)[:, None]).sum(axis=0)
    assert np.abs(total).max() < 1e-13 * np.abs(r).max() * mesh.K


def test_worked_example_coarsens_back():
    """Refining the worked example and merging the four children restores the
    parent triangle with colors (DB, BA, AD) = (2, 1, 3) (1-based)."""
    st, _ = R.refine(_single((2, 1, 3)), [True])
    st2, n = R.coarsen(st, [True] * 4)
    assert n == 1 and len(st2.leaves) == 1 and st2.origin == [(5, [0, 1, 2, 3])]
    lf = st2.leaves[0]
    assert lf.verts == [0, 1, 2] and lf.level == 0
    assert [e.color + 1 for e in lf.edges] == [2, 1, 3]
    assert all(e.children is None for e in lf.edges)


def test_coarsening_restores_the_base_mesh():
    """Coarsen every family of a three-level refinement, level by level: the
    face table, orientation codes and colors of the conforming base come back."""
    m = synth.periodic_tri(24, jitter=0.0, seed=4)
    M = build_mesh(m["elem_vert"], m["elem_xyz"])
    col, _ = color_faces(M, seed=0)
    base = R.to_mesh(R.from_base(M, col))
    st = _c3_like()
    for _ in range(3):
        st, n = R.coarsen(st, [True] * len(st.leaves))
        assert n > 0 and R.check_balance(st)
    got = R.to_mesh(st)
    assert got[0].K == M.K and got[3].max() == 0
    for a, b in zip(_mesh_arrays_from(got), _mesh_arrays_from(base)):
        assert np.array_equal(a, b)


def _mesh_arrays_from(t):
    mesh, color, orient, levels = t
    return mesh.face_elem, mesh.face_local, orient, color, mesh.elem_vert


def test_coarsening_keeps_balance_and_valid_six_coloring():
    """Random coarsening flags: only families whose children are all flagged
    and unsplit merge; the result stays 2:1 balanced and validly colored."""
    st = _c3_like(n=16, levels=3, radius=0.2)
    rng = np.random.default_rng(3)
    K0 = len(st.leaves)
    st2, n = R.coarsen(st, rng.random(K0) < 0.8)
    assert 0 < n and len(st2.leaves) == K0 - 3 * n
    assert R.check_balance(st2)
    mesh, color, orient, levels = R.to_mesh(st2)
    check_coloring(mesh, color, 6)
    assert abs(mesh.elem_measure.sum() - 1.0) < 1e-13
    assert all(kind in (0, 5) for kind, _ in st2.origin)
    # refining the merged parents again gives a balanced mesh
    flags = [kind == 5 for kind, _ in st2.origin]
    st3, ncl = R.refine(st2, flags)
    assert R.check_balance(st3)
