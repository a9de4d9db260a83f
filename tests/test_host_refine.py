"""Native refinement (dgc_mesh_refine) against the oracle: bit-exact leaves,
vertex ids, coordinates, face table, six-color map and layout."""
import numpy as np
import pytest

import synth
from oracle import refine as R
from oracle.coloring import check_coloring, color_faces
from oracle.layout import make_layout
from oracle.mesh import build_mesh

dgc = pytest.importorskip("paper_1601_07613_amd")


def _run(m, levels, radius, cseed):
    O = build_mesh(m["elem_vert"], m["elem_xyz"])
    col, _ = color_faces(O, seed=cseed)
    st = R.from_base(O, col)
    M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    M.color(seed=cseed)
    assert np.array_equal(M.export("color").astype(np.int64), col)
    for lvl in range(1, levels + 1):
        xyz = np.array([lf.xyz for lf in st.leaves])
        lev = np.array([lf.level for lf in st.leaves])
        flags = synth.refine_flags(xyz, lev, lvl - 1, radius=radius)
        st, ncl = R.refine(st, flags)
        M, ncl_c = M.refine(flags)
        assert ncl_c == ncl
    return st, M


def _compare(st, M):
    mesh, color, orient, levels = R.to_mesh(st)
    info = M.info()
    assert (info["n_elem"], info["n_face"]) == (mesh.K, mesh.E)
    assert info["max_level"] == levels.max()
    assert np.array_equal(M.export("elem_vert").reshape(-1, 3), mesh.elem_vert)
    assert np.array_equal(M.export("elem_xyz").reshape(-1, 3, 2), mesh.elem_xyz)
    assert np.array_equal(M.export("elem_level").astype(np.int64), levels)
    assert np.array_equal(M.export("face_elem").reshape(-1, 2), mesh.face_elem)
    assert np.array_equal(M.export("face_local").reshape(-1, 2), mesh.face_local)
    assert np.array_equal(M.export("color").astype(np.int64), color)
    assert np.array_equal(M.export("elem_face").reshape(mesh.K, -1), mesh.elem_face)
    assert np.allclose(M.export("face_normal").reshape(-1, 2), mesh.normal, atol=1e-15)
    assert np.allclose(M.export("face_measure"), mesh.measure, rtol=1e-14)
    new, order, off = make_layout(mesh, color, "paper")
    assert np.array_equal(M.export("elem_new"), new)
    assert np.array_equal(M.export("face_order"), order)
    assert np.array_equal(M.export("color_off"), off)
    code = M.export("dev_face_code").reshape(2, -1)
    E = mesh.E
    inter = mesh.face_elem[order, 1] >= 0
    assert np.array_equal(code[0], mesh.face_local[order, 0] * 4 + orient[order, 0])
    assert np.array_equal(code[1][inter], mesh.face_local[order, 1][inter] * 4 + orient[order, 1][inter])
    check_coloring(mesh, color, 6)
    return mesh, color


def test_refine_periodic_three_levels_bit_exact():
    m = synth.periodic_tri(24, jitter=0.0, seed=4)
    st, M = _run(m, 3, 0.15, 0)
    mesh, color = _compare(st, M)
    assert M.info()["n_colors"] == 6


def test_refine_delaunay_walls_bit_exact():
    m = synth.poisson_delaunay(1500, seed=7)
    st, M = _run(m, 2, 0.3, 3)
    _compare(st, M)


def test_refine_requires_colored_parent_and_triangles():
    m = synth.periodic_tri(6, seed=1)
    M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    with pytest.raises(dgc.DgcError) as e:
        M.refine(np.zeros(M.info()["n_elem"], dtype=np.uint8))
    assert e.value.name == "DGC_E_NOT_COLORED"
    t = synth.kuhn_tets(4)
    T = dgc.Mesh.build(t["elem_vert"], t["elem_xyz"])
    T.color(seed=0)
    with pytest.raises(dgc.DgcError) as e:
        T.refine(np.zeros(T.info()["n_elem"], dtype=np.uint8))
    assert e.value.name == "DGC_E_UNSUPPORTED"


def test_no_flags_gives_same_mesh():
    m = synth.periodic_tri(8, jitter=0.1, seed=2)
    M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    M.color(seed=1)
    M2, ncl = M.refine(np.zeros(M.info()["n_elem"], dtype=np.uint8))
    assert ncl == 0
    assert np.array_equal(M2.export("face_elem"), M.export("face_elem"))
    assert np.array_equal(M2.export("color"), M.export("color"))
