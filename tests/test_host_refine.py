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


def test_refine_configured_size_bit_exact():
    """The refined workload at its configured size (128 x 128 x 2 base, three
    passes within 0.15 of the center): 178,724 leaves, bit-exact."""
    m = synth.periodic_tri(128, jitter=0.0, seed=4)
    st, M = _run(m, 3, 0.15, 0)
    mesh, color = _compare(st, M)
    assert mesh.K == 178_724 and M.info()["n_colors"] == 6


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


def _origin_arrays(origin):
    kind = np.array([k for k, _ in origin], dtype=np.int64)
    src = np.full((len(origin), 4), -1, dtype=np.int64)
    for i, (_, s) in enumerate(origin):
        src[i, :len(s)] = s
    return kind, src


def _check_origin(st, M, prev_new):
    kind, src = _origin_arrays(st.origin)
    assert np.array_equal(M.export("adapt_kind").astype(np.int64), kind)
    assert np.array_equal(M.export("adapt_src").reshape(-1, 4), src)
    # device form: rows in layout order, sources as layout ids of the previous mesh
    new = M.export("elem_new")
    dk = M.export("dev_adapt_kind").astype(np.int64)
    ds = M.export("dev_adapt_src").reshape(4, -1)
    assert np.array_equal(dk[new], kind)
    want = np.where(src >= 0, prev_new[np.maximum(src, 0)], -1)
    assert np.array_equal(ds[:, new].T, want)


def test_moving_feature_refine_and_coarsen_bit_exact():
    """Several adapt cycles around a moving center (coarsen, then refine one
    level), native against the oracle: leaves, vertex ids, face table, colors,
    layout and the origin of every leaf."""
    m = synth.periodic_tri(16, jitter=0.0, seed=4)
    O = build_mesh(m["elem_vert"], m["elem_xyz"])
    col, _ = color_faces(O, seed=0)
    st = R.from_base(O, col)
    M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    M.color(seed=0)
    merged_total = 0
    for cyc in range(6):
        center = (0.3 + 0.08 * cyc, 0.35 + 0.05 * cyc)
        xyz = np.array([lf.xyz for lf in st.leaves])
        lev = np.array([lf.level for lf in st.leaves])
        _, coarse = synth.adapt_flags(xyz, lev, center, 0.12, 0.16, max_level=2)
        prev_new = M.export("elem_new")
        st, n = R.coarsen(st, coarse)
        M, n_c = M.coarsen(coarse)
        assert n_c == n
        merged_total += n
        _compare(st, M)
        _check_origin(st, M, prev_new)
        assert R.check_balance(st)
        xyz = np.array([lf.xyz for lf in st.leaves])
        lev = np.array([lf.level for lf in st.leaves])
        fine, _ = synth.adapt_flags(xyz, lev, center, 0.12, 0.16, max_level=2)
        prev_new = M.export("elem_new")
        st, ncl = R.refine(st, fine)
        M, ncl_c = M.refine(fine)
        assert ncl_c == ncl
        _compare(st, M)
        _check_origin(st, M, prev_new)
    assert merged_total > 0 and M.info()["max_level"] == 2


def test_coarsen_all_the_way_back_to_the_base_coloring():
    m = synth.periodic_tri(24, jitter=0.0, seed=4)
    st, M = _run(m, 3, 0.15, 0)
    O = build_mesh(m["elem_vert"], m["elem_xyz"])
    col, _ = color_faces(O, seed=0)
    base = R.to_mesh(R.from_base(O, col))
    for _ in range(3):
        K = M.info()["n_elem"]
        st, n = R.coarsen(st, np.ones(K, dtype=bool))
        M, n_c = M.coarsen(np.ones(K, dtype=np.uint8))
        assert n_c == n > 0
    _compare(st, M)
    assert M.info()["max_level"] == 0 and M.info()["n_colors"] == 3
    assert np.array_equal(M.export("color").astype(np.int64), base[1])
    assert np.array_equal(M.export("face_elem").reshape(-1, 2), base[0].face_elem)


@pytest.mark.parametrize("mode", ["paired", "paper_sfc", "renumber", "none"])
def test_refined_mesh_other_layouts_bit_exact(mode):
    """A refined mesh (six colors, elements missing colors) laid out again in
    every other mode: the library's numbering and face order equal the
    oracle's."""
    m = synth.periodic_tri(24, jitter=0.0, seed=4)
    st, M = _run(m, 3, 0.15, 0)
    mesh, color = _compare(st, M)
    M.set_colors(color.astype(np.int8), layout=mode)
    new, order, off = make_layout(mesh, color, mode)
    assert np.array_equal(M.export("elem_new"), new)
    assert np.array_equal(M.export("face_order"), order)
    assert np.array_equal(M.export("color_off"), off)
