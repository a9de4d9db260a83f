"""Pins of the oracle mesh build (counts, closure, measures, errors)."""
import numpy as np
import pytest

import synth
from oracle.mesh import MeshError, build_mesh


def _closure(M):
    acc = np.zeros((M.K, M.dim))
    w = M.normal * M.measure[:, None]
    np.add.at(acc, M.face_elem[:, 0], w)
    inter = M.face_elem[:, 1] >= 0
    np.add.at(acc, M.face_elem[inter, 1], -w[inter])
    return acc


def test_periodic_triangles_counts_and_closure():
    n = 12
    m = synth.periodic_tri(n, seed=4)
    M = build_mesh(m["elem_vert"], m["elem_xyz"])
    assert M.K == 2 * n * n
    assert M.E == 3 * M.K // 2 and M.n_boundary == 0
    # Euler characteristic of the torus: V - E + K = 0
    assert m["n_vert"] - M.E + M.K == 0
    assert abs(M.elem_measure.sum() - 1.0) < 1e-13
    assert np.abs(_closure(M)).max() < 1e-15
    assert np.allclose(np.linalg.norm(M.normal, axis=1), 1.0)
    # each element lists each of its faces once
    assert (np.sort(M.elem_face, axis=1)[:, 1:] != np.sort(M.elem_face, axis=1)[:, :-1]).all()


def test_periodic_tets_counts_and_closure():
    n = 4
    t = synth.kuhn_tets(n, seed=4)
    M = build_mesh(t["elem_vert"], t["elem_xyz"])
    assert M.K == 6 * n ** 3 and M.E == 2 * M.K and M.n_boundary == 0
    assert abs(M.elem_measure.sum() - 1.0) < 1e-13
    assert np.abs(_closure(M)).max() < 1e-15
    # on a periodic seam the right element's own coordinates give the same face
    # area as the left element's
    L, R = M.face_elem[:, 0], M.face_elem[:, 1]
    for f in range(0, M.E, 97):
        pos = [list(M.elem_vert[R[f]]).index(v) for v in M.face_vert[f]]
        P = M.elem_xyz[R[f], pos]
        area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
        assert abs(area - M.measure[f]) < 1e-14


def test_delaunay_walls():
    d = synth.poisson_delaunay(3000, seed=9)
    M = build_mesh(d["elem_vert"], d["elem_xyz"])
    assert abs(M.elem_measure.sum() - 1.0) < 1e-12
    # 2 E = 3 K + n_boundary on a triangulated disc
    assert 2 * M.E == 3 * M.K + M.n_boundary
    # boundary faces lie on the unit square and point outward
    b = M.face_elem[:, 1] < 0
    nb = M.normal[b]
    assert np.allclose(np.abs(nb).max(axis=1), 1.0)
    # total boundary length = perimeter
    assert abs(M.measure[b].sum() - 4.0) < 1e-12


def test_errors():
    m = synth.periodic_tri(4)
    ev, xyz = m["elem_vert"].copy(), m["elem_xyz"].copy()
    bad = xyz.copy()
    bad[0, [1, 2]] = bad[0, [2, 1]]
    with pytest.raises(MeshError):
        build_mesh(ev, bad)
    ev3 = np.concatenate([ev, ev[:1]])
    xyz3 = np.concatenate([xyz, xyz[:1]])
    with pytest.raises(MeshError):
        build_mesh(ev3, xyz3)
