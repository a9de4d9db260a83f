"""Pins of the oracle on mixed triangle / quadrilateral meshes (the hybrid
mesh of the paper's Table 2): mesh and coloring invariants, the padded mode
layout, free stream, conservation and convergence order p + 1 across the
triangle / quadrilateral interfaces."""
import math

import numpy as np
import pytest

import synth
from oracle import dg
from oracle.coloring import check_coloring, color_faces
from oracle.layout import make_layout
from oracle.mesh import build_mesh
from synth.fields import _conservative


def _mesh(n=10, seed=3, periodic=True):
    h = synth.hybrid_grid(n, seed=seed, periodic=periodic)
    return h, build_mesh(h["elem_vert"], h["elem_xyz"])


def test_mixed_mesh_counts_and_four_colors():
    for periodic in (True, False):
        h, M = _mesh(periodic=periodic)
        assert M.kind == "mixed" and (M.elem_kind == 0).sum() == h["n_tri"] and (M.elem_kind == 1).sum() == h["n_quad"]
        assert h["n_tri"] > 0 and h["n_quad"] > 0
        assert abs(M.elem_measure.sum() - 1.0) < 1e-13
        inter = M.face_elem[:, 1] >= 0
        assert 2 * inter.sum() + (~inter).sum() == 3 * h["n_tri"] + 4 * h["n_quad"]
        assert ((M.elem_face >= 0).sum(axis=1) == np.where(M.elem_kind == 1, 4, 3)).all()
        col, st = color_faces(M, seed=2)
        check_coloring(M, col, 4)
        # a color touches every quadrilateral once and every triangle at most once
        for c in range(4):
            touched = np.zeros(M.K, dtype=int)
            np.add.at(touched, M.face_elem[col == c, 0], 1)
            r = M.face_elem[col == c, 1]
            np.add.at(touched, r[r >= 0], 1)
            assert touched.max() == 1 and (touched[M.elem_kind == 1] == 1).all()
        new, order, off = make_layout(M, col, "paper")
        assert np.array_equal(np.sort(new), np.arange(M.K))


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_mixed_free_stream_and_padding(p):
    h, M = _mesh(8, seed=4)
    d = dg.Discretization(M, p)
    assert d.n_p == (p + 1) ** 2
    # the constant state: c_0 = sqrt(|Omega|) u on both kinds (v_0 = 1 / sqrt(|Omega|))
    U = synth.perturbed_dofs(M.elem_measure, synth.uniform_states(M.K, vel=(0.6, -0.3)), d.n_p, eps=0.0)
    r = dg.rhs(d, U)
    assert np.abs(r).max() < 1e-13 * np.abs(dg.surface_abs(d, U)).max()
    # the padded modes of triangles get no contribution
    ntri = (p + 1) * (p + 2) // 2
    if ntri == d.n_p:
        return
    V = synth.perturbed_dofs(M.elem_measure, synth.uniform_states(M.K), d.n_p, eps=0.005, seed=1)
    V[M.elem_kind == 0, :, ntri:] = 0.0
    assert np.abs(dg.rhs(d, V)[M.elem_kind == 0][:, :, ntri:]).max() == 0.0


def test_mixed_conservation():
    h, M = _mesh(8, seed=5)
    d = dg.Discretization(M, 2)
    U = synth.perturbed_dofs(M.elem_measure, synth.uniform_states(M.K), d.n_p, eps=0.01, seed=4)
    U[M.elem_kind == 0, :, 6:] = 0.0
    r = dg.rhs(d, U)
    # int v_0 = sqrt(|Omega|) on both kinds
    total = (r[:, :, 0] * np.sqrt(M.elem_measure)[:, None]).sum(axis=0)
    assert np.abs(total).max() < 1e-13 * np.abs(r).max() * M.K


def _wave(X, t):
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * (X[:, 0] + X[:, 1] - 2.0 * t))
    return _conservative(rho, np.tile([1.0, 1.0], (len(X), 1)), np.ones(len(X)))


@pytest.mark.parametrize("p", [1, 2])
def test_mixed_convergence_density_wave(p):
    errs = []
    T = 0.05
    for n in (8, 16, 32):
        h = synth.hybrid_grid(n, seed=7, radius=0.3)
        M = build_mesh(h["elem_vert"], h["elem_xyz"])
        d = dg.Discretization(M, p)
        U = dg.project(d, lambda X: _wave(X, 0.0))
        dt = dg.cfl_dt(d, U, 0.1)
        nst = int(np.ceil(T / dt))
        for _ in range(nst):
            U = dg.rk3_step(d, U, T / nst)
        errs.append(dg.l2_error(d, U, lambda X: _wave(X, T), var=0))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[-1] >= p + 1 - 0.2, (rates, errs)
