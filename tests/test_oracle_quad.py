"""Pins of the oracle's quadrilateral family: the tensor rule, the tensor
Legendre basis, parallelogram meshes, four colors (the paper's Table 2), and
the DG operator (free stream, conservation, convergence)."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import basis, dg, quadrature as Q
from oracle.coloring import check_coloring, color_faces
from oracle.mesh import MeshError, build_mesh
from synth.fields import _conservative

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_square_rule_exact(n):
    x, w = Q.quad_volume_rule(n)
    assert abs(w.sum() - 1.0) < 1e-15
    for a in range(2 * n):
        for b in range(2 * n):
            assert abs((w * x[:, 0] ** a * x[:, 1] ** b).sum() - 1.0 / ((a + 1) * (b + 1))) < 1e-15
    # degree 2n in one variable is not integrated exactly
    assert abs((w * x[:, 0] ** (2 * n)).sum() - 1.0 / (2 * n + 1)) > 1e-8


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_tensor_basis_orthonormal(p):
    x, w = Q.quad_volume_rule(p + 2)
    B = basis.eval_basis_quad(p, x)
    assert B.shape[1] == (p + 1) ** 2
    assert np.abs(B.T @ (w[:, None] * B) - np.eye(B.shape[1])).max() < 1e-13


def test_tensor_basis_p1_closed_forms():
    rng = np.random.default_rng(2)
    X = rng.random((30, 2))
    B = basis.eval_basis_quad(1, X)
    s3 = math.sqrt(3.0)
    want = np.stack([np.ones(30), s3 * (2 * X[:, 0] - 1), s3 * (2 * X[:, 1] - 1),
                     3.0 * (2 * X[:, 0] - 1) * (2 * X[:, 1] - 1)], axis=1)
    assert np.abs(B - want).max() < 1e-14


@pytest.mark.parametrize("p", [1, 2, 3])
def test_tensor_basis_spans_Qp_and_gradients(p):
    # every mode is a polynomial of degree <= p in each variable: the fit in
    # the monomials x^a y^b (a, b <= p) on a (p+1)^2 lattice reproduces it at
    # random points; gradients agree with central differences
    g = np.linspace(0.1, 0.9, p + 1)
    L = np.array([(u, v) for v in g for u in g])
    exps = [(a, b) for b in range(p + 1) for a in range(p + 1)]
    V = np.stack([L[:, 0] ** a * L[:, 1] ** b for a, b in exps], axis=1)
    C = np.linalg.solve(V, basis.eval_basis_quad(p, L))
    rng = np.random.default_rng(p)
    X = rng.random((50, 2))
    W = np.stack([X[:, 0] ** a * X[:, 1] ** b for a, b in exps], axis=1)
    assert np.abs(W @ C - basis.eval_basis_quad(p, X)).max() < 1e-10
    G = basis.eval_grad_quad(p, X)
    h = 1e-6
    for d in range(2):
        e = np.zeros(2)
        e[d] = h
        fd = (basis.eval_basis_quad(p, X + e) - basis.eval_basis_quad(p, X - e)) / (2 * h)
        assert np.abs(G[:, d, :] - fd).max() < 1e-6


def test_parallelogram_meshes_and_four_colors():
    for periodic in (True, False):
        m = synth.quad_grid(10, seed=5, periodic=periodic)
        M = build_mesh(m["elem_vert"], m["elem_xyz"])
        assert M.kind == "quad" and M.K == 100
        assert abs(M.elem_measure.sum() - 1.0) < 1e-13
        assert M.E == (200 if periodic else 220)
        col, st = color_faces(M, seed=1)
        check_coloring(M, col, 4)
        # every element has one face of each color: 2 N_c^int + N_c^bnd = K
        inter = M.face_elem[:, 1] >= 0
        for c in range(4):
            assert 2 * (inter & (col == c)).sum() + (~inter & (col == c)).sum() == M.K
    bad = synth.quad_grid(4, seed=1)
    xyz = bad["elem_xyz"].copy()
    xyz[5, 2] += 0.01                      # no longer a parallelogram
    with pytest.raises(MeshError):
        build_mesh(bad["elem_vert"], xyz)


def test_golden_table2_transcription():
    """Checks the stored fixture of Table 2, not the oracle: the color counts
    add up to the sides, and 2 sides - 4 K (the boundary edges when every
    element has four edges of four colors) is positive and roughly doubles
    from mesh to mesh."""
    rows = GOLDEN["table2_quadrilaterals"]["rows"]
    bnd = []
    for r in rows:
        assert sum(r["colors"]) == r["sides"], r["mesh"]
        if r["mesh"] != "hybrid tri/quad":
            b = 2 * r["sides"] - 4 * r["elements"]
            assert b > 0
            for c in r["colors"]:
                assert 2 * c >= r["elements"] - b // 2      # one face of every color per element
            bnd.append(b)
    ratios = [bnd[i + 1] / bnd[i] for i in range(len(bnd) - 1)]
    assert all(1.9 < x < 2.1 for x in ratios), ratios


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_free_stream_and_rest_state_on_quads(p):
    M = build_mesh(**{k: v for k, v in synth.quad_grid(6, seed=2).items() if k in ("elem_vert", "elem_xyz")})
    d = dg.Discretization(M, p)
    U = synth.perturbed_dofs(M.elem_measure, synth.uniform_states(M.K, vel=(0.7, -0.4)), d.n_p, eps=0.0)
    assert np.abs(dg.rhs(d, U)).max() < 1e-13 * np.abs(dg.surface_abs(d, U)).max()
    W = synth.quad_grid(6, seed=2, periodic=False)
    Mw = build_mesh(W["elem_vert"], W["elem_xyz"])
    dw = dg.Discretization(Mw, p)
    U = synth.perturbed_dofs(Mw.elem_measure, synth.uniform_states(Mw.K, vel=(0.0, 0.0)), dw.n_p, eps=0.0)
    assert np.abs(dg.rhs(dw, U)).max() < 1e-13 * np.abs(dg.surface_abs(dw, U)).max()


def test_conservation_on_periodic_quads():
    M = build_mesh(**{k: v for k, v in synth.quad_grid(6, seed=3).items() if k in ("elem_vert", "elem_xyz")})
    d = dg.Discretization(M, 2)
    U = synth.perturbed_dofs(M.elem_measure, synth.uniform_states(M.K), d.n_p, eps=0.05, seed=4)
    r = dg.rhs(d, U)
    total = (r[:, :, 0] * np.sqrt(M.detJ)[:, None] * d.phi0).sum(axis=0)
    assert np.abs(total).max() < 1e-13 * np.abs(r).max() * M.K


def _wave(X, t):
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * (X[:, 0] + X[:, 1] - 2.0 * t))
    return _conservative(rho, np.tile([1.0, 1.0], (len(X), 1)), np.ones(len(X)))


@pytest.mark.parametrize("p", [1, 2])
def test_convergence_density_wave_on_parallelograms(p):
    errs = []
    T = 0.05
    for n in (8, 16, 32):
        g = synth.quad_grid(n, jitter=0.1, seed=7)
        M = build_mesh(g["elem_vert"], g["elem_xyz"])
        d = dg.Discretization(M, p)
        U = dg.project(d, lambda X: _wave(X, 0.0))
        dt = dg.cfl_dt(d, U, 0.1)
        nst = int(np.ceil(T / dt))
        for _ in range(nst):
            U = dg.rk3_step(d, U, T / nst)
        errs.append(dg.l2_error(d, U, lambda X: _wave(X, T), var=0))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[-1] >= p + 1 - 0.2, (rates, errs)
