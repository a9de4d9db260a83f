"""Pins of the oracle DOF transfer between a triangle and its children."""
import numpy as np
import pytest

from oracle import basis, refine as R, transfer as T


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_children_tile_the_parent(p):
    # sum_k P_k^T P_k is the parent mass matrix, the identity for an
    # orthonormal basis: restriction undoes prolongation exactly
    P = T.prolongation(p)
    G = sum(P[k].T @ P[k] for k in range(4))
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3])
def test_prolongation_reproduces_the_parent_polynomial(p):
    rng = np.random.default_rng(p)
    c = rng.standard_normal(basis.n_modes(2, p))
    P = T.prolongation(p)
    xi = rng.random((40, 2))
    xi = xi[xi.sum(axis=1) < 1]
    for k in range(4):
        # physical values: parent sum_l c_l phi_l(x) / sqrt(J); child uses
        # det J_child = J / 4, hence the factor 2
        child = 2.0 * basis.eval_basis(2, p, xi) @ (P[k] @ c)
        parent = basis.eval_basis(2, p, T.child_map(k, xi)) @ c
        assert np.abs(child - parent).max() < 1e-12


def test_child_maps_tile_the_reference_triangle():
    areas = []
    for k in range(4):
        X = T.CHILD_VERTS[k]
        a = 0.5 * ((X[1, 0] - X[0, 0]) * (X[2, 1] - X[0, 1]) - (X[2, 0] - X[0, 0]) * (X[1, 1] - X[0, 1]))
        areas.append(a)
    assert np.allclose(areas, 0.125)     # four positively oriented quarters


def test_restriction_preserves_mass_of_discontinuous_data():
    rng = np.random.default_rng(7)
    p = 2
    kids = rng.standard_normal((4, 4, basis.n_modes(2, p)))          # [child, M, Np]
    origin = [(5, [0, 1, 2, 3])]
    par = T.transfer(p, kids, origin)[0]
    # int u = c_0 phi_0 sqrt(det J); children have det J / 4
    assert np.abs(par[:, 0] - 0.5 * kids[:, :, 0].sum(axis=0)).max() < 1e-13


def test_transfer_follows_refine_then_coarsen():
    st, _ = R.refine(R.RefineState([R.Leaf([0, 1, 2], np.array([[0.0, 0], [1, 0], [0, 1]]), 0,
                                          [R.Edge(0, 1, 0), R.Edge(1, 2, 1), R.Edge(2, 0, 2)])], 3), [True])
    assert st.origin == [(1, [0]), (2, [0]), (3, [0]), (4, [0])]
    rng = np.random.default_rng(1)
    U = rng.standard_normal((1, 4, 6))
    kids = T.transfer(2, U, st.origin)
    st2, _ = R.coarsen(st, [True] * 4)
    back = T.transfer(2, kids, st2.origin)
    assert np.abs(back - U).max() < 1e-13
