"""Pins of the oracle's orthonormal Dubiner basis."""
import math

import numpy as np
import pytest

from oracle import basis, quadrature as Q


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_triangle_orthonormal(p):
    x, w = Q.tri_volume_rule(p + 2)
    B = basis.eval_basis(2, p, x)
    assert B.shape[1] == (p + 1) * (p + 2) // 2
    G = B.T @ (w[:, None] * B)
    assert np.abs(G - np.eye(B.shape[1])).max() < 1e-13


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_tet_orthonormal(p):
    x, w = Q.tet_volume_rule(p + 2)
    B = basis.eval_basis(3, p, x)
    assert B.shape[1] == (p + 1) * (p + 2) * (p + 3) // 6
    G = B.T @ (w[:, None] * B)
    assert np.abs(G - np.eye(B.shape[1])).max() < 1e-13


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (2, 4), (2, 5), (3, 1), (3, 2)])
def test_span_is_polynomials_of_degree_p(dim, p):
    rng = np.random.default_rng(5)
    pts = rng.random((200, dim))
    pts = pts[pts.sum(axis=1) < 1.0]
    a = basis.eval_basis(dim, p, pts)
    b = basis.eval_basis_monomial(dim, p, pts)
    assert np.abs(a - b).max() < 1e-11


def test_p1_triangle_closed_forms():
    # hand-derived from the collapsed-coordinate definition
    rng = np.random.default_rng(1)
    pts = rng.random((50, 2))
    pts = pts[pts.sum(axis=1) < 1.0]
    xi, eta = pts[:, 0], pts[:, 1]
    B = basis.eval_basis(2, 1, pts)
    assert np.allclose(B[:, 0], math.sqrt(2.0), atol=1e-15)
    assert np.allclose(B[:, 1], 2.0 * math.sqrt(3.0) * (2.0 * xi + eta - 1.0), atol=1e-14)
    assert np.allclose(B[:, 2], 6.0 * eta - 2.0, atol=1e-14)


def test_tet_constant_mode():
    x, _ = Q.tet_volume_rule(2)
    assert np.allclose(basis.eval_basis(3, 0, x), math.sqrt(6.0), atol=1e-14)


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 3), (3, 1), (3, 2)])
def test_gradients_central_differences(dim, p):
    rng = np.random.default_rng(2)
    pts = rng.random((40, dim)) * 0.6 + 0.05
    pts = pts[pts.sum(axis=1) < 0.9]
    G = basis.eval_grad(dim, p, pts)
    h = 1e-6
    for d in range(dim):
        e = np.zeros(dim)
        e[d] = h
        fd = (basis.eval_basis(dim, p, pts + e) - basis.eval_basis(dim, p, pts - e)) / (2 * h)
        assert np.abs(fd - G[:, d, :]).max() < 1e-7
