"""Pins of the oracle quadrature rules against closed-form monomial integrals."""
import math

import numpy as np
import pytest

from oracle import quadrature as Q


@pytest.mark.parametrize("q", [1, 2, 3, 4, 5])
def test_gauss_legendre_01_exact(q):
    x, w = Q.gauss_legendre_01(q)
    assert np.all(np.diff(x) > 0) and x[0] > 0 and x[-1] < 1
    for k in range(2 * q):
        assert abs((w * x ** k).sum() - 1.0 / (k + 1)) < 1e-14
    # degree 2q is not integrated exactly
    assert abs((w * x ** (2 * q)).sum() - 1.0 / (2 * q + 1)) > 1e-8


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_triangle_rule_exact(n):
    x, w = Q.tri_volume_rule(n)
    assert abs(w.sum() - 0.5) < 1e-15
    for a in range(2 * n):
        for b in range(2 * n - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs((w * x[:, 0] ** a * x[:, 1] ** b).sum() - exact) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_tet_rule_exact(n):
    x, w = Q.tet_volume_rule(n)
    assert abs(w.sum() - 1.0 / 6.0) < 1e-15
    for a in range(2 * n):
        for b in range(2 * n - a):
            for c in range(2 * n - a - b):
                exact = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
                assert abs((w * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c).sum() - exact) < 1e-15


def test_tet_face_rule_degree_two():
    bary, w = Q.tet_face_rule_p1()
    assert abs(w.sum() - 1.0) < 1e-15
    # average over a triangle of l1^a l2^b l3^c = 2 a! b! c! / (a + b + c + 2)!
    for a in range(3):
        for b in range(3 - a):
            for c in range(3 - a - b):
                exact = 2.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 2)
                got = (w * bary[:, 0] ** a * bary[:, 1] ** b * bary[:, 2] ** c).sum()
                assert abs(got - exact) < 1e-15


@pytest.mark.parametrize("n", [3, 4])
def test_tet_face_rule_collapsed_barycentric(n):
    # the p >= 2 face rule: every barycentric monomial of degree <= 2n - 1 is
    # averaged exactly (closed form 2 a! b! c! / (a + b + c + 2)!), and the
    # same rule is exact when the face's vertices are listed in any order
    bary, w = Q.tri_face_rule_bary(n)
    assert bary.shape == (n * n, 3) and abs(w.sum() - 1.0) < 1e-15
    assert np.abs(bary.sum(axis=1) - 1.0).max() < 1e-15 and bary.min() > 0
    for perm in ([0, 1, 2], [2, 0, 1], [1, 0, 2]):
        B = bary[:, perm]
        for a in range(2 * n):
            for b in range(2 * n - a):
                for c in range(2 * n - a - b):
                    exact = 2.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(
                        a + b + c + 2)
                    got = (w * B[:, 0] ** a * B[:, 1] ** b * B[:, 2] ** c).sum()
                    assert abs(got - exact) < 1e-14
