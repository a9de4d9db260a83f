"""Quadrature rules (oracle).  TEST INFRASTRUCTURE ONLY.

The paper does not name its quadrature (its DG solver is only cited), so the
rules are the readings chosen for this project:

* edges: Gauss-Legendre with ``p + 1`` points on ``[0, 1]`` (weights sum to 1);
* triangle volume: collapsed (conical) product of Gauss-Legendre in the first
  collapsed coordinate and Gauss-Jacobi ``(1, 0)`` in the second, ``n`` points
  each, exact for total degree ``2 n - 1``;
* tetrahedron volume: collapsed product Gauss-Legendre x Gauss-Jacobi (1, 0)
  x Gauss-Jacobi (2, 0), ``n`` points each;
* unit square (quadrilaterals): tensor Gauss-Legendre with ``n`` points per
  direction (weights sum to 1); quadrilateral edges use the edge rule;
* tetrahedron faces at ``p <= 1``: the symmetric three-point rule with
  barycentric points ``(2/3, 1/6, 1/6)`` and permutations, weight 1/3 each
  (exact for degree 2; weights sum to 1);
* tetrahedron faces at ``p >= 2``: the collapsed triangle rule above with
  ``n = p + 1`` points per direction, written in barycentric coordinates of
  the face's vertices (exact for degree ``2 p + 1``; weights sum to 1).  The
  rule is not symmetric, so each side of a face places its points through the
  face's vertex order as seen from the left element.

Pins: monomial exactness against ``a! b! / (a + b + 2)!`` (unit triangle),
``a! b! c! / (a + b + c + 3)!`` (unit tetrahedron) and ``1 / (k + 1)`` on
``[0, 1]`` -- see ``tests/test_oracle_quadrature.py``.
"""

from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi


def gauss_legendre_01(q: int):
    """``q`` Gauss-Legendre points on ``[0, 1]`` in ascending order, weights summing to 1."""
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_jacobi(n: int, alpha: float, beta: float):
    """Gauss-Jacobi nodes/weights on ``[-1, 1]`` for the weight ``(1-x)^alpha (1+x)^beta``."""
    x, w = roots_jacobi(n, alpha, beta)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def tri_volume_rule(n: int):
    """Collapsed rule on the unit triangle ``(0,0),(1,0),(0,1)``.

    Returns points ``[n*n, 2]`` in ``(xi, eta)`` and weights summing to 1/2.
    The collapsed coordinates are ``a`` (Gauss-Legendre) and ``b``
    (Gauss-Jacobi (1, 0), absorbing the Jacobian factor ``(1 - b) / 2``).
    """
    a, wa = gauss_jacobi(n, 0.0, 0.0)
    b, wb = gauss_jacobi(n, 1.0, 0.0)
    pts = []
    wts = []
    for i in range(n):
        for k in range(n):
            r = 0.5 * (1.0 + a[i]) * (1.0 - b[k]) - 1.0
            s = b[k]
            pts.append((0.5 * (1.0 + r), 0.5 * (1.0 + s)))
            # biunit area element: dr ds = (1 - b)/2 da db; unit triangle: 1/4 of that
            wts.append(wa[i] * wb[k] / 8.0)
    return np.array(pts), np.array(wts)


def tet_volume_rule(n: int):
    """Collapsed rule on the unit tetrahedron; weights sum to 1/6."""
    a, wa = gauss_jacobi(n, 0.0, 0.0)
    b, wb = gauss_jacobi(n, 1.0, 0.0)
    c, wc = gauss_jacobi(n, 2.0, 0.0)
    pts = []
    wts = []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                r = 0.25 * (1.0 + a[i]) * (1.0 - b[j]) * (1.0 - c[k]) - 1.0
                s = 0.5 * (1.0 + b[j]) * (1.0 - c[k]) - 1.0
                t = c[k]
                pts.append((0.5 * (1.0 + r), 0.5 * (1.0 + s), 0.5 * (1.0 + t)))
                # biunit: dr ds dt = (1-b)/2 ((1-c)/2)^2 da db dc -> w/8; unit: another 1/8
                wts.append(wa[i] * wb[j] * wc[k] / 64.0)
    return np.array(pts), np.array(wts)


def tet_face_rule_p1():
    """Barycentric points ``[3, 3]`` and weights ``[3]`` of the symmetric three-point triangle rule."""
    bary = np.full((3, 3), 1.0 / 6.0)
    for q in range(3):
        bary[q, q] = 2.0 / 3.0
    return bary, np.full(3, 1.0 / 3.0)


def tri_face_rule_bary(n: int):
    """Collapsed rule of :func:`tri_volume_rule` as barycentric points ``[n*n, 3]``
    ``(1 - xi - eta, xi, eta)`` on a face triangle, weights ``[n*n]`` summing to 1."""
    pts, w = tri_volume_rule(n)
    bary = np.stack([1.0 - pts[:, 0] - pts[:, 1], pts[:, 0], pts[:, 1]], axis=1)
    return bary, 2.0 * w


def quad_volume_rule(n: int):
    """Tensor Gauss-Legendre rule on the unit square: points ``[n*n, 2]`` with
    the first coordinate running fastest, weights summing to 1 (exact for
    degree ``2 n - 1`` in each variable)."""
    x, w = gauss_legendre_01(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    WX, WY = np.meshgrid(w, w, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1), (WX * WY).ravel()
