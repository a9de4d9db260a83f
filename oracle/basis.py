"""Orthonormal modal bases (oracle): Dubiner on the unit triangle and
tetrahedron, tensor Legendre on the unit square.

TEST INFRASTRUCTURE ONLY.

Eq. (2) of the paper expands the solution on element ``i`` in ``N_p``
orthonormal basis functions ``v_ij``; the family is not named there.  The
reading used here: on the unit reference element the functions are the
Dubiner polynomials, built in collapsed coordinates from Jacobi polynomials
``P_n^(alpha, beta)`` (positive at ``x = 1``) normalised so that
``int phi_j phi_k = delta_jk`` on the unit element; on a physical element
``v_ij = phi_j / sqrt(det J_i)``, which makes the mass matrix the identity.

Mode order: total degree ascending; within a degree ``d`` the triangle modes
run ``(d,0), (d-1,1), ..., (0,d)`` (second index ascending), the tetrahedron
modes run over ``k`` ascending, then ``j`` ascending, with ``i = d - j - k``.

Gradients are obtained without the collapsed-coordinate chain rule: each
basis function is interpolated exactly in the monomial basis on the
equispaced lattice (unisolvent for degree ``p``), and the monomials are
differentiated term by term.

Pins (``tests/test_oracle_basis.py``): Gram matrix equal to the identity
under an exact rule; every basis function lies in ``P_p`` (lattice
interpolant reproduces it at random points); the hand-derived ``p = 1``
triangle modes ``sqrt(2)``, ``2 sqrt(3) (2 xi + eta - 1)``, ``6 eta - 2``;
gradients against central differences.
"""

from __future__ import annotations

import math

import numpy as np


def jacobi(n: int, alpha: float, beta: float, x):
    """Jacobi polynomial ``P_n^(alpha,beta)(x)`` by the three-term recurrence (DLMF 18.9.1)."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0
    p1 = 0.5 * ((alpha + beta + 2.0) * x + (alpha - beta))
    for k in range(1, n):
        c = 2.0 * k + alpha + beta
        a1 = 2.0 * (k + 1) * (k + alpha + beta + 1) * c
        a2 = (c + 1.0) * (alpha * alpha - beta * beta)
        a3 = c * (c + 1.0) * (c + 2.0)
        a4 = 2.0 * (k + alpha) * (k + beta) * (c + 2.0)
        p0, p1 = p1, ((a2 + a3 * x) * p1 - a4 * p0) / a1
    return p1


def jacobi_norm2(n: int, alpha: float, beta: float) -> float:
    """``int_{-1}^{1} (1-x)^alpha (1+x)^beta P_n^2 dx``."""
    return (2.0 ** (alpha + beta + 1.0) / (2 * n + alpha + beta + 1.0)
            * math.gamma(n + alpha + 1.0) * math.gamma(n + beta + 1.0)
            / (math.gamma(n + alpha + beta + 1.0) * math.factorial(n)))


def _pn(n, alpha, beta, x):
    return jacobi(n, alpha, beta, x) / math.sqrt(jacobi_norm2(n, alpha, beta))


def n_modes(dim: int, p: int) -> int:
    return (p + 1) * (p + 2) // 2 if dim == 2 else (p + 1) * (p + 2) * (p + 3) // 6


def mode_list(dim: int, p: int):
    out = []
    for d in range(p + 1):
        if dim == 2:
            for j in range(d + 1):
                out.append((d - j, j))
        else:
            for k in range(d + 1):
                for j in range(d - k + 1):
                    out.append((d - j - k, j, k))
    return out


def eval_basis(dim: int, p: int, pts) -> np.ndarray:
    """Values ``[n_pts, N_p]`` of the unit-element basis at reference points ``[n_pts, dim]``."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    modes = mode_list(dim, p)
    out = np.empty((pts.shape[0], len(modes)))
    if dim == 2:
        r = 2.0 * pts[:, 0] - 1.0
        s = 2.0 * pts[:, 1] - 1.0
        den = 1.0 - s
        safe = np.abs(den) > 1e-15
        a = np.where(safe, 2.0 * (1.0 + r) / np.where(safe, den, 1.0) - 1.0, -1.0)
        b = s
        for m, (i, j) in enumerate(modes):
            # orthonormal on the biunit triangle, times 2 for the unit triangle
            out[:, m] = 2.0 * math.sqrt(2.0) * _pn(i, 0, 0, a) * _pn(j, 2 * i + 1, 0, b) * (1.0 - b) ** i
        return out
    r = 2.0 * pts[:, 0] - 1.0
    s = 2.0 * pts[:, 1] - 1.0
    t = 2.0 * pts[:, 2] - 1.0
    dst = -(s + t)
    safe1 = np.abs(dst) > 1e-15
    a = np.where(safe1, 2.0 * (1.0 + r) / np.where(safe1, dst, 1.0) - 1.0, -1.0)
    dt = 1.0 - t
    safe2 = np.abs(dt) > 1e-15
    b = np.where(safe2, 2.0 * (1.0 + s) / np.where(safe2, dt, 1.0) - 1.0, -1.0)
    c = t
    for m, (i, j, k) in enumerate(modes):
        # orthonormal on the biunit tetrahedron, times sqrt(8) for the unit one
        out[:, m] = (math.sqrt(8.0) * 2.0 * math.sqrt(2.0)
                     * _pn(i, 0, 0, a) * _pn(j, 2 * i + 1, 0, b) * (1.0 - b) ** i
                     * _pn(k, 2 * i + 2 * j + 2, 0, c) * (1.0 - c) ** (i + j))
    return out


def lattice(dim: int, p: int) -> np.ndarray:
    """Equispaced lattice of the unit element (``N_p`` points, unisolvent for degree ``p``)."""
    if p == 0:
        return np.full((1, dim), 1.0 / (dim + 1))
    pts = []
    if dim == 2:
        for j in range(p + 1):
            for i in range(p + 1 - j):
                pts.append((i / p, j / p))
    else:
        for k in range(p + 1):
            for j in range(p + 1 - k):
                for i in range(p + 1 - j - k):
                    pts.append((i / p, j / p, k / p))
    return np.array(pts, dtype=np.float64)


def monomial_exponents(dim: int, p: int):
    if dim == 2:
        return [(a, b) for a in range(p + 1) for b in range(p + 1 - a)]
    return [(a, b, c) for a in range(p + 1) for b in range(p + 1 - a) for c in range(p + 1 - a - b)]


def _monomials(exps, pts):
    pts = np.atleast_2d(pts)
    V = np.ones((pts.shape[0], len(exps)))
    for m, e in enumerate(exps):
        for d, k in enumerate(e):
            V[:, m] *= pts[:, d] ** k
    return V


def monomial_coefficients(dim: int, p: int) -> np.ndarray:
    """Coefficients ``[n_monomials, N_p]`` of each basis function in the monomials."""
    exps = monomial_exponents(dim, p)
    X = lattice(dim, p)
    V = _monomials(exps, X)
    return np.linalg.solve(V, eval_basis(dim, p, X))


def eval_basis_monomial(dim: int, p: int, pts) -> np.ndarray:
    """Values of the basis via its monomial interpolant (used for the span check)."""
    exps = monomial_exponents(dim, p)
    return _monomials(exps, np.asarray(pts, dtype=np.float64)) @ monomial_coefficients(dim, p)


def eval_grad(dim: int, p: int, pts) -> np.ndarray:
    """Reference gradients ``[n_pts, dim, N_p]`` (d/dxi, d/deta[, d/dzeta])."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    exps = monomial_exponents(dim, p)
    C = monomial_coefficients(dim, p)
    out = np.zeros((pts.shape[0], dim, C.shape[1]))
    for m, e in enumerate(exps):
        for d in range(dim):
            if e[d] == 0:
                continue
            term = np.full(pts.shape[0], float(e[d]))
            for dd, k in enumerate(e):
                kk = k - 1 if dd == d else k
                term = term * pts[:, dd] ** kk
            out[:, d, :] += term[:, None] * C[m][None, :]
    return out


# reference vertices of the unit elements
REF_VERTS = {
    2: np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]),
    3: np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]),
    "tri": np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]),
    "tet": np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]),
    "quad": np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]]),
}


# -- quadrilaterals ---------------------------------------------------------
# The unit square (0,0), (1,0), (1,1), (0,1) with the tensor-product basis
# phi_(a,b)(xi, eta) = L_a(xi) L_b(eta), 0 <= a, b <= p, where
# L_n(x) = sqrt(2n + 1) P_n(2x - 1) is the Legendre polynomial normalised on
# [0, 1]; N_p = (p + 1)^2, mode index j = b (p + 1) + a.  (The paper names no
# quadrilateral basis; this orthonormal family makes the mass matrix of an
# affine quadrilateral the identity, as the Dubiner basis does on simplices.)

def quad_modes(p: int):
    return [(a, b) for b in range(p + 1) for a in range(p + 1)]


def _leg01(n: int, x):
    return math.sqrt(2 * n + 1) * jacobi(n, 0.0, 0.0, 2.0 * np.asarray(x, dtype=np.float64) - 1.0)


def _dleg01(n: int, x):
    """d/dx of ``_leg01``: (d/dt) P_n(t) = (n + 1)/2 P_{n-1}^(1,1)(t) with t = 2x - 1."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.zeros_like(x)
    return math.sqrt(2 * n + 1) * (n + 1) * jacobi(n - 1, 1.0, 1.0, 2.0 * x - 1.0)


def eval_basis_quad(p: int, pts) -> np.ndarray:
    """Values ``[n_pts, (p+1)^2]`` of the tensor Legendre basis on the unit square."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    return np.stack([_leg01(a, pts[:, 0]) * _leg01(b, pts[:, 1]) for a, b in quad_modes(p)], axis=1)


def eval_grad_quad(p: int, pts) -> np.ndarray:
    """Reference gradients ``[n_pts, 2, (p+1)^2]``."""
    pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
    gx = [_dleg01(a, pts[:, 0]) * _leg01(b, pts[:, 1]) for a, b in quad_modes(p)]
    gy = [_leg01(a, pts[:, 0]) * _dleg01(b, pts[:, 1]) for a, b in quad_modes(p)]
    return np.stack([np.stack(gx, axis=1), np.stack(gy, axis=1)], axis=1)


def elem_n_modes(kind: str, p: int) -> int:
    return (p + 1) ** 2 if kind == "quad" else n_modes(2 if kind == "tri" else 3, p)


def elem_basis(kind: str, p: int, pts) -> np.ndarray:
    return eval_basis_quad(p, pts) if kind == "quad" else eval_basis(2 if kind == "tri" else 3, p, pts)


def elem_grad(kind: str, p: int, pts) -> np.ndarray:
    return eval_grad_quad(p, pts) if kind == "quad" else eval_grad(2 if kind == "tri" else 3, p, pts)
