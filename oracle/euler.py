"""Compressible Euler flux, Rusanov numerical flux and reflective wall (oracle).

TEST INFRASTRUCTURE ONLY.

The paper's conservation law (Eq. 1) is written for a general flux; its
experiments solve the Euler equations.  The numerical flux and boundary
treatment of its solver are not given (its DG reference is not included), so
the readings here are: ideal gas with ``gamma = 1.4``; conserved variables
``(rho, rho u[, rho v[, rho w]], E)``; the Rusanov (local Lax-Friedrichs)
flux ``F* = (F(uL).n + F(uR).n)/2 - lambda (uR - uL)/2`` with
``lambda = max(|uL.n| + cL, |uR.n| + cR)``, ``c = sqrt(gamma p / rho)``; a
reflective wall uses the mirror ghost state ``(rho, rho u - 2 (rho u . n) n, E)``.

Pins (``tests/test_oracle_euler.py``): consistency ``F*(u, u, n) = F(u).n``;
conservation ``F*(uL, uR, n) = -F*(uR, uL, -n)``; the wall flux of a state
at rest is the pure pressure term ``(0, p n, 0)``; a hand-computed flux value.
"""

from __future__ import annotations

import numpy as np

GAMMA = 1.4


def pressure(U, gamma=GAMMA):
    rho = U[..., 0]
    mom = U[..., 1:-1]
    return (gamma - 1.0) * (U[..., -1] - 0.5 * (mom ** 2).sum(axis=-1) / rho)


def normal_flux(U, n, gamma=GAMMA):
    """``F(U) . n`` for states ``[..., M]`` and unit normals ``[..., dim]``."""
    rho = U[..., 0]
    mom = U[..., 1:-1]
    E = U[..., -1]
    vel = mom / rho[..., None]
    p = pressure(U, gamma)
    un = (vel * n).sum(axis=-1)
    out = np.empty(np.broadcast_shapes(U.shape, n.shape[:-1] + (U.shape[-1],)))
    out[..., 0] = rho * un
    out[..., 1:-1] = mom * un[..., None] + p[..., None] * n
    out[..., -1] = (E + p) * un
    return out


def physical_flux(U, gamma=GAMMA):
    """``F(U)`` as ``[..., M, dim]`` (column ``d`` is the flux in direction ``d``)."""
    dim = U.shape[-1] - 2
    cols = []
    for d in range(dim):
        n = np.zeros(dim)
        n[d] = 1.0
        cols.append(normal_flux(U, np.broadcast_to(n, U.shape[:-1] + (dim,)), gamma))
    return np.stack(cols, axis=-1)


def sound_speed(U, gamma=GAMMA):
    return np.sqrt(gamma * pressure(U, gamma) / U[..., 0])


def rusanov(UL, UR, n, gamma=GAMMA):
    fl = normal_flux(UL, n, gamma)
    fr = normal_flux(UR, n, gamma)
    unl = (UL[..., 1:-1] / UL[..., :1] * n).sum(axis=-1)
    unr = (UR[..., 1:-1] / UR[..., :1] * n).sum(axis=-1)
    lam = np.maximum(np.abs(unl) + sound_speed(UL, gamma), np.abs(unr) + sound_speed(UR, gamma))
    return 0.5 * (fl + fr) - 0.5 * lam[..., None] * (UR - UL)


def wall_ghost(U, n):
    """Mirror state across a reflective wall with unit normal ``n``."""
    G = np.array(U, dtype=np.float64, copy=True)
    mn = (U[..., 1:-1] * n).sum(axis=-1)
    G[..., 1:-1] = U[..., 1:-1] - 2.0 * mn[..., None] * n
    return G
