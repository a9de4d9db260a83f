"""Seeded per-element states and modal DOF arrays.

DOF arrays have shape ``[K, M, N_p]`` (element, conserved variable, mode).
For an orthonormal modal basis whose first function is constant, the
constant mode of a physical element with measure ``|Omega|`` is
``1 / sqrt(|Omega|)``; a state ``u`` therefore has first coefficient
``sqrt(|Omega|) u``.  Higher modes get seeded Gaussian perturbations of a
stated relative size, small enough to keep density and pressure positive.
"""

from __future__ import annotations

import numpy as np

GAMMA = 1.4


def _conservative(rho, vel, p, gamma=GAMMA):
    rho = np.asarray(rho, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    kin = 0.5 * rho * (vel ** 2).sum(axis=-1)
    cols = [rho] + [rho * vel[..., d] for d in range(vel.shape[-1])] + [p / (gamma - 1.0) + kin]
    return np.stack(cols, axis=-1)


def uniform_states(K: int, rho=1.0, vel=(0.3, -0.2), p=1.0, gamma=GAMMA):
    vel = np.broadcast_to(np.asarray(vel, dtype=np.float64), (K, len(vel)))
    return _conservative(np.full(K, rho), vel, np.full(K, p), gamma)


def shock_tube_states(centroids: np.ndarray, x0: float = 0.5, left=(1.0, 0.0, 0.0, 1.0),
                      right=(0.1, 0.0, 0.0, 0.1), gamma=GAMMA):
    """Density-ratio-10 shock tube: primitive ``(rho, u, v, p)`` left/right of ``x = x0``.

    Each element takes the state on the side of its centroid.
    """
    c = np.asarray(centroids, dtype=np.float64)
    isl = c[:, 0] < x0
    prim = np.where(isl[:, None], np.asarray(left)[None, :], np.asarray(right)[None, :])
    return _conservative(prim[:, 0], prim[:, 1:3], prim[:, 3], gamma)


def density_wave_states(centroids: np.ndarray, amp: float = 0.2, vel=(1.0, 1.0, 1.0), p=1.0,
                        gamma=GAMMA):
    """3D density wave ``rho = 1 + amp sin(2 pi (x + y + z))`` at uniform velocity and pressure."""
    c = np.asarray(centroids, dtype=np.float64)
    rho = 1.0 + amp * np.sin(2.0 * np.pi * c.sum(axis=1))
    K = c.shape[0]
    v = np.broadcast_to(np.asarray(vel, dtype=np.float64), (K, len(vel)))
    return _conservative(rho, v, np.full(K, p), gamma)


def perturbed_dofs(measure: np.ndarray, states: np.ndarray, n_p: int, eps: float = 0.01,
                   seed: int = 0) -> np.ndarray:
    """Modal DOFs ``[K, M, n_p]``: the state in mode 0, seeded noise in the others.

    ``c[:, m, 0] = sqrt(|Omega|) * state[:, m]`` and, for ``j >= 1``,
    ``c[:, m, j] = sqrt(|Omega|) * eps * (|state[:, m]| + 0.1) * N(0, 1)``.
    """
    meas = np.asarray(measure, dtype=np.float64)
    st = np.asarray(states, dtype=np.float64)
    K, M = st.shape
    rng = np.random.default_rng(seed)
    c = np.zeros((K, M, n_p), dtype=np.float64)
    sq = np.sqrt(meas)[:, None]
    c[:, :, 0] = sq * st
    if n_p > 1:
        noise = rng.standard_normal((K, M, n_p - 1))
        c[:, :, 1:] = sq[:, :, None] * eps * (np.abs(st)[:, :, None] + 0.1) * noise
    return c


def isentropic_vortex(points: np.ndarray, t: float = 0.0, center=(0.5, 0.5), beta: float = 5.0,
                      radius: float = 1.0 / 15.0, u_inf=(1.0, 1.0), period: float = 1.0,
                      gamma=GAMMA) -> np.ndarray:
    """Conservative state of the isentropic vortex advected by ``u_inf`` on a periodic square.

    With ``r`` the distance (in units of ``radius``) from the nearest periodic
    image of the moving center: ``du = beta/(2 pi) exp((1 - r^2)/2) (-dy, dx)/radius``,
    ``T = 1 - (gamma - 1) beta^2 / (8 gamma pi^2) exp(1 - r^2)``,
    ``rho = T^(1/(gamma-1))``, ``p = rho^gamma``.  The exact solution at time
    ``t`` is the translate of the initial state.
    """
    x = np.asarray(points, dtype=np.float64)
    cx = center[0] + u_inf[0] * t
    cy = center[1] + u_inf[1] * t
    dx = x[:, 0] - cx
    dy = x[:, 1] - cy
    dx = dx - period * np.round(dx / period)
    dy = dy - period * np.round(dy / period)
    r2 = (dx * dx + dy * dy) / (radius * radius)
    f = np.exp(0.5 * (1.0 - r2))
    du = beta / (2.0 * np.pi) * f * (-dy / radius)
    dv = beta / (2.0 * np.pi) * f * (dx / radius)
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * np.pi * np.pi) * f * f
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    vel = np.stack([u_inf[0] + du, u_inf[1] + dv], axis=1)
    return _conservative(rho, vel, p, gamma)
