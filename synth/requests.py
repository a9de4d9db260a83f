"""Seeded request stream of the serving workload (inputs only).

256 independent 2D Euler solves arriving as a Poisson process: exponential
inter-arrival times with rate ``rate`` (per second); target element counts
log-uniform on ``[k_lo, k_hi]`` realised as periodic ``n x n x 2`` jittered
triangle meshes with ``n = round(sqrt(K / 2))``; order ``p`` uniform in
``{1, 2, 3}``; half isentropic vortices (center uniform in ``[0.25, 0.75]^2``,
strength ``beta`` uniform in ``[3, 5]``), half tanh-smoothed planar fronts
(width three cells, random normal direction, density and pressure ratio 2).
Initial DOFs are the state at each element's centroid in the constant mode.
"""

from __future__ import annotations

import math

import numpy as np

from .fields import GAMMA, _conservative, isentropic_vortex
from .meshes import element_centroid, element_measure, periodic_tri


def request_stream(n: int = 256, rate: float = 50.0, k_lo: float = 2e3, k_hi: float = 2e5, seed: int = 5,
                   steps: int = 100):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    out = []
    for i in range(n):
        K = math.exp(rng.uniform(math.log(k_lo), math.log(k_hi)))
        side = max(3, int(round(math.sqrt(K / 2.0))))
        p = int(rng.integers(1, 4))
        kind = "vortex" if rng.random() < 0.5 else "front"
        ic = {"kind": kind}
        if kind == "vortex":
            ic.update(center=(float(rng.uniform(0.25, 0.75)), float(rng.uniform(0.25, 0.75))),
                      beta=float(rng.uniform(3.0, 5.0)))
        else:
            ang = float(rng.uniform(0.0, 2.0 * math.pi))
            ic.update(normal=(math.cos(ang), math.sin(ang)), offset=float(rng.uniform(0.3, 0.7)))
        out.append({"rid": i, "arrival": float(t[i]), "n": side, "p": p, "ic": ic, "mesh_seed": int(1000 + i),
                    "steps": steps})
    return out


def front_state(points, normal, offset, width, gamma=GAMMA):
    """Planar front smoothed by tanh over ``width``: (rho, p) = (2, 2) behind, (1, 1) ahead, at rest."""
    x = np.asarray(points, dtype=np.float64)
    s = x[:, 0] * normal[0] + x[:, 1] * normal[1] - offset
    w = 0.5 * (1.0 - np.tanh(s / width))
    rho = 1.0 + w
    p = 1.0 + w
    vel = np.zeros((len(x), 2))
    return _conservative(rho, vel, p, gamma)


def request_dt(req, m=None, cfl: float = 0.1, gamma=GAMMA) -> float:
    """Time step supplied with a request: ``cfl * min(2 r_in) / max(|u| + c)``
    over the initial state at the element centroids (``r_in`` the inradius,
    ``c`` the sound speed of the ideal gas)."""
    if m is None:
        m, _ = request_input(req)
    xyz = m["elem_xyz"]
    st = _initial_states(req, element_centroid(xyz))
    rho = st[:, 0]
    vel = st[:, 1:3] / rho[:, None]
    pres = (gamma - 1.0) * (st[:, 3] - 0.5 * rho * (vel ** 2).sum(axis=1))
    smax = float((np.linalg.norm(vel, axis=1) + np.sqrt(gamma * pres / rho)).max())
    per = sum(np.linalg.norm(xyz[:, (k + 1) % 3] - xyz[:, k], axis=1) for k in range(3))
    two_rin = 4.0 * element_measure(xyz) / per
    return cfl * float(two_rin.min()) / smax


def _initial_states(req, cen):
    ic = req["ic"]
    if ic["kind"] == "vortex":
        return isentropic_vortex(cen, 0.0, center=ic["center"], beta=ic["beta"], radius=0.1)
    return front_state(cen, ic["normal"], ic["offset"], 3.0 / req["n"])


def request_input(req):
    """Mesh arrays and constant-mode initial DOFs ``[K, 4, N_p]`` of one request."""
    m = periodic_tri(req["n"], jitter=0.1, seed=req["mesh_seed"])
    cen = element_centroid(m["elem_xyz"])
    st = _initial_states(req, cen)
    p = req["p"]
    n_p = (p + 1) * (p + 2) // 2
    U = np.zeros((len(cen), 4, n_p))
    U[:, :, 0] = np.sqrt(element_measure(m["elem_xyz"]))[:, None] * st
    return m, U
