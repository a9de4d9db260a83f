"""Pins of the oracle Euler / Rusanov / wall functions."""
import math

import numpy as np

from oracle import euler


def _states(rng, n, dim):
    rho = rng.uniform(0.5, 2.0, n)
    vel = rng.uniform(-1, 1, (n, dim))
    p = rng.uniform(0.5, 2.0, n)
    E = p / 0.4 + 0.5 * rho * (vel ** 2).sum(1)
    return np.concatenate([rho[:, None], rho[:, None] * vel, E[:, None]], axis=1)


def _normals(rng, n, dim):
    v = rng.standard_normal((n, dim))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_consistency_and_conservation():
    rng = np.random.default_rng(0)
    for dim in (2, 3):
        a, b = _states(rng, 100, dim), _states(rng, 100, dim)
        n = _normals(rng, 100, dim)
        assert np.abs(euler.rusanov(a, a, n) - euler.normal_flux(a, n)).max() < 1e-14
        assert np.abs(euler.rusanov(a, b, n) + euler.rusanov(b, a, -n)).max() < 1e-13


def test_wall_at_rest_is_pressure_only():
    U = np.array([1.2, 0.0, 0.0, 2.5])
    n = np.array([0.6, 0.8])
    F = euler.rusanov(U, euler.wall_ghost(U, n), n)
    p = 0.4 * 2.5
    assert np.allclose(F, [0.0, p * 0.6, p * 0.8, 0.0], atol=1e-15)


def test_hand_computed_flux():
    # rho = 1, u = (1, 0), p = 1 -> E = 1/0.4 + 0.5 = 3; n = (1, 0)
    U = np.array([1.0, 1.0, 0.0, 3.0])
    n = np.array([1.0, 0.0])
    assert np.allclose(euler.normal_flux(U, n), [1.0, 2.0, 0.0, 4.0], atol=1e-15)
    assert abs(euler.sound_speed(U) - math.sqrt(1.4)) < 1e-15
