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


def test_rusanov_between_two_rest_states_closed_form():
    """Rusanov flux (Eq. 2's numerical flux; reading: local Lax-Friedrichs)
    between the Sod states at rest, left (rho, p) = (1, 1), right
    (0.125, 0.1), n = (1, 0).  By hand: F(uL).n = (0, 1, 0, 0),
    F(uR).n = (0, 0.1, 0, 0), cL = sqrt(1.4) > cR = sqrt(1.12), so
    lambda = sqrt(1.4) and F* = (0.4375 lambda, 0.55, 0, 1.125 lambda).
    The dissipation term depends on lambda, so taking the smaller wave speed
    (0.463 for the mass flux) or dropping the factor 1/2 fails."""
    UL = np.array([1.0, 0.0, 0.0, 2.5])
    UR = np.array([0.125, 0.0, 0.0, 0.25])
    n = np.array([1.0, 0.0])
    want = np.array([0.517656981021216403724641225511, 0.55, 0.0, 1.33111795119741360957764886560])
    assert np.abs(euler.rusanov(UL, UR, n) - want).max() < 2e-15
    # the same pair seen from the other side: the larger speed is now on the right
    assert np.abs(euler.rusanov(UR, UL, -n) + want).max() < 2e-15


def test_wall_of_a_moving_state_closed_form():
    """A reflective wall carries no mass and no energy, for any state.  State
    (rho, u, v, p) = (1.2, 0.5, -0.3, 2.0), n = (0.6, 0.8): u.n = 0.06,
    c = sqrt(1.4 * 2 / 1.2).  With the mirror ghost state the Rusanov
    momentum flux is (p + rho un^2 + rho un (|un| + c)) n, worked out by hand
    below; a ghost that only removes the normal velocity (factor 1 instead of
    2) gives a mass flux of rho un / 2 = 0.036."""
    rho, u, v, p = 1.2, 0.5, -0.3, 2.0
    U = np.array([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])
    n = np.array([0.6, 0.8])
    F = euler.rusanov(U, euler.wall_ghost(U, n), n)
    assert abs(F[0]) < 1e-15 and abs(F[3]) < 1e-14
    assert abs(F[1] - 1.27117309000736409609486787959) < 2e-15
    assert abs(F[2] - 1.69489745334315212812649050612) < 2e-15
