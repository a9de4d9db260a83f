"""Pins of the oracle DG operator: free stream, conservation, the p = 0
finite-volume closed form, convergence order and the SSP-RK3 factor."""
import numpy as np
import pytest

import synth
from synth.fields import _conservative
from oracle import dg, euler
from oracle.mesh import build_mesh


def _tri(n=8, seed=1):
    m = synth.periodic_tri(n, seed=seed)
    return build_mesh(m["elem_vert"], m["elem_xyz"])


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_free_stream_triangles(p):
    M = _tri(6)
    d = dg.Discretization(M, p)
    U = synth.perturbed_dofs(M.elem_measure, synth.uniform_states(M.K, vel=(0.7, -0.4)), d.n_p, eps=0.0)
    scale = np.abs(dg.surface_abs(d, U)).max()
    assert np.abs(dg.rhs(d, U)).max() < 1e-13 * scale


@pytest.mark.parametrize("p", [0, 1, 2])
def test_free_stream_tets(p):
    t = synth.kuhn_tets(3)
    M = build_mesh(t["elem_vert"], t["elem_xyz"])
    d = dg.Discretization(M, p)
    U = synth.perturbed_dofs(M.elem_measure, synth.uniform_states(M.K, vel=(0.3, -0.2, 0.5)), d.n_p, eps=0.0)
    scale = np.abs(dg.surface_abs(d, U)).max()
    assert np.abs(dg.rhs(d, U)).max() < 1e-13 * scale


@pytest.mark.parametrize("p", [1, 2])
def test_conservation_periodic(p):
    M = _tri(6)
    d = dg.Discretization(M, p)
    U = synth.perturbed_dofs(M.elem_measure, synth.uniform_states(M.K), d.n_p, eps=0.05, seed=3)
    r = dg.rhs(d, U)
    # the mean of every conserved variable changes by sum_i c_i0 phi_0 sqrt(det J_i) ... = 0
    total = (r[:, :, 0] * np.sqrt(M.detJ)[:, None]).sum(axis=0)
    assert np.abs(total).max() < 1e-13 * np.abs(r).max() * M.K


def test_p0_surface_term_is_first_order_finite_volume():
    d0 = synth.poisson_delaunay(800, seed=11)
    M = build_mesh(d0["elem_vert"], d0["elem_xyz"])
    rng = np.random.default_rng(0)
    cen = synth.element_centroid(d0["elem_xyz"])
    st = synth.shock_tube_states(cen)
    st[:, 1:3] += 0.05 * st[:, :1] * rng.standard_normal((M.K, 2))
    # textbook FV: du_i/dt = -(1/|O_i|) sum_faces |f| F*(u_i, u_nb, n_out)
    fv = np.zeros_like(st)
    for f in range(M.E):
        L, R = M.face_elem[f]
        n = M.normal[f]
        uR = st[R] if R >= 0 else euler.wall_ghost(st[L], n)
        F = euler.rusanov(st[L], uR, n)
        fv[L] -= M.measure[f] * F / M.elem_measure[L]
        if R >= 0:
            fv[R] += M.measure[f] * F / M.elem_measure[R]
    d = dg.Discretization(M, 0)
    U = synth.perturbed_dofs(M.elem_measure, st, 1, eps=0.0)
    r = dg.surface_rhs(d, U)[:, :, 0] / np.sqrt(M.elem_measure)[:, None]
    assert np.abs(r - fv).max() < 1e-12 * np.abs(fv).max()


def test_sampled_rows_match_full():
    M = _tri(8)
    d = dg.Discretization(M, 2)
    U = synth.perturbed_dofs(M.elem_measure, synth.uniform_states(M.K), d.n_p, eps=0.05, seed=1)
    full = dg.surface_rhs(d, U)
    S = np.array([0, 5, 17, 100, M.K - 1])
    part = dg.surface_rhs(d, U, elems=S)
    assert np.array_equal(part[S], full[S])


def test_ssp_rk3_amplification():
    lam, dt = -2.0, 0.3
    z = lam * dt
    u = np.array([1.0, -2.0, 0.5])
    got = dg.ssp_rk3(lambda v: lam * v, u, dt)
    assert np.allclose(got, (1 + z + z * z / 2 + z ** 3 / 6) * u, rtol=1e-15, atol=0)


def test_ssp_rk3_nonlinear_step_closed_form():
    """One step of u' = u^2, u(0) = 1, dt = 0.1.  The Shu-Osher stages by hand:
    u1 = 1.1, u2 = 3/4 + (1.1 + 0.121)/4 = 1.05525,
    u3 = 1/3 + 2/3 (1.05525 + 0.1 * 1.05525^2) = 1.1110701708333...
    Every three-stage third-order method has the same linear amplification
    factor, so only a nonlinear right-hand side tells them apart: Kutta's
    classical RK3 gives 1.1110920041666..."""
    got = dg.ssp_rk3(lambda v: v * v, np.array([1.0]), 0.1)
    assert abs(got[0] - 1.11107017083333333333333333333) < 4e-16


def _wave(X, t):
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * (X[:, 0] + X[:, 1] - 2.0 * t))
    return _conservative(rho, np.tile([1.0, 1.0], (len(X), 1)), np.ones(len(X)))


def _rates(p, ns, T, init, exact, cfl=0.1):
    errs = []
    for n in ns:
        M = _tri(n)
        d = dg.Discretization(M, p)
        U = dg.project(d, init)
        dt = dg.cfl_dt(d, U, cfl)
        nst = int(np.ceil(T / dt))
        for _ in range(nst):
            U = dg.rk3_step(d, U, T / nst)
        errs.append(dg.l2_error(d, U, exact, var=0))
    return [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)], errs


@pytest.mark.parametrize("p", [1, 2])
def test_convergence_density_wave(p):
    rates, errs = _rates(p, [8, 16, 32], 0.05, lambda X: _wave(X, 0.0), lambda X: _wave(X, 0.05))
    assert rates[-1] >= p + 1 - 0.2, (rates, errs)


def test_convergence_isentropic_vortex_p1():
    R = 0.1
    rates, errs = _rates(1, [8, 16, 32], 0.05, lambda X: synth.isentropic_vortex(X, 0.0, radius=R),
                         lambda X: synth.isentropic_vortex(X, 0.05, radius=R))
    assert rates[-1] >= 1.8, (rates, errs)


@pytest.mark.parametrize("kind,p", [("tri", 1), ("tri", 3), ("quad", 1), ("quad", 3), ("mixed", 2), ("tet", 1),
                                    ("tet", 2)])
def test_face_points_coincide_from_both_sides(kind, p):
    # every face quadrature point, mapped through the left and through the right
    # element's affine map, lands on the same physical point (up to a whole
    # period on the torus): a wrong vertex order on either side fails this
    if kind == "tri":
        m = synth.periodic_tri(5, seed=4)
    elif kind == "quad":
        m = synth.quad_grid(5, seed=4)
    elif kind == "mixed":
        m = synth.hybrid_grid(8, seed=4)
    else:
        m = synth.kuhn_tets(4, seed=4)
    M = build_mesh(m["elem_vert"], m["elem_xyz"])
    d = dg.Discretization(M, p)
    inter = np.nonzero(M.face_elem[:, 1] >= 0)[0]
    xyz = M.elem_xyz
    phys = []
    for side in (0, 1):
        e = M.face_elem[inter, side]
        ref = np.einsum("qv,fvd->fqd", d.face_bary, M.face_ref[inter, side])
        if M.dim == 3:
            J = np.stack([xyz[e, a] - xyz[e, 0] for a in (1, 2, 3)], axis=2)   # columns = edge vectors
        else:
            quad = (M.elem_kind[e] == 1) if M.kind == "mixed" else np.full(len(e), M.kind == "quad")
            J = np.stack([xyz[e, 1] - xyz[e, 0], xyz[e, np.where(quad, 3, 2)] - xyz[e, 0]], axis=2)
        phys.append(xyz[e, 0][:, None, :] + np.einsum("fde,fqe->fqd", J, ref))
    diff = phys[0] - phys[1]
    assert np.abs(diff - np.round(diff)).max() < 1e-13
    # and the rule is not degenerate: distinct points on every face
    if d.face_bary.shape[0] > 1:
        assert np.abs(np.diff(phys[0], axis=1)).max(axis=2).min() > 1e-6
