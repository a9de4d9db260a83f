"""DG right-hand side of Eq. (2) and SSP-RK3 time stepping (oracle).

TEST INFRASTRUCTURE ONLY.

Eq. (2) of the paper: for element ``i`` and basis function ``v_ij``,

    d c_ij / dt = int_{Omega_i} F(U_i) . grad v_ij
                  - sum_q int_{I_iq} v_ij F*(U_i, U_pq) . n_iq,

with ``v_ij = phi_j / sqrt(det J_i)`` orthonormal on the physical element.

* :func:`volume_rhs` -- the first (element-local) term, evaluated with the
  collapsed volume rule of :mod:`oracle.quadrature` (``n = p + 1`` points per
  direction):  ``rhs_ij = sqrt(det J) sum_q w_q sum_d d_d phi_j(xi_q) G_d(U_q)``
  with the contravariant flux ``G_d = sum_e (J^-1)_{de} F_e``.
* :func:`surface_rhs` -- the second term as a *plain loop over faces in id
  order*, each face adding ``-|f| sum_q w_q v_Lj F*_q`` to its left element
  and ``+|f| sum_q w_q v_Rj F*_q`` to its right element (``F*_q`` taken along
  the L-to-R normal; the right element's outward normal is ``-n`` and the
  Rusanov flux is conservative).  This is the order-dependent "race" form
  that the paper's coloring makes safe on a GPU; its result does not
  depend on any coloring or layout.
* :func:`rk3_step` -- three-stage SSP Runge-Kutta in Shu-Osher form (the
  time integrator is not named in the paper; this is the project's reading).

Pins (``tests/test_oracle_dg.py``): free-stream preservation on periodic
triangle and tetrahedral meshes; discrete conservation of the mode-0 mass;
the ``p = 0`` surface term equals the first-order finite-volume Rusanov
update ``-(1/|Omega|) sum |f| F* . n`` (times ``sqrt(|Omega|)``); order
``p + 1`` convergence on the isentropic vortex; the SSP-RK3 amplification
factor ``1 + z + z^2/2 + z^3/6`` on a linear problem.
"""

from __future__ import annotations

import numpy as np

from . import basis, euler, quadrature


class Discretization:
    """Quadrature, basis values and per-face reference points for one mesh and order.

    A mixed triangle / quadrilateral mesh stores every element's DOFs in
    ``N_p = (p + 1)^2`` slots (the quadrilateral count); a triangle uses the
    first ``(p + 1)(p + 2)/2`` and its other slots stay zero: its tables are
    zero beyond its own modes."""

    def __init__(self, mesh, p: int):
        self.mesh = mesh
        self.p = p
        self.dim = mesh.dim
        self.kind = mesh.kind
        self.kinds = ["tri", "quad"] if self.kind == "mixed" else [self.kind]
        self.elem_kind = (mesh.elem_kind if self.kind == "mixed" else np.zeros(mesh.K, dtype=np.int64))
        self.n_p = max(basis.elem_n_modes(k, p) for k in self.kinds)
        self.M = self.dim + 2
        if self.dim == 2:
            s, w = quadrature.gauss_legendre_01(p + 1)
            self.face_bary = np.stack([1.0 - s, s], axis=1)
            self.face_w = w
        elif p <= 1:
            self.face_bary, self.face_w = quadrature.tet_face_rule_p1()
        else:
            self.face_bary, self.face_w = quadrature.tri_face_rule_bary(p + 1)
        # volume rule and tables of every element kind (padded to n_p modes)
        self.vol = []
        for k in self.kinds:
            pts, w = _fine_rule(k, p + 1)
            B = self._pad(basis.elem_basis(k, p, pts))
            D = self._pad(basis.elem_grad(k, p, pts))
            self.vol.append((pts, w, B, D))
        self.phi_0 = np.array([float(basis.elem_basis(k, 0, self.vol[i][0][:1])[0, 0])
                               for i, k in enumerate(self.kinds)])
        if len(self.kinds) == 1:
            self.vol_pts, self.vol_w, self.vol_B, self.vol_D = self.vol[0]   # [Qv, dim], [Qv], [Qv, Np], [Qv, dim, Np]
            self.phi0 = float(self.phi_0[0])
        self._face_cache = {}

    def _pad(self, a: np.ndarray) -> np.ndarray:
        """Zero-pad the mode axis (last) to ``n_p``."""
        if a.shape[-1] == self.n_p:
            return a
        out = np.zeros(a.shape[:-1] + (self.n_p,))
        out[..., :a.shape[-1]] = a
        return out

    def face_basis(self, side: int) -> np.ndarray:
        """``[E, Q, Np]`` basis values at the face quadrature points seen from ``side``."""
        if side not in self._face_cache:
            ref = self.mesh.face_ref[:, side]                       # [E, nfv, dim]
            pts = np.einsum("qv,evd->eqd", self.face_bary, ref)     # [E, Q, dim]
            E, Q, _ = pts.shape
            e = self.mesh.face_elem[:, side]
            ek = self.elem_kind[np.where(e >= 0, e, 0)]
            out = np.zeros((E, Q, self.n_p))
            for i, k in enumerate(self.kinds):
                sel = ek == i
                if sel.any():
                    out[sel] = self._pad(basis.elem_basis(k, self.p, pts[sel].reshape(-1, self.dim))).reshape(
                        -1, Q, self.n_p)
            self._face_cache[side] = out
        return self._face_cache[side]


def traces(B, C, detJ):
    """``U(x_q) = sum_j c_j phi_j(xi_q) / sqrt(det J)`` -> ``[..., Q, M]``."""
    return np.einsum("fqj,fmj->fqm", B, C) / np.sqrt(detJ)[:, None, None]


def volume_rhs(d: Discretization, U: np.ndarray) -> np.ndarray:
    mesh = d.mesh
    rhs = np.zeros_like(U)
    for i, (pts, w, B, D) in enumerate(d.vol):
        idx = np.nonzero(d.elem_kind == i)[0]
        sq = np.sqrt(mesh.detJ[idx])
        Uq = np.einsum("qj,kmj->kqm", B, U[idx]) / sq[:, None, None]       # [k, Qv, M]
        Fq = euler.physical_flux(Uq)                                        # [k, Qv, M, dim(e)]
        G = np.einsum("kde,kqme->kqmd", mesh.Jinv[idx], Fq)                 # contravariant
        rhs[idx] = np.einsum("q,qdj,kqmd->kmj", w, D, G) * sq[:, None, None]
    return rhs


def surface_rhs(d: Discretization, U: np.ndarray, elems=None) -> np.ndarray:
    """Surface term of Eq. (2) by a plain face loop (vectorised over faces, then
    accumulated in face order with ``np.add.at``).

    If ``elems`` is given, only faces touching those elements are evaluated
    (rows of other elements are then incomplete and must not be used).
    """
    mesh = d.mesh
    L = mesh.face_elem[:, 0]
    R = mesh.face_elem[:, 1]
    faces = np.arange(mesh.E)
    if elems is not None:
        sel = np.zeros(mesh.K, dtype=bool)
        sel[np.asarray(elems)] = True
        faces = faces[sel[L] | (R >= 0) & sel[np.where(R >= 0, R, 0)]]
    Lf = L[faces]
    Rf = R[faces]
    inter = Rf >= 0
    n = mesh.normal[faces]
    BL = d.face_basis(0)[faces]
    BR = d.face_basis(1)[faces]
    UL = traces(BL, U[Lf], mesh.detJ[Lf])
    Rs = np.where(inter, Rf, 0)
    UR = traces(BR, U[Rs], mesh.detJ[Rs])
    ghost = euler.wall_ghost(UL, n[:, None, :])
    UR = np.where(inter[:, None, None], UR, ghost)
    Fs = euler.rusanov(UL, UR, n[:, None, :])                            # [nf, Q, M]
    scale_L = mesh.measure[faces] / np.sqrt(mesh.detJ[Lf])
    scale_R = mesh.measure[faces] / np.sqrt(mesh.detJ[Rs])
    dL = np.einsum("q,fqj,fqm->fmj", d.face_w, BL, Fs) * scale_L[:, None, None]
    dR = np.einsum("q,fqj,fqm->fmj", d.face_w, BR, Fs) * scale_R[:, None, None]
    rhs = np.zeros_like(U)
    np.add.at(rhs, Lf, -dL)
    np.add.at(rhs, Rf[inter], dR[inter])
    return rhs


def surface_abs(d: Discretization, U: np.ndarray) -> np.ndarray:
    """Sum of absolute per-face contributions per entry (scale for parity tolerances)."""
    mesh = d.mesh
    L = mesh.face_elem[:, 0]
    R = mesh.face_elem[:, 1]
    inter = R >= 0
    n = mesh.normal
    BL = d.face_basis(0)
    BR = d.face_basis(1)
    Rs = np.where(inter, R, 0)
    UL = traces(BL, U[L], mesh.detJ[L])
    UR = np.where(inter[:, None, None], traces(BR, U[Rs], mesh.detJ[Rs]), euler.wall_ghost(UL, n[:, None, :]))
    Fs = euler.rusanov(UL, UR, n[:, None, :])
    aL = np.einsum("q,fqj,fqm->fmj", d.face_w, np.abs(BL), np.abs(Fs)) * (mesh.measure / np.sqrt(mesh.detJ[L]))[:, None, None]
    aR = np.einsum("q,fqj,fqm->fmj", d.face_w, np.abs(BR), np.abs(Fs)) * (mesh.measure / np.sqrt(mesh.detJ[Rs]))[:, None, None]
    out = np.zeros_like(U)
    np.add.at(out, L, aL)
    np.add.at(out, R[inter], aR[inter])
    return out


def rhs(d: Discretization, U: np.ndarray) -> np.ndarray:
    return volume_rhs(d, U) + surface_rhs(d, U)


def ssp_rk3(f, U: np.ndarray, dt: float) -> np.ndarray:
    """One step of the three-stage SSP Runge-Kutta method in Shu-Osher form for ``U' = f(U)``."""
    U1 = U + dt * f(U)
    U2 = 0.75 * U + 0.25 * (U1 + dt * f(U1))
    return U / 3.0 + 2.0 / 3.0 * (U2 + dt * f(U2))


def rk3_step(d: Discretization, U: np.ndarray, dt: float) -> np.ndarray:
    """One SSP-RK3 step of the semi-discrete DG system."""
    return ssp_rk3(lambda V: rhs(d, V), U, dt)


def mean_states(d: Discretization, U: np.ndarray) -> np.ndarray:
    """Element means ``c_0 phi_0 / sqrt(det J)``."""
    return U[:, :, 0] * d.phi_0[d.elem_kind][:, None] / np.sqrt(d.mesh.detJ)[:, None]


def inradius(mesh) -> np.ndarray:
    per = np.zeros(mesh.K)
    np.add.at(per, mesh.face_elem[:, 0], mesh.measure)
    inter = mesh.face_elem[:, 1] >= 0
    np.add.at(per, mesh.face_elem[inter, 1], mesh.measure[inter])
    return mesh.dim * mesh.elem_measure / per


def cfl_dt(d: Discretization, U: np.ndarray, cfl: float) -> float:
    """``dt = cfl * min(2 r_in) / max(|u| + c)`` at the element means."""
    m = mean_states(d, U)
    vel = m[:, 1:-1] / m[:, :1]
    smax = (np.linalg.norm(vel, axis=1) + euler.sound_speed(m)).max()
    return float(cfl * (2.0 * inradius(d.mesh)).min() / smax)


def physical_points(mesh, ref_pts: np.ndarray, elems=None) -> np.ndarray:
    """``x = x_0 + J xi`` for every (or the given) element and reference point -> ``[k, nq, dim]``."""
    idx = np.arange(mesh.K) if elems is None else np.asarray(elems)
    xyz = mesh.elem_xyz[idx]
    x0 = xyz[:, 0, :]
    if mesh.dim == 3:
        J = np.stack([xyz[:, a, :] - x0 for a in (1, 2, 3)], axis=2)
    else:
        quad = np.full(len(idx), mesh.kind == "quad") if mesh.elem_kind is None else mesh.elem_kind[idx] == 1
        second = np.where(quad, 3, 2)
        J = np.stack([xyz[:, 1, :] - x0, xyz[np.arange(len(idx)), second, :] - x0], axis=2)
    return x0[:, None, :] + np.einsum("ked,qd->kqe", J, ref_pts)


def _fine_rule(kind: str, n: int):
    if kind == "quad":
        return quadrature.quad_volume_rule(n)
    return quadrature.tri_volume_rule(n) if kind == "tri" else quadrature.tet_volume_rule(n)


def project(d: Discretization, func, extra: int = 3) -> np.ndarray:
    """L2 projection ``c_ij = sqrt(det J) sum_q w_q u(x_q) phi_j(xi_q)``."""
    mesh = d.mesh
    n = d.p + 1 + extra
    out = np.zeros((mesh.K, d.M, d.n_p))
    for i, k in enumerate(d.kinds):
        idx = np.nonzero(d.elem_kind == i)[0]
        pts, w = _fine_rule(k, n)
        B = d._pad(basis.elem_basis(k, d.p, pts))
        X = physical_points(mesh, pts, idx)
        u = func(X.reshape(-1, d.dim)).reshape(len(idx), len(w), -1)
        out[idx] = np.einsum("q,qj,kqm->kmj", w, B, u) * np.sqrt(mesh.detJ[idx])[:, None, None]
    return out


def l2_error(d: Discretization, U: np.ndarray, func, var: int = 0, extra: int = 3) -> float:
    mesh = d.mesh
    n = d.p + 1 + extra
    tot = 0.0
    for i, k in enumerate(d.kinds):
        idx = np.nonzero(d.elem_kind == i)[0]
        pts, w = _fine_rule(k, n)
        B = d._pad(basis.elem_basis(k, d.p, pts))
        X = physical_points(mesh, pts, idx)
        ex = func(X.reshape(-1, d.dim)).reshape(len(idx), len(w), -1)[:, :, var]
        num = np.einsum("qj,kj->kq", B, U[idx, var, :]) / np.sqrt(mesh.detJ[idx])[:, None]
        tot += (np.einsum("q,kq->k", w, (num - ex) ** 2) * mesh.detJ[idx]).sum()
    return float(np.sqrt(tot))
