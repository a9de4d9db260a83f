"""DOF transfer between a triangle and its four children (oracle).

TEST INFRASTRUCTURE ONLY.

Refinement and coarsening (Section 3.2) change the mesh under a running DG
solution; the solution moves by L2 projection, the plain definition:

* prolongation: child ``k`` of a parent with modal DOFs ``c`` (physical basis
  ``v_j = phi_j / sqrt(det J)``, orthonormal on each element) gets
  ``c_k = P_k c`` with ``(P_k)_{jl} = int_{child k} v_j^child v_l^parent``.
  In reference coordinates ``det J_child = det J_parent / 4``, so
  ``(P_k)_{jl} = 1/2 int_T phi_j(xi) phi_l(A_k xi + b_k) dxi`` where
  ``xi -> A_k xi + b_k`` maps the unit triangle onto child ``k`` inside the
  parent's reference triangle.  The integrand has degree ``2 p``; the
  collapsed rule with ``p + 1`` points per direction is exact for it.
* restriction: the parent DOFs of a function given on the four children are
  ``c = sum_k P_k^T c_k`` (the same integrals read the other way).

Children (in the parent's reference coordinates, vertices in each child's own
order): ``(V0, M01, M20)``, ``(M01, V1, M12)``, ``(M20, M12, V2)`` and the
center child ``(M12, M20, M01)`` -- the split of :mod:`oracle.refine`.

Pins (``tests/test_oracle_transfer.py``): ``sum_k P_k^T P_k = I`` (the
children tile the parent and the parent basis is orthonormal), so
restriction undoes prolongation exactly; prolongation reproduces the parent
polynomial point by point; restriction of a piecewise function preserves its
integral (mass).
"""

from __future__ import annotations

import numpy as np

from . import basis, quadrature

_V = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
_M01, _M12, _M20 = 0.5 * (_V[0] + _V[1]), 0.5 * (_V[1] + _V[2]), 0.5 * (_V[2] + _V[0])
CHILD_VERTS = [np.array(c) for c in ((_V[0], _M01, _M20), (_M01, _V[1], _M12), (_M20, _M12, _V[2]),
                                     (_M12, _M20, _M01))]


def child_map(k: int, xi: np.ndarray) -> np.ndarray:
    """Parent reference coordinates of the child-``k`` reference points ``xi [n, 2]``."""
    X = CHILD_VERTS[k]
    return X[0][None, :] + xi[:, :1] * (X[1] - X[0])[None, :] + xi[:, 1:2] * (X[2] - X[0])[None, :]


def prolongation(p: int) -> np.ndarray:
    """``[4, N_p, N_p]``: ``P[k] @ c_parent`` = DOFs of child ``k``."""
    x, w = quadrature.tri_volume_rule(p + 1)
    Bc = basis.eval_basis(2, p, x)                               # [Q, Np] child basis
    out = []
    for k in range(4):
        Bp = basis.eval_basis(2, p, child_map(k, x))             # parent basis at the same points
        out.append(0.5 * np.einsum("q,qj,ql->jl", w, Bc, Bp))
    return np.array(out)


def transfer(p: int, U_old: np.ndarray, origin) -> np.ndarray:
    """DOFs ``[K_new, M, N_p]`` of the new leaves from those of the previous
    leaves, following ``origin`` (see :class:`oracle.refine.RefineState`)."""
    P = prolongation(p)
    K = len(origin)
    out = np.zeros((K,) + U_old.shape[1:])
    for i, (kind, src) in enumerate(origin):
        if kind == 0:
            out[i] = U_old[src[0]]
        elif 1 <= kind <= 4:
            out[i] = U_old[src[0]] @ P[kind - 1].T
        elif kind == 5:
            out[i] = sum(U_old[src[k]] @ P[k] for k in range(4))
        else:
            raise ValueError("unknown origin kind %r" % (kind,))
    return out
