"""Dynamic refinement under a running solution (Section 3.2 applied in time).

Every ``every`` SSP-RK3 steps the mesh follows a moving feature: leaves the
caller's criterion marks are coarsened (four siblings merge back into their
parent, whose edge colors were kept in the edge tree), then leaves it marks
are refined by one level (children colored by the closed-form six-color
map), and the solution is moved to each new mesh by L2 projection on the
device (``DeviceMesh.transfer_from``).  No coloring search runs after the
base mesh is colored.  The host side (tree surgery, face table, layout) is
native code; the solution never leaves the device.
"""

from __future__ import annotations

import time

import numpy as np

from . import DeviceMesh


class AdaptiveRun:
    """``criterion(elem_xyz [K,3,2], levels [K], t) -> (refine, coarsen)``
    boolean flags per leaf (original leaf order of the mesh it is given)."""

    def __init__(self, mesh, p: int, U, dt: float, criterion, every: int = 5, precision: str = "f64"):
        self.mesh = mesh
        self.p = p
        self.dt = float(dt)
        self.criterion = criterion
        self.every = int(every)
        self.precision = precision
        self.D = DeviceMesh(mesh, p)
        self.U = U
        self.ws = self.D.workspace("rk", "colored", precision)
        self.t = 0.0
        self.steps = 0
        self.log = []

    def _leaves(self, M):
        K = M.info()["n_elem"]
        return M.export("elem_xyz").reshape(K, 3, 2), M.export("elem_level")

    def adapt(self):
        """One coarsen + refine cycle at the current time; returns its record."""
        import torch

        t0 = time.perf_counter()
        xyz, lev = self._leaves(self.mesh)
        _, coarse = self.criterion(xyz, lev, self.t)
        M1, merged = self.mesh.coarsen(coarse)
        xyz, lev = self._leaves(M1)
        refine, _ = self.criterion(xyz, lev, self.t)
        M2, closure = M1.refine(refine)
        host_s = time.perf_counter() - t0
        D1 = DeviceMesh(M1, self.p)
        D2 = DeviceMesh(M2, self.p)
        D1.adapt_arrays()
        D2.adapt_arrays()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        U1 = D1.transfer_from(self.U)
        U2 = D2.transfer_from(U1)
        ev[1].record()
        ev[1].synchronize()
        rec = {"t": self.t, "step": self.steps, "merged": merged, "refined": int(np.count_nonzero(refine)),
               "closure": closure, "n_elem": D2.K, "n_face": D2.E, "n_colors": D2.info["n_colors"],
               "host_ms": host_s * 1e3, "transfer_us": ev[0].elapsed_time(ev[1]) * 1e3}
        self.mesh, self.D, self.U = M2, D2, U2
        self.ws = self.D.workspace("rk", "colored", self.precision)
        self.log.append(rec)
        return rec

    def run(self, n_steps: int):
        """Advance ``n_steps`` SSP-RK3 steps, adapting before every ``every``-th."""
        for _ in range(n_steps):
            if self.every > 0 and self.steps % self.every == 0:
                self.adapt()
            self.D.rk_step(self.U, self.dt, precision=self.precision, ws=self.ws)
            self.steps += 1
            self.t += self.dt
        return self.U
