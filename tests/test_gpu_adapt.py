"""Dynamic refinement on the GPU against the oracle: the L2 transfer of the
solution onto refined / coarsened meshes (dgc_adapt_transfer) and a
moving-feature adaptive run (coarsen + refine every few SSP-RK3 steps).

Tolerances (float64): a transfer is a handful of N_p-term sums, compared at
1e-13 of the largest DOF magnitude; the adaptive run at 1e-12 relative, the
bar of the fixed-mesh RK tests.
"""
import numpy as np
import pytest

import synth
from oracle import dg, refine as R, transfer as T
from oracle.coloring import color_faces
from oracle.mesh import build_mesh

pytestmark = pytest.mark.gpu


def _dgc():
    import paper_1601_07613_amd as dgc

    return dgc


def _base(n, seed=4, jitter=0.05, cseed=0):
    dgc = _dgc()
    m = synth.periodic_tri(n, jitter=jitter, seed=seed)
    O = build_mesh(m["elem_vert"], m["elem_xyz"])
    col, _ = color_faces(O, seed=cseed)
    M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    M.color(seed=cseed)
    return m, O, col, M


def _leaves(st):
    return np.array([lf.xyz for lf in st.leaves]), np.array([lf.level for lf in st.leaves])


def _dofs(K, p, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((K, 4, (p + 1) * (p + 2) // 2))


@pytest.mark.parametrize("p", [0, 1, 2, 3, 5])
def test_transfer_refine_and_coarsen_match_oracle(p):
    import torch

    m, O, col, M = _base(12)
    st = R.from_base(O, col)
    D0 = _dgc().DeviceMesh(M, p)
    U = _dofs(O.K, p, seed=p)
    Ug = torch.from_numpy(D0.to_layout(U)).cuda()
    print("transfer p", p, "K", O.K, flush=True)
    for cyc, center in enumerate([(0.5, 0.5), (0.6, 0.45), (0.3, 0.7)]):
        xyz, lev = _leaves(st)
        _, coarse = synth.adapt_flags(xyz, lev, center, 0.2, 0.25, max_level=2)
        st, n = R.coarsen(st, coarse)
        U = T.transfer(p, U, st.origin)
        M, n_c = M.coarsen(coarse)
        assert n_c == n
        D = _dgc().DeviceMesh(M, p)
        Ug = D.transfer_from(Ug)
        xyz, lev = _leaves(st)
        fine, _ = synth.adapt_flags(xyz, lev, center, 0.2, 0.25, max_level=2)
        st, _ = R.refine(st, fine)
        U = T.transfer(p, U, st.origin)
        M, _ = M.refine(fine)
        D = _dgc().DeviceMesh(M, p)
        Ug = D.transfer_from(Ug)
        torch.cuda.synchronize()
        got = D.from_layout(Ug.cpu().numpy())
        assert got.shape == U.shape
        assert np.abs(got - U).max() <= 1e-13 * np.abs(U).max(), "cycle %d" % cyc
    assert M.info()["max_level"] == 2


def test_refine_then_coarsen_is_the_identity_on_device():
    import torch

    dgc = _dgc()
    m, O, col, M = _base(10)
    p = 2
    D0 = dgc.DeviceMesh(M, p)
    U = _dofs(O.K, p, seed=11)
    Ug = torch.from_numpy(D0.to_layout(U)).cuda()
    flags = np.zeros(O.K, dtype=np.uint8)
    flags[::3] = 1
    M1, _ = M.refine(flags)
    D1 = dgc.DeviceMesh(M1, p)
    U1 = D1.transfer_from(Ug)
    # merge every family again: the base leaves come back (renumbered as a refined mesh)
    M2, n = M1.coarsen(np.ones(D1.K, dtype=np.uint8))
    assert n == (M1.export("elem_level") == 1).sum() // 4
    D2 = dgc.DeviceMesh(M2, p)
    U2 = D2.transfer_from(U1)
    torch.cuda.synchronize()
    back = D2.from_layout(U2.cpu().numpy())
    assert np.abs(back - U).max() <= 1e-13 * np.abs(U).max()


def test_transfer_marks_out_of_range_sources_with_nan():
    import torch

    dgc = _dgc()
    m, O, col, M = _base(6)
    p = 1
    D0 = dgc.DeviceMesh(M, p)
    Ug = torch.ones((O.K, 4, 3), dtype=torch.float64, device="cuda")
    flags = np.zeros(O.K, dtype=np.uint8)
    flags[0] = 1
    M1, _ = M.refine(flags)
    D1 = dgc.DeviceMesh(M1, p)
    # claim the old array is shorter than it is: records whose source lies
    # beyond it are rejected by the kernel's bounds check (no access happens)
    short = Ug[: O.K // 2].contiguous()
    out = D1.transfer_from(short)
    torch.cuda.synchronize()
    src = D1.mesh.export("dev_adapt_src").reshape(4, -1)
    bad = (src >= O.K // 2).any(axis=0)
    o = out.cpu().numpy()
    assert bad.any() and (~bad).any()
    assert np.isnan(o[bad]).all() and np.isfinite(o[~bad]).all()
    with pytest.raises(ValueError):
        D1.transfer_from(torch.zeros((4, 4, 3), dtype=torch.float32, device="cuda"))


def test_moving_feature_adaptive_run_matches_oracle():
    """Isentropic vortex on a 12 x 12 periodic base, p = 1; every 4 SSP-RK3
    steps coarsen away from a moving center and refine one level around it
    (up to level 2).  The GPU run (native tree surgery, device transfer,
    device steps) equals the oracle run (oracle tree, oracle transfer, oracle
    steps) to 1e-12 relative after 24 steps."""
    import torch

    from paper_1601_07613_amd.amr import AdaptiveRun

    p, L, every, n_steps = 1, 2, 4, 24
    m, O, col, M = _base(12)
    d0 = dg.Discretization(O, p)
    U0 = dg.project(d0, lambda X: synth.isentropic_vortex(X, 0.0, beta=4.0, radius=0.1))
    dt = dg.cfl_dt(d0, U0, 0.1) / 2 ** L

    def crit(xyz, lev, t):
        # a criterion center much faster than the flow, so families merge within the run
        center = (0.5 + 40.0 * t, 0.5 + 25.0 * t)
        return synth.adapt_flags(xyz, lev, center, 0.12, 0.14, max_level=L)

    D0 = _dgc().DeviceMesh(M, p)
    run = AdaptiveRun(M, p, torch.from_numpy(D0.to_layout(U0)).cuda(), dt, crit, every=every)
    run.run(n_steps)
    torch.cuda.synchronize()
    got = run.D.from_layout(run.U.cpu().numpy())

    st = R.from_base(O, col)
    U = U0.copy()
    t = 0.0
    d = None
    for step in range(n_steps):
        if step % every == 0:
            xyz, lev = _leaves(st)
            _, coarse = crit(xyz, lev, t)
            st, _ = R.coarsen(st, coarse)
            U = T.transfer(p, U, st.origin)
            xyz, lev = _leaves(st)
            fine, _ = crit(xyz, lev, t)
            st, _ = R.refine(st, fine)
            U = T.transfer(p, U, st.origin)
            d = dg.Discretization(R.to_mesh(st)[0], p)
        U = dg.rk3_step(d, U, dt)
        t += dt
    merged = sum(r["merged"] for r in run.log)
    print("adaptive run: K", len(st.leaves), "merged", merged, "log", run.log[-1], flush=True)
    assert merged > 0 and max(r["n_colors"] for r in run.log) <= 6
    assert got.shape == U.shape
    assert np.abs(got - U).max() / np.abs(U).max() <= 1e-12
    # the transfers and the steps conserve every variable's integral (periodic)
    mass0 = (U0[:, :, 0] * np.sqrt(O.detJ)[:, None]).sum(axis=0)
    mesh = R.to_mesh(st)[0]
    mass = (got[:, :, 0] * np.sqrt(mesh.detJ)[:, None]).sum(axis=0)
    assert np.abs(mass - mass0).max() <= 1e-12 * np.abs(mass0).max()
