"""dgc_rk_step_noalloc: the SSP-RK3 step with the library's fixed stage
storage instead of a caller workspace, against dgc_rk_step with a workspace
(same kernels, so the results must be bitwise equal), through the C ABI."""
from __future__ import annotations

import ctypes as C

import pytest

import synth
from tests.helpers import make_input

dgc = pytest.importorskip("paper_1601_07613_amd")
from paper_1601_07613_amd import _lib  # noqa: E402

VARIANT = {"colored": 0, "atomic": 1, "gather": 2}
PREC = {"f64": 0, "f32": 1}


def _device_case(kind, size, p, seed):
    import torch

    m = make_input(kind, size, seed)
    M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    M.color(seed=seed)
    D = dgc.DeviceMesh(M, p)
    cen = synth.element_centroid(m["elem_xyz"])
    st = synth.density_wave_states(cen) if kind == "tets" else \
        synth.density_wave_states(cen, vel=(0.5, 0.3))
    U0 = synth.perturbed_dofs(synth.element_measure(m["elem_xyz"]), st, D.n_p, eps=0.01, seed=seed)
    return D, torch.from_numpy(D.to_layout(U0)).cuda()


def _both(D, U0, dt, variant, precision, steps=2):
    """U after `steps` steps through dgc_rk_step (torch workspace) and
    through dgc_rk_step_noalloc, both called through the C ABI."""
    import torch

    L = _lib.load()
    stream = torch.cuda.current_stream().cuda_stream
    ws = D.workspace("rk", variant, precision)
    Ua, Ub = U0.clone(), U0.clone()
    for _ in range(steps):
        _lib.check(L.dgc_rk_step(C.byref(D.dm), Ua.data_ptr(), dt, VARIANT[variant], PREC[precision],
                                 ws.data_ptr(), ws.numel(), stream), "dgc_rk_step")
        _lib.check(L.dgc_rk_step_noalloc(C.byref(D.dm), Ub.data_ptr(), dt, VARIANT[variant], PREC[precision],
                                         stream), "dgc_rk_step_noalloc")
    torch.cuda.synchronize()
    return Ua, Ub


@pytest.mark.gpu
@pytest.mark.parametrize("variant,precision,cases", [
    ("colored", "f64", [("periodic", 60, 2), ("periodic", 16, 2)]),
    ("colored", "f32", [("delaunay", 6000, 2), ("periodic", 12, 1)]),
    ("gather", "f64", [("tets", 6, 1), ("tets", 3, 1)]),
    ("atomic", "f64", [("quads", 30, 2), ("quads", 10, 2)]),
])
def test_noalloc_step_equals_workspace_step(gpu_device, variant, precision, cases):
    """Two calls in a row, the second on a smaller mesh (the array still holds
    the first call's larger contents): each equals the workspace step."""
    import torch

    for i, (kind, size, p) in enumerate(cases):
        print("noalloc case", variant, precision, kind, size, p, flush=True)
        D, U0 = _device_case(kind, size, p, seed=3 + i)
        need = D.workspace_bytes("rk", variant, precision)
        assert need <= _lib.DGC_NOALLOC_MAX_BYTES
        Ua, Ub = _both(D, U0, 1e-4, variant, precision)
        assert torch.isfinite(Ua).all()
        assert not torch.equal(Ua, U0)
        if variant == "atomic":
            # atomic adds land in any order: equal up to rounding (the f64 bar)
            err = ((Ua - Ub).abs().amax(dim=(0, 2)) / Ua.abs().amax(dim=(0, 2))).max().item()
            assert err <= 1e-12, err
        else:
            assert torch.equal(Ua, Ub), (Ua - Ub).abs().max().item()


@pytest.mark.gpu
def test_noalloc_step_keeps_no_state_between_meshes(gpu_device):
    """A large mesh, then a small one, then the large one again: the third
    call equals a fresh workspace step although the array holds the small
    mesh's stage states at the front."""
    import torch

    Db, Ub0 = _device_case("periodic", 64, 2, seed=5)
    Ds, Us0 = _device_case("periodic", 8, 2, seed=6)
    for D, U0 in ((Db, Ub0), (Ds, Us0), (Db, Ub0)):
        Ua, Ub = _both(D, U0, 1e-4, "colored", "f64", steps=1)
        assert torch.equal(Ua, Ub)


def test_noalloc_rejects_a_mesh_beyond_the_fixed_storage():
    """A mesh whose stage storage exceeds DGC_NOALLOC_MAX_BYTES is refused
    with DGC_E_WORKSPACE before any device call (the pointers below are never
    dereferenced)."""
    info, _ = dgc.tables(0, 2)
    dm = _lib.DMesh()
    dm.elem_type, dm.p, dm.n_p, dm.n_var = 0, 2, info["n_p"], 4
    dm.n_qf, dm.n_qv, dm.n_codes, dm.n_orient = info["n_qf"], info["n_qv"], info["n_codes"], info["n_orient"]
    dm.n_elem, dm.n_face, dm.max_slots, dm.n_colors = 200_000, 300_000, 3, 3
    for c, off in enumerate((0, 100_000, 200_000, 300_000)):
        dm.color_off[c] = off
    dm.face_lr = dm.face_code = dm.face_geo = dm.elem_geo = dm.tables = dm.elem_slots = 0x1000
    L = _lib.load()
    b = C.c_size_t()
    _lib.check(L.dgc_workspace_bytes(C.byref(dm), 1, 0, 0, C.byref(b)), "ws")
    assert b.value > _lib.DGC_NOALLOC_MAX_BYTES
    assert L.dgc_rk_step_noalloc(C.byref(dm), 0x1000, 1e-3, 0, 0, None) == -7  # DGC_E_WORKSPACE
    assert b"dgc_rk_step_noalloc" in L.dgc_last_error()
    # bad arguments are still reported as such, before any device call
    dm.n_elem, dm.n_face = 100, 150
    for c, off in enumerate((0, 50, 100, 150)):
        dm.color_off[c] = off
    assert L.dgc_rk_step_noalloc(C.byref(dm), None, 1e-3, 0, 0, None) == -1  # DGC_E_ARG (null U)
    dm.p = 7
    assert L.dgc_rk_step_noalloc(C.byref(dm), 0x1000, 1e-3, 0, 0, None) == -6  # DGC_E_UNSUPPORTED
