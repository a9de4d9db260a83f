"""Batched (many meshes per launch) forms against the single-mesh path."""
import numpy as np
import pytest

import synth
from tests.helpers import make_input

pytestmark = pytest.mark.gpu


def _member(kind, size, seed, p, precision="f64", smooth=False):
    import torch

    import paper_1601_07613_amd as dgc

    m = make_input(kind, size, seed)
    M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    M.color(seed=seed)
    D = dgc.DeviceMesh(M, p)
    cen = synth.element_centroid(m["elem_xyz"])
    if smooth:  # stays physical over many steps (no limiter)
        st = synth.uniform_states(len(cen), vel=(0.3, -0.2, 0.1)[:D.dim])
    else:
        st = synth.density_wave_states(cen) if D.dim == 3 else synth.shock_tube_states(cen)
    # smaller high-mode noise at p >= 3 keeps every trace state physical
    U = synth.perturbed_dofs(synth.element_measure(m["elem_xyz"]), st, D.n_p, eps=0.02 if p <= 2 else 0.005,
                             seed=seed)
    Ug = torch.from_numpy(D.to_layout(U)).cuda()
    ws = D.workspace("rk", "colored", precision)
    dt = 1e-4 * (1 + seed % 3)
    print("member", kind, size, seed, "K", D.K, flush=True)
    return D, Ug, ws, dt


def _batch_volume_form(D, precision):
    """The vector volume form the batched kernels use for this member: one
    work-item per element for tetrahedra, for f32 triangles and f32
    quadrilaterals at p = 3 and for f64 triangles at p = 3, else the team."""
    quad = D.n_p in (4, 9, 16)
    if D.dim == 3:
        return "valu"
    if precision == "f32":
        return "team" if quad and D.n_p != 16 else "valu"
    return "valu" if D.n_p == 10 else "team"


TRI = [("periodic", 12, 1), ("delaunay", 3000, 2), ("periodic", 16, 3), ("periodic", 9, 4), ("delaunay", 1200, 5)]


QUAD = [("quads", 8, 1), ("quadbox", 9, 2), ("quads", 12, 3)]


@pytest.mark.parametrize("family,p", [("tri", 1), ("tri", 2), ("tri", 3), ("quad", 1), ("quad", 2), ("quad", 3)])
def test_batched_stage_rhs_is_bitwise_single(family, p):
    import torch

    import paper_1601_07613_amd as dgc

    members = [_member(k, s, sd, p) for k, s, sd in (TRI if family == "tri" else QUAD)]
    B = dgc.Batch(members)
    B.volume(0)
    B.surface(0)
    torch.cuda.synchronize()
    for i, (D, Ug, ws, dt) in enumerate(members):
        # the batch runs the vector volume forms: compare against the same form
        D.set_volume_form(_batch_volume_form(D, "f64"))
        r = torch.zeros_like(Ug)
        D.volume_rhs(Ug, r)
        D.surface_rhs(Ug, r)
        torch.cuda.synchronize()
        assert torch.equal(B.stage_rhs(i), r), i


def test_batched_tets_bitwise_single():
    import torch

    import paper_1601_07613_amd as dgc

    members = [_member("tets", 4, 1, 1), _member("tets", 5, 2, 1)]
    B = dgc.Batch(members)
    B.volume(0)
    B.surface(0)
    torch.cuda.synchronize()
    for i, (D, Ug, ws, dt) in enumerate(members):
        r = torch.zeros_like(Ug)
        D.volume_rhs(Ug, r)
        D.surface_rhs(Ug, r)
        torch.cuda.synchronize()
        assert torch.equal(B.stage_rhs(i), r), i


TET = [("tets", 4, 1), ("tets", 6, 2), ("tets", 4, 3)]


@pytest.mark.parametrize("family,p", [("tri", 2), ("quad", 2), ("quad", 1), ("tet", 1)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batched_rk_steps_match_single(precision, family, p):
    """Batched SSP-RK3 steps (the first color's launch carrying the volume
    term for triangles and parallelograms, the last color's the stage
    combination in f64) equal the single-mesh default steps, walls
    included."""
    import torch

    import paper_1601_07613_amd as dgc

    fam = {"tri": TRI, "quad": QUAD, "tet": TET}[family]
    members = [_member(k, s, sd, p, precision, smooth=True) for k, s, sd in fam]
    ref = [(D, Ug.clone(), D.workspace("rk", "colored", precision), dt) for D, Ug, ws, dt in members]
    B = dgc.Batch(members, precision=precision)
    # the batched step fuses the volume term and the stage combination into
    # the first and last colors' launches like the single-mesh default step,
    # so both round alike (the f32 form would show a differently ordered
    # volume sum)
    for D, _, _, _ in ref:
        D.set_volume_form("default")
        D.set_rk_form("default")
    for _ in range(10):
        B.rk_step()
        for D, U, w, dt in ref:
            D.rk_step(U, dt, precision=precision, ws=w)
    torch.cuda.synchronize()
    for (D, Ug, _, _), (_, U, _, _) in zip(members, ref):
        assert torch.isfinite(U).all()
        err = float((Ug - U).abs().max() / U.abs().max())
        assert err <= 1e-14, err


def test_member_alone_equals_member_in_mix():
    import torch

    import paper_1601_07613_amd as dgc

    mix = [_member(k, s, sd, 2, smooth=True) for k, s, sd in TRI]
    alone = [_member("delaunay", 3000, 2, 2, smooth=True)]
    Bm = dgc.Batch(mix)
    Ba = dgc.Batch(alone)
    for _ in range(5):
        Bm.rk_step()
        Ba.rk_step()
    torch.cuda.synchronize()
    assert torch.equal(mix[1][1], alone[0][1])


def test_graph_replays_match_eager():
    """A captured batched RK3 step, replayed several times with eager work and
    synchronisation between replays, matches eager batched steps every time."""
    import torch

    import paper_1601_07613_amd as dgc

    g_members = [_member(k, s, sd, 1, smooth=True) for k, s, sd in TRI[:3]]
    e_members = [(D, U.clone(), D.workspace("rk", "colored"), dt) for D, U, ws, dt in g_members]
    Bg = dgc.Batch(g_members)
    Be = dgc.Batch(e_members)
    graph = Bg.capture()
    for rep in range(4):
        graph.replay()
        Be.rk_step()
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        for (_, Ug, _, _), (_, Ue, _, _) in zip(g_members, e_members):
            assert torch.equal(Ug, Ue), rep
        del junk
