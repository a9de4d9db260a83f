"""HIP kernels (through the C ABI) against the CPU oracle on the same seeded inputs.

Tolerance (float64): for every conserved variable m,
    max |gpu - oracle| <= 1e-12 * max |contribution sums| of that variable,
where the scale is the oracle's sum of absolute per-face (surface) or
per-point (volume) contributions, so cancellation cannot hide an error.
Integer outputs (layouts) are compared exactly in test_host_parity.
"""
import os

import numpy as np
import pytest

import synth
from oracle import dg
from oracle.mesh import build_mesh
from tests.helpers import make_input

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _dgc():
    import paper_1601_07613_amd as dgc

    return dgc


def _states(m, K):
    cen = synth.element_centroid(m["elem_xyz"], m["elem_vert"])
    if m["elem_xyz"].shape[2] == 3:
        return synth.density_wave_states(cen)
    return synth.shock_tube_states(cen)


def _eps(kind, p):
    """Noise level of the higher modes that keeps every trace state physical
    (orthonormal modes grow towards the vertices with the order)."""
    if kind in ("tets", "tetbox"):
        return 0.02 if p <= 1 else 0.005
    if kind in ("quads", "quadbox", "quadshuf", "hybrid", "hybridbox"):
        return 0.02 if p <= 2 else 0.005
    return 0.02 if p <= 3 else 0.004


class Case:
    def __init__(self, kind, size, seed, p, cseed=0, eps=None, layout="paper"):
        eps = _eps(kind, p) if eps is None else eps
        import torch

        dgc = _dgc()
        m = make_input(kind, size, seed)
        self.m = m
        self.O = build_mesh(m["elem_vert"], m["elem_xyz"])
        self.d = dg.Discretization(self.O, p)
        self.M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
        self.stats = self.M.color(seed=cseed, layout=layout)
        self.D = dgc.DeviceMesh(self.M, p)
        self.U = synth.perturbed_dofs(self.O.elem_measure, _states(m, self.O.K), self.d.n_p, eps=eps, seed=seed + 100)
        self.Ug = torch.from_numpy(self.D.to_layout(self.U)).cuda()
        print("case", kind, size, seed, "p", p, "K", self.O.K, "E", self.O.E, flush=True)

    def surface(self, variant, rhs0=None, D=None):
        import torch

        D = D or self.D
        rhs = torch.zeros_like(self.Ug) if rhs0 is None else rhs0.clone()
        ws = D.workspace("surface", variant) if variant in ("gather", "compact") else None
        D.surface_rhs(self.Ug, rhs, variant=variant, ws=ws)
        torch.cuda.synchronize()
        return rhs

    def to_host(self, t):
        return self.D.from_layout(t.cpu().numpy())


def _check(got, ref, scale, what):
    s = np.asarray(scale).max(axis=(0, 2))
    diff = np.abs(got - ref).max(axis=(0, 2))
    # a variable whose contributions all vanish (p = 0 volume term) must come out exactly zero
    err = np.where(s > 0, diff / np.where(s > 0, s, 1.0), np.where(diff == 0, 0.0, np.inf))
    assert err.max() <= TOL, "%s: relative error per variable %s" % (what, err)


def _volume_abs(d, U):
    """Sum of absolute per-point volume contributions (every element kind)."""
    from oracle import euler

    mesh = d.mesh
    out = np.zeros_like(U)
    for i, (pts, w, B, D) in enumerate(d.vol):
        idx = d.elem_kind == i
        sq = np.sqrt(mesh.detJ[idx])
        Uq = np.einsum("qj,kmj->kqm", B, U[idx]) / sq[:, None, None]
        Fq = euler.physical_flux(Uq)
        G = np.abs(np.einsum("kde,kqme->kqmd", mesh.Jinv[idx], Fq))
        out[idx] = np.einsum("q,qdj,kqmd->kmj", w, np.abs(D), G) * sq[:, None, None]
    return out


@pytest.mark.parametrize("form", ["team", "team_prefetch", "thread"])
@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("variant", ["colored", "atomic", "gather", "compact"])
def test_surface_periodic_triangles(p, variant, form):
    c = Case("periodic", 16, 1, p)
    c.D.set_launch(form)
    got = c.to_host(c.surface(variant))
    _check(got, dg.surface_rhs(c.d, c.U), dg.surface_abs(c.d, c.U), "surface %s p=%d" % (variant, p))


@pytest.mark.parametrize("form,block,xcd", [("team", 256, False), ("team", 64, False), ("team", 256, True),
                                            ("team_prefetch", 256, False), ("team_prefetch", 128, True),
                                            ("thread", 256, False), ("thread", 128, True)])
@pytest.mark.parametrize("variant", ["colored", "atomic", "gather", "compact"])
def test_surface_delaunay_walls_ragged(variant, form, block, xcd):
    c = Case("delaunay", 12000, 2, 2)
    assert c.O.E % 256 != 0 and c.O.n_boundary > 0
    c.D.set_launch(form, block, xcd)
    got = c.to_host(c.surface(variant))
    _check(got, dg.surface_rhs(c.d, c.U), dg.surface_abs(c.d, c.U), "surface delaunay " + variant)


@pytest.mark.parametrize("kind,size", [("quads", 12), ("quadbox", 11), ("quadshuf", 14)])
@pytest.mark.parametrize("form", ["default", "team", "thread"])
@pytest.mark.parametrize("p", [0, 1, 2, 3])
@pytest.mark.parametrize("variant", ["colored", "atomic", "gather", "compact"])
def test_surface_quads(p, variant, form, kind, size):
    """Parallelogram meshes (periodic, and walled with a ragged face count),
    four colors, tensor Legendre basis."""
    c = Case(kind, size, 1, p)
    c.D.set_launch(form)
    assert c.stats["n_colors"] == 4
    got = c.to_host(c.surface(variant))
    _check(got, dg.surface_rhs(c.d, c.U), dg.surface_abs(c.d, c.U), "surface %s %s p=%d" % (kind, variant, p))


@pytest.mark.parametrize("kind,size", [("hybrid", 14), ("hybridbox", 13)])
@pytest.mark.parametrize("form", ["default", "thread"])
@pytest.mark.parametrize("p", [0, 1, 2, 3])
@pytest.mark.parametrize("variant", ["colored", "atomic", "gather", "compact"])
def test_surface_mixed(p, variant, form, kind, size):
    """Mixed triangle / parallelogram meshes (four colors; every element has
    (p+1)^2 slots, a triangle's tables are zero beyond its own modes)."""
    c = Case(kind, size, 2, p)
    c.D.set_launch(form)
    assert c.stats["n_colors"] == 4 and c.D.info["elem_type"] == 3
    got = c.to_host(c.surface(variant))
    _check(got, dg.surface_rhs(c.d, c.U), dg.surface_abs(c.d, c.U), "surface %s %s p=%d" % (kind, variant, p))


@pytest.mark.parametrize("kind,size,p", [("hybrid", 14, 1), ("hybrid", 14, 3), ("hybridbox", 13, 2)])
def test_volume_mixed(kind, size, p):
    import torch

    c = Case(kind, size, 5, p)
    rhs = torch.full_like(c.Ug, 7.0)
    c.D.volume_rhs(c.Ug, rhs)
    torch.cuda.synchronize()
    _check(c.to_host(rhs), dg.volume_rhs(c.d, c.U), _volume_abs(c.d, c.U), "volume %s p=%d" % (kind, p))


def test_rk3_mixed_vortex_20_steps():
    """Isentropic vortex on a periodic hybrid mesh (triangles around the
    center, parallelograms elsewhere), p = 2: 20 SSP-RK3 steps against the
    oracle."""
    import torch

    c = Case("hybrid", 14, 8, 2)
    U0 = dg.project(c.d, lambda X: synth.isentropic_vortex(X, 0.0, beta=4.0, radius=0.1))
    dt = dg.cfl_dt(c.d, U0, 0.1)
    Ug = torch.from_numpy(c.D.to_layout(U0)).cuda()
    ws = c.D.workspace("rk", "colored")
    U = U0.copy()
    for _ in range(20):
        c.D.rk_step(Ug, dt, ws=ws)
        U = dg.rk3_step(c.d, U, dt)
    torch.cuda.synchronize()
    got = c.to_host(Ug)
    assert np.abs(got - U).max() / np.abs(U).max() <= TOL


@pytest.mark.parametrize("form,p", [("default", 0), ("default", 1), ("default", 2), ("team", 1), ("thread", 2),
                                    ("mode_team", 1), ("pair_team", 1)])
@pytest.mark.parametrize("variant", ["colored", "atomic", "gather", "compact"])
def test_surface_tets_walls(p, variant, form):
    """Tetrahedra in a closed box (reflective walls on all six sides)."""
    c = Case("tetbox", 4, 5, p)
    assert c.O.n_boundary > 0 and c.stats["n_colors"] == 4
    c.D.set_launch(form)
    got = c.to_host(c.surface(variant))
    _check(got, dg.surface_rhs(c.d, c.U), dg.surface_abs(c.d, c.U), "surface walled tets %s p=%d" % (variant, p))


# the mode and pair teams exist for N_p = 4 only (tetrahedra at p = 1)
TET_FORMS = [(f, p) for p in (0, 1, 2) for f in ("default", "team", "thread")] + [("mode_team", 1), ("pair_team", 1)]


@pytest.mark.parametrize("form,p", TET_FORMS)
@pytest.mark.parametrize("variant", ["colored", "atomic", "gather", "compact"])
def test_surface_tets(p, variant, form):
    c = Case("tets", 6, 3, p)
    c.D.set_launch(form)
    assert c.stats["n_colors"] == 4
    got = c.to_host(c.surface(variant))
    _check(got, dg.surface_rhs(c.d, c.U), dg.surface_abs(c.d, c.U), "surface tets %s p=%d" % (variant, p))


@pytest.mark.parametrize("kind,size,p", [("periodic", 16, 0), ("periodic", 16, 1), ("periodic", 16, 2),
                                         ("periodic", 16, 3), ("periodic", 16, 4), ("periodic", 16, 5),
                                         ("delaunay", 6000, 2), ("tets", 5, 0),
                                         ("tets", 5, 1), ("tets", 5, 2), ("quads", 12, 1), ("quads", 12, 3),
                                         ("quadbox", 11, 2)])
@pytest.mark.parametrize("form", ["default", "valu"])
def test_volume(kind, size, p, form):
    import torch

    c = Case(kind, size, 4, p)
    c.D.set_volume_form(form)
    rhs = torch.full_like(c.Ug, 7.0)  # overwritten by the kernel
    c.D.volume_rhs(c.Ug, rhs)
    torch.cuda.synchronize()
    _check(c.to_host(rhs), dg.volume_rhs(c.d, c.U), _volume_abs(c.d, c.U), "volume %s p=%d" % (kind, p))


@pytest.mark.parametrize("kind,size,p", [("periodic", 16, 0), ("periodic", 16, 1), ("periodic", 16, 2),
                                         ("periodic", 16, 3), ("delaunay", 6000, 2), ("delaunay", 6001, 1),
                                         ("quads", 12, 2), ("quadbox", 11, 3)])
def test_volume_forms(kind, size, p):
    """The MFMA form (four elements per 16 x 16 x 4 f64 product chain), the
    one-work-item form and the team form against the oracle and each other;
    ragged element counts exercise the masked rows of the last group."""
    import torch

    c = Case(kind, size, 14, p)
    ref = dg.volume_rhs(c.d, c.U)
    out = {}
    for form in ("mfma", "valu", "team"):
        c.D.set_volume_form(form)
        rhs = torch.full_like(c.Ug, 7.0)
        c.D.volume_rhs(c.Ug, rhs)
        torch.cuda.synchronize()
        out[form] = c.to_host(rhs)
        _check(out[form], ref, _volume_abs(c.d, c.U), "volume %s %s p=%d" % (form, kind, p))
    c.D.set_volume_form("default")
    scale = np.abs(ref).max()
    assert np.abs(out["mfma"] - out["valu"]).max() <= 1e-13 * max(scale, 1e-300)
    assert np.abs(out["team"] - out["valu"]).max() <= 1e-13 * max(scale, 1e-300)


@pytest.mark.parametrize("algorithm", ["paper", "greedy"])
@pytest.mark.parametrize("layout", ["paper", "paper_sfc", "paired", "renumber", "none"])
def test_surface_other_layouts(layout, algorithm):
    """Every layout of the paper's coloring and of the standard greedy
    coloring (up to five colors on triangles, Section 1; the Table 7
    comparison): the colored pass gives the oracle's uncolored face sum."""
    import torch

    dgc = _dgc()
    c = Case("delaunay", 9000, 3, 2)
    if algorithm == "greedy":
        st = c.M.color(algorithm="greedy", layout=layout)
        assert 3 <= st["n_colors"] <= 5
    else:
        c.M.set_colors(c.M.export("color"), layout=layout)
    D = dgc.DeviceMesh(c.M, 2)
    D.set_launch("team", 256, True)
    Ug = torch.from_numpy(D.to_layout(c.U)).cuda()
    rhs = torch.zeros_like(Ug)
    D.surface_rhs(Ug, rhs)
    torch.cuda.synchronize()
    _check(D.from_layout(rhs.cpu().numpy()), dg.surface_rhs(c.d, c.U), dg.surface_abs(c.d, c.U), "layout " + layout)


@pytest.mark.parametrize("kind,size,p", [("quads", 12, 2), ("quadshuf", 20, 2), ("hybrid", 14, 2), ("tets", 5, 1),
                                         ("tetbox", 4, 1), ("periodic", 16, 3)])
def test_surface_paired_layout_other_kinds(kind, size, p):
    """The paired numbering on parallelograms (grid and random numbering),
    mixed meshes, tetrahedra (periodic and walled) and triangles at p = 3,
    in the default launch: the colored pass and one RK3 step of the default
    form against the oracle."""
    import torch

    c = Case(kind, size, 31, p, layout="paired")
    c.D.set_launch("default")
    got = c.to_host(c.surface("colored"))
    _check(got, dg.surface_rhs(c.d, c.U), dg.surface_abs(c.d, c.U), "paired layout " + kind)
    dt = 1e-4
    ref = dg.rk3_step(c.d, c.U, dt)
    U = c.Ug.clone()
    c.D.rk_step(U, dt, ws=c.D.workspace("rk", "colored"))
    torch.cuda.synchronize()
    assert np.abs(c.to_host(U) - ref).max() <= TOL * np.abs(ref).max()


def test_surface_accumulates_onto_volume_term():
    import torch

    c = Case("periodic", 16, 5, 2)
    rhs = torch.zeros_like(c.Ug)
    c.D.volume_rhs(c.Ug, rhs)
    out = c.surface("colored", rhs0=rhs)
    ref = dg.rhs(c.d, c.U)
    scale = dg.surface_abs(c.d, c.U) + _volume_abs(c.d, c.U)
    _check(c.to_host(out), ref, scale, "volume + surface")


def test_colored_is_race_free_and_bitwise_deterministic():
    """Permuting the faces inside every color cannot change a single bit of the
    colored result (each element is touched once per color), and two runs agree."""
    import torch

    c = Case("delaunay", 8000, 6, 2)
    a = c.surface("colored")
    b = c.surface("colored")
    assert torch.equal(a, b)
    D = c.D
    off = D.info["color_off"]
    rng = np.random.default_rng(0)
    perm = np.concatenate([off[k] + rng.permutation(off[k + 1] - off[k]) for k in range(len(off) - 1)])
    pt = torch.from_numpy(perm).cuda()
    E = D.E
    saved = (D.face_lr, D.face_code, D.face_geo)
    D.face_lr = D.face_lr.view(2, E)[:, pt].contiguous().view(-1)
    D.face_code = D.face_code.view(2, E)[:, pt].contiguous().view(-1)
    D.face_geo = D.face_geo.view(-1, E)[:, pt].contiguous().view(-1)
    D.dm.face_lr, D.dm.face_code, D.dm.face_geo = D.face_lr.data_ptr(), D.face_code.data_ptr(), D.face_geo.data_ptr()
    try:
        p = c.surface("colored")
    finally:
        D.face_lr, D.face_code, D.face_geo = saved
        D.dm.face_lr, D.dm.face_code, D.dm.face_geo = (D.face_lr.data_ptr(), D.face_code.data_ptr(),
                                                       D.face_geo.data_ptr())
    assert torch.equal(a, p)


def test_empty_color_and_tiny_mesh():
    import torch

    dgc = _dgc()
    # a valid coloring whose color 2 is empty (colors 0, 1, 3)
    c = Case("periodic", 6, 7, 1)
    col = c.M.export("color").astype(np.int8)
    col[col == 2] = 3
    c.M.set_colors(col)
    D = dgc.DeviceMesh(c.M, 1)
    assert D.info["n_colors"] == 4 and D.info["color_off"][2] == D.info["color_off"][3]
    Ug = torch.from_numpy(D.to_layout(c.U)).cuda()
    rhs = torch.zeros_like(Ug)
    D.surface_rhs(Ug, rhs)
    torch.cuda.synchronize()
    _check(D.from_layout(rhs.cpu().numpy()), dg.surface_rhs(c.d, c.U), dg.surface_abs(c.d, c.U), "empty color")
    # smallest periodic mesh the generator makes: 3 x 3 x 2 triangles
    t = Case("periodic", 3, 8, 2)
    _check(t.to_host(t.surface("colored")), dg.surface_rhs(t.d, t.U), dg.surface_abs(t.d, t.U), "tiny mesh")


def test_rk3_100_steps_vortex():
    """16 x 16 periodic p = 1 isentropic vortex, 100 SSP-RK3 steps at CFL 0.1."""
    import torch

    m = make_input("periodic", 16, 1)
    O = build_mesh(m["elem_vert"], m["elem_xyz"])
    d = dg.Discretization(O, 1)
    U0 = dg.project(d, lambda X: synth.isentropic_vortex(X, 0.0))
    dt = dg.cfl_dt(d, U0, 0.1)
    dgc = _dgc()
    M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    M.color(seed=1)
    D = dgc.DeviceMesh(M, 1)
    Ug = torch.from_numpy(D.to_layout(U0)).cuda()
    ws = D.workspace("rk", "colored")
    U = U0.copy()
    for _ in range(100):
        D.rk_step(Ug, dt, ws=ws)
        U = dg.rk3_step(d, U, dt)
    torch.cuda.synchronize()
    got = D.from_layout(Ug.cpu().numpy())
    err = np.abs(got - U).max() / np.abs(U).max()
    assert err <= TOL, err


@pytest.mark.parametrize("kind,size,p", [("delaunay", 6000, 2), ("periodic", 16, 1), ("periodic", 16, 3),
                                         ("tets", 5, 1), ("tets", 4, 2), ("tetbox", 4, 1), ("quads", 12, 2),
                                         ("quadbox", 11, 1)])
def test_rk3_step_forms_agree(kind, size, p):
    """The stage combination fused into the last color's face kernel, the
    volume term fused into the first color's, and the whole step in one
    work-group give the separate-kernel step (same formulas; only the
    compiler's contraction of a x + b (y + dt r) and, with the fused volume
    term, the summation order of the volume term may differ) over several
    steps, walls included."""
    import torch

    c = Case(kind, size, 21, p)
    if c.D.dim == 2:
        # a smooth state: the shock tube has no limiter to survive several steps at p >= 1
        st = synth.density_wave_states(synth.element_centroid(c.m["elem_xyz"]), vel=(0.5, 0.3))
        c.Ug = torch.from_numpy(c.D.to_layout(synth.perturbed_dofs(c.O.elem_measure, st, c.d.n_p, eps=0.01,
                                                                   seed=3))).cuda()
    U0 = c.Ug.clone()
    dt = 1e-4
    out = {}
    for form in ("fused", "fused_volume", "block", "separate", "default"):
        c.D.set_rk_form(form)
        U = U0.clone()
        ws = c.D.workspace("rk", "colored")
        for _ in range(5):
            c.D.rk_step(U, dt, ws=ws)
        torch.cuda.synchronize()
        out[form] = U
    c.D.set_rk_form("default")
    scale = out["separate"].abs().max().item()
    for form in ("fused", "fused_volume", "block", "default"):
        assert (out[form] - out["separate"]).abs().max().item() <= 1e-14 * scale, form
    assert not torch.equal(out["default"], U0)
    # the single-work-group form needs f64
    with pytest.raises(_dgc().DgcError):
        c.D.set_rk_form("block")
        c.D.rk_step(U0.clone(), dt, precision="f32", ws=c.D.workspace("rk", "colored", "f32"))
    c.D.set_rk_form("default")


@pytest.mark.parametrize("kind,size,p", [("delaunay", 6000, 2), ("periodic", 16, 1), ("periodic", 16, 3),
                                         ("quads", 12, 2), ("quadbox", 11, 1)])
def test_rk3_compact_stage(kind, size, p):
    """The compact variant's step (a face pass and one element pass per stage,
    the element pass adding the volume term and writing the combination)
    against the oracle's step and, over 5 steps, against the compact step
    with separate kernels and the colored default step (the same formulas;
    only the order of sums differs)."""
    import torch

    c = Case(kind, size, 24, p)
    st = synth.density_wave_states(synth.element_centroid(c.m["elem_xyz"]), vel=(0.5, 0.3))
    U0h = synth.perturbed_dofs(c.O.elem_measure, st, c.d.n_p, eps=0.01, seed=6)
    dt = 1e-4
    ref = dg.rk3_step(c.d, U0h, dt)
    U0 = torch.from_numpy(c.D.to_layout(U0h)).cuda()
    U = U0.clone()
    wsc = c.D.workspace("rk", "compact")
    c.D.rk_step(U, dt, variant="compact", ws=wsc)
    torch.cuda.synchronize()
    assert np.abs(c.to_host(U) - ref).max() <= TOL * np.abs(ref).max()
    out = {}
    for name, variant, form in (("stage", "compact", "default"), ("separate", "compact", "separate"),
                                ("colored", "colored", "default")):
        c.D.set_rk_form(form)
        U = U0.clone()
        ws = c.D.workspace("rk", variant)
        for _ in range(5):
            c.D.rk_step(U, dt, variant=variant, ws=ws)
        torch.cuda.synchronize()
        out[name] = U
    c.D.set_rk_form("default")
    scale = out["colored"].abs().max().item()
    assert not torch.equal(out["stage"], U0)
    for name in ("separate", "colored"):
        assert (out["stage"] - out[name]).abs().max().item() <= 1e-14 * scale, name


@pytest.mark.parametrize("kind,size,p", [("delaunay", 6000, 2), ("periodic", 16, 1), ("tets", 5, 1),
                                         ("quadbox", 11, 1)])
def test_rk3_f32_form_fused_volume(kind, size, p):
    """The f32 form with the volume term fused into the first color's face
    kernel matches the f32 form with a separate volume kernel: over 5 steps
    the two states differ by at most 1e-5 of the change the steps made (f32
    rounding of a differently ordered sum; a missing or doubled volume term
    would differ by O(1) of it)."""
    import torch

    c = Case(kind, size, 22, p)
    if kind != "tets":
        st = synth.density_wave_states(synth.element_centroid(c.m["elem_xyz"]), vel=(0.5, 0.3))
        c.Ug = torch.from_numpy(c.D.to_layout(synth.perturbed_dofs(c.O.elem_measure, st, c.d.n_p, eps=0.01,
                                                                   seed=4))).cuda()
    U0 = c.Ug.clone()
    dt = 1e-4
    out = {}
    for form in ("separate", "fused_volume"):
        c.D.set_rk_form(form)
        U = U0.clone()
        ws = c.D.workspace("rk", "colored", "f32")
        for _ in range(5):
            c.D.rk_step(U, dt, precision="f32", ws=ws)
        torch.cuda.synchronize()
        out[form] = U
    c.D.set_rk_form("default")
    change = (out["separate"] - U0).abs().max().item()
    assert change > 0
    assert (out["fused_volume"] - out["separate"]).abs().max().item() <= 1e-5 * change


def test_rk3_quads_vortex_20_steps():
    """Isentropic vortex on a 12 x 12 periodic parallelogram mesh, p = 2:
    20 SSP-RK3 steps (fused stage combination) against the oracle."""
    import torch

    c = Case("quads", 12, 8, 2)
    U0 = dg.project(c.d, lambda X: synth.isentropic_vortex(X, 0.0, beta=4.0, radius=0.1))
    dt = dg.cfl_dt(c.d, U0, 0.1)
    Ug = torch.from_numpy(c.D.to_layout(U0)).cuda()
    ws = c.D.workspace("rk", "colored")
    U = U0.copy()
    for _ in range(20):
        c.D.rk_step(Ug, dt, ws=ws)
        U = dg.rk3_step(c.d, U, dt)
    torch.cuda.synchronize()
    got = c.to_host(Ug)
    assert np.abs(got - U).max() / np.abs(U).max() <= TOL


def test_workspace_errors_on_device():
    import torch

    dgc = _dgc()
    c = Case("periodic", 8, 9, 1)
    rhs = torch.zeros_like(c.Ug)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    for variant in ("gather", "compact"):
        with pytest.raises(dgc.DgcError) as e:
            c.D.surface_rhs(c.Ug, rhs, variant=variant, ws=small)
        assert e.value.name == "DGC_E_WORKSPACE"
    with pytest.raises(dgc.DgcError) as e:
        c.D.rk_step(c.Ug, 1e-3, ws=small)
    assert e.value.name == "DGC_E_WORKSPACE"
    torch.cuda.synchronize()
    assert float(rhs.abs().max()) == 0.0


@pytest.mark.parametrize("kind,size,p", [("tets", 4, 2), ("periodic", 9, 4), ("delaunay", 1500, 5),
                                         ("quadbox", 7, 3), ("delaunay", 2000, 2)])
@pytest.mark.parametrize("variant", ["colored", "atomic", "gather", "compact"])
def test_surface_stream_form(kind, size, p, variant):
    """The streaming team form (quadrature points visited one at a time)
    against the oracle, every variant, walls included."""
    c = Case(kind, size, 23, p)
    c.D.set_launch("team_stream")
    got = c.to_host(c.surface(variant))
    c.D.set_launch("default")
    _check(got, dg.surface_rhs(c.d, c.U), dg.surface_abs(c.d, c.U), "stream %s" % variant)


def test_surface_stream_form_f32():
    import torch

    c = Case("tets", 4, 24, 2)
    U32 = c.U.astype(np.float32)
    Ug = torch.from_numpy(c.D.to_layout(U32)).cuda()
    rhs = torch.zeros_like(Ug)
    c.D.set_launch("team_stream")
    c.D.surface_rhs(Ug, rhs, variant="colored", precision="f32")
    c.D.set_launch("default")
    torch.cuda.synchronize()
    U = U32.astype(np.float64)
    tol = TOL32 * max(1.0, (c.D.n_p + c.D.tinfo["n_qf"]) / 9.0)
    _check_tol(c.D.from_layout(rhs.cpu().numpy()).astype(np.float64), dg.surface_rhs(c.d, U),
               dg.surface_abs(c.d, U), "stream f32", tol)


@pytest.fixture(scope="module")
def full_c1():
    """The full Delaunay workload (~500 k Poisson-disc points, ~1 M triangles, p = 2)
    in the paired layout the benchmark times."""
    c = Case("delaunay", 500_000, 2, 2, cseed=0, eps=0.01, layout="paired")
    return c


def test_full_size_every_element(full_c1):
    """The colored pass of the whole Delaunay workload in the launch the bench
    times, against the oracle's face sum on every one of its ~1M elements."""
    c = full_c1
    c.D.set_launch("default")
    got = c.to_host(c.surface("colored"))
    ref = dg.surface_rhs(c.d, c.U)
    _check(got, ref, dg.surface_abs(c.d, c.U), "full-size colored, every element")
    # the other variants agree with the colored one on every entry
    for v in ("atomic", "gather", "compact"):
        other = c.to_host(c.surface(v))
        _check(other, got, dg.surface_abs(c.d, c.U), "full-size %s vs colored" % v)
    c.D.set_launch("thread")
    other = c.to_host(c.surface("colored"))
    c.D.set_launch("default")
    _check(other, got, dg.surface_abs(c.d, c.U), "full-size thread form vs team form")
    # the paper's own layout of the same coloring, every element against the oracle
    import torch

    colors = c.M.export("color")
    c.M.set_colors(colors, layout="paper")
    Dp = _dgc().DeviceMesh(c.M, 2)
    c.M.set_colors(colors, layout="paired")
    Ugp = torch.from_numpy(Dp.to_layout(c.U)).cuda()
    rp = torch.zeros_like(Ugp)
    Dp.surface_rhs(Ugp, rp)
    torch.cuda.synchronize()
    _check(Dp.from_layout(rp.cpu().numpy()), ref, dg.surface_abs(c.d, c.U), "full-size colored, paper layout")


def test_full_size_rk_step(full_c1):
    """One SSP-RK3 step of the full Delaunay workload in the default form
    (volume term in the first color's face kernel, stage combination in the
    last color's) against the oracle's step: the new state at 1e-12 of its
    largest entry, the change the step made at 1e-10 of the largest change."""
    import torch

    c = full_c1
    # a smooth state (the shock tube's noisy traces reach negative pressures
    # within a step: there is no limiter)
    st = synth.density_wave_states(synth.element_centroid(c.m["elem_xyz"]), vel=(0.5, 0.3))
    U0 = synth.perturbed_dofs(c.O.elem_measure, st, c.d.n_p, eps=0.01, seed=5)
    dt = dg.cfl_dt(c.d, U0, 0.1)
    ref = dg.rk3_step(c.d, U0, dt)
    assert np.isfinite(ref).all()
    U = torch.from_numpy(c.D.to_layout(U0)).cuda()
    c.D.set_rk_form("default")
    c.D.rk_step(U, dt, ws=c.D.workspace("rk", "colored"))
    got = c.to_host(U)
    assert np.isfinite(got).all()
    assert np.abs(got - ref).max() <= TOL * np.abs(ref).max()
    change = np.abs(ref - U0).max()
    assert np.abs((got - U0) - (ref - U0)).max() <= 1e-10 * change


@pytest.fixture(scope="module")
def full_c2():
    """The full tetrahedral workload: 64^3 periodic cubes x 6 Kuhn tetrahedra
    (1,572,864 tetrahedra), p = 1, density wave plus 1 % high-mode noise, in
    the paired layout the benchmark times."""
    return Case("tets", 64, 3, 1, cseed=0, eps=0.01, layout="paired")


def test_full_size_tets_every_element(full_c2):
    """The whole tetrahedral workload: every element against the oracle (f64);
    the f32 form on 3,002 sampled elements at its own bar."""
    c = full_c2
    assert c.D.info["n_colors"] == 4
    c.D.set_launch("default")
    got = c.to_host(c.surface("colored"))
    scale = dg.surface_abs(c.d, c.U)
    _check(got, dg.surface_rhs(c.d, c.U), scale, "full-size tets colored, every element")
    rng = np.random.default_rng(43)
    S = np.unique(np.concatenate([rng.choice(c.O.K, 3000, replace=False), [0, c.O.K - 1]]))
    # the f32 form of the same pass at its own bar
    import torch

    U32 = c.U.astype(np.float32)
    Ug32 = torch.from_numpy(c.D.to_layout(U32)).cuda()
    r32 = torch.zeros_like(Ug32)
    c.D.surface_rhs(Ug32, r32, variant="colored", precision="f32")
    torch.cuda.synchronize()
    got32 = c.D.from_layout(r32.cpu().numpy()).astype(np.float64)
    ref32 = dg.surface_rhs(c.d, U32.astype(np.float64), elems=S)
    _check_tol(got32[S], ref32[S], scale[S], "full-size tets sampled f32", TOL32)


# ---------------------------------------------------------------- FP32 form

TOL32 = 2e-6


@pytest.mark.parametrize("kind,size,p", [("periodic", 16, 2), ("periodic", 16, 5), ("delaunay", 6000, 2),
                                         ("tets", 5, 1), ("tets", 5, 2), ("quads", 12, 2), ("hybrid", 14, 2)])
@pytest.mark.parametrize("variant", ["colored", "atomic", "gather", "compact"])
def test_surface_and_volume_f32(kind, size, p, variant):
    """f32 storage and arithmetic (geometry stored in f64) against the f64
    oracle evaluated on the same f32-rounded DOFs.  The worst-case rounding
    error of the trace and projection sums grows linearly with their length
    N_p + Q, so the bar set at p = 2 (N_p + Q = 9) is scaled by that length."""
    import torch

    c = Case(kind, size, 12, p)
    tol = TOL32 * max(1.0, (c.D.n_p + c.D.tinfo["n_qf"]) / 9.0)
    U32 = c.U.astype(np.float32)
    U = U32.astype(np.float64)
    Ug = torch.from_numpy(c.D.to_layout(U32)).cuda()
    rhs = torch.zeros_like(Ug)
    ws = c.D.workspace("surface", variant, "f32") if variant in ("gather", "compact") else None
    c.D.surface_rhs(Ug, rhs, variant=variant, precision="f32", ws=ws)
    vol = torch.zeros_like(Ug)
    c.D.volume_rhs(Ug, vol, precision="f32")
    torch.cuda.synchronize()
    _check32 = lambda got, ref, scale, what: _check_tol(got, ref, scale, what, tol)
    _check32(c.D.from_layout(rhs.cpu().numpy()).astype(np.float64), dg.surface_rhs(c.d, U),
             dg.surface_abs(c.d, U), "f32 surface")
    _check32(c.D.from_layout(vol.cpu().numpy()).astype(np.float64), dg.volume_rhs(c.d, U),
             _volume_abs(c.d, U), "f32 volume")


def _check_tol(got, ref, scale, what, tol):
    s = np.asarray(scale).max(axis=(0, 2))
    diff = np.abs(got - ref).max(axis=(0, 2))
    err = np.where(s > 0, diff / np.where(s > 0, s, 1.0), np.where(diff == 0, 0.0, np.inf))
    assert err.max() <= tol, "%s: relative error per variable %s" % (what, err)


def test_rk3_f32_form_error_budget():
    """100 SSP-RK3 steps of the 16 x 16 vortex with the f32 form (f32 shadow,
    f32 flux and quadrature, f64 stage accumulation): relative L2 error of
    every variable against the f64 oracle stays below 1e-6."""
    import torch

    m = make_input("periodic", 16, 1)
    O = build_mesh(m["elem_vert"], m["elem_xyz"])
    d = dg.Discretization(O, 1)
    U0 = dg.project(d, lambda X: synth.isentropic_vortex(X, 0.0))
    dt = dg.cfl_dt(d, U0, 0.1)
    dgc = _dgc()
    M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    M.color(seed=1)
    D = dgc.DeviceMesh(M, 1)
    Ug = torch.from_numpy(D.to_layout(U0)).cuda()
    ws = D.workspace("rk", "colored", "f32")
    U = U0.copy()
    for _ in range(100):
        D.rk_step(Ug, dt, precision="f32", ws=ws)
        U = dg.rk3_step(d, U, dt)
    torch.cuda.synchronize()
    got = D.from_layout(Ug.cpu().numpy())
    # by orthonormality the L2 norm of a field is the Euclidean norm of its DOFs
    rel = np.sqrt(((got - U) ** 2).sum(axis=(0, 2)) / (U ** 2).sum(axis=(0, 2)))
    print("f32 form relative L2 error per variable:", rel)
    assert rel.max() <= 1e-6, rel


# ------------------------------------------------- nonconforming (refined) mesh

def _refined(n=24, levels=3, radius=0.15, p=2, cseed=0, layout=None):
    from oracle import refine as R
    from oracle.coloring import color_faces

    dgc = _dgc()
    m = synth.periodic_tri(n, jitter=0.0, seed=4)
    O = build_mesh(m["elem_vert"], m["elem_xyz"])
    col, _ = color_faces(O, seed=cseed)
    st = R.from_base(O, col)
    M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    M.color(seed=cseed)
    for lvl in range(1, levels + 1):
        xyz = np.array([lf.xyz for lf in st.leaves])
        lev = np.array([lf.level for lf in st.leaves])
        flags = synth.refine_flags(xyz, lev, lvl - 1, radius=radius)
        st, _ = R.refine(st, flags)
        M, _ = M.refine(flags)
    mesh, color, orient, levels_ = R.to_mesh(st)
    d = dg.Discretization(mesh, p)
    if layout is not None:
        M.set_colors(M.export("color"), layout=layout)
    D = dgc.DeviceMesh(M, p)
    print("refined mesh K", mesh.K, "E", mesh.E, "hanging", int((orient[:, 1] >= 2).sum()), flush=True)
    return mesh, d, D


def test_surface_refined_configured_size():
    """The refined workload at its configured size: 128 x 128 x 2 base, three
    refinement passes within 0.15 of the center (178,724 leaves, six colors,
    hanging faces), every variant against the oracle on every element."""
    import torch

    mesh, d, D = _refined(n=128)
    assert D.info["n_colors"] == 6 and mesh.K == 178_724
    U = synth.perturbed_dofs(mesh.elem_measure, synth.shock_tube_states(mesh.elem_xyz.mean(axis=1)), d.n_p,
                             eps=0.02, seed=21)
    Ug = torch.from_numpy(D.to_layout(U)).cuda()
    ref, scale = dg.surface_rhs(d, U), dg.surface_abs(d, U)
    for variant in ("colored", "atomic", "gather", "compact"):
        rhs = torch.zeros_like(Ug)
        ws = D.workspace("surface", variant) if variant in ("gather", "compact") else None
        D.surface_rhs(Ug, rhs, variant=variant, ws=ws)
        torch.cuda.synchronize()
        _check(D.from_layout(rhs.cpu().numpy()), ref, scale, "refined 128 base " + variant)


@pytest.mark.parametrize("variant", ["colored", "atomic", "gather", "compact"])
@pytest.mark.parametrize("form", ["default", "thread"])
def test_surface_refined_six_colors(variant, form):
    import torch

    mesh, d, D = _refined()
    assert D.info["n_colors"] == 6 and D.info["max_slots"] >= 5
    D.set_launch(form)
    U = synth.perturbed_dofs(mesh.elem_measure, synth.shock_tube_states(mesh.elem_xyz.mean(axis=1)), d.n_p,
                             eps=0.02, seed=21)
    Ug = torch.from_numpy(D.to_layout(U)).cuda()
    rhs = torch.zeros_like(Ug)
    ws = D.workspace("surface", variant) if variant in ("gather", "compact") else None
    D.surface_rhs(Ug, rhs, variant=variant, ws=ws)
    torch.cuda.synchronize()
    _check(D.from_layout(rhs.cpu().numpy()), dg.surface_rhs(d, U), dg.surface_abs(d, U), "refined " + variant)


def test_refined_paired_layout():
    """The refined mesh (hanging faces, six colors, elements missing colors)
    renumbered in the paired layout: every variant of the surface pass and
    five SSP-RK3 steps against the oracle."""
    import torch

    mesh, d, D = _refined(n=16, levels=2, radius=0.2, p=2, layout="paired")
    assert D.info["n_colors"] == 6
    U = synth.perturbed_dofs(mesh.elem_measure, synth.shock_tube_states(mesh.elem_xyz.mean(axis=1)), d.n_p,
                             eps=0.02, seed=23)
    Ug = torch.from_numpy(D.to_layout(U)).cuda()
    ref, scale = dg.surface_rhs(d, U), dg.surface_abs(d, U)
    for variant in ("colored", "atomic", "gather", "compact"):
        rhs = torch.zeros_like(Ug)
        ws = D.workspace("surface", variant) if variant in ("gather", "compact") else None
        D.surface_rhs(Ug, rhs, variant=variant, ws=ws)
        torch.cuda.synchronize()
        _check(D.from_layout(rhs.cpu().numpy()), ref, scale, "refined, paired layout, " + variant)
    U0 = dg.project(d, lambda X: synth.isentropic_vortex(X, 0.0))
    dt = dg.cfl_dt(d, U0, 0.1)
    Ug = torch.from_numpy(D.to_layout(U0)).cuda()
    ws = D.workspace("rk", "colored")
    Uo = U0.copy()
    for _ in range(5):
        D.rk_step(Ug, dt, ws=ws)
        Uo = dg.rk3_step(d, Uo, dt)
    torch.cuda.synchronize()
    assert np.abs(D.from_layout(Ug.cpu().numpy()) - Uo).max() / np.abs(Uo).max() <= TOL


def test_rk3_refined_vortex_20_steps():
    import torch

    mesh, d, D = _refined(n=16, levels=2, radius=0.2, p=2)
    U0 = dg.project(d, lambda X: synth.isentropic_vortex(X, 0.0))
    dt = dg.cfl_dt(d, U0, 0.1)
    Ug = torch.from_numpy(D.to_layout(U0)).cuda()
    ws = D.workspace("rk", "colored")
    U = U0.copy()
    for _ in range(20):
        D.rk_step(Ug, dt, ws=ws)
        U = dg.rk3_step(d, U, dt)
    torch.cuda.synchronize()
    got = D.from_layout(Ug.cpu().numpy())
    assert np.abs(got - U).max() / np.abs(U).max() <= TOL


def test_device_layout_permutation_round_trip():
    import torch

    c = Case("delaunay", 5000, 13, 2)
    Uo = torch.from_numpy(c.U).cuda()
    Ul = c.D.to_layout_device(Uo)
    torch.cuda.synchronize()
    assert torch.equal(Ul.cpu(), torch.from_numpy(c.D.to_layout(c.U)))
    back = c.D.from_layout_device(Ul)
    torch.cuda.synchronize()
    assert torch.equal(back, Uo)


def test_device_child_color_map_matches_refinement():
    """The GPU closed-form map gives the colors the refinement assigns: halves
    c / (c+3) mod 6 of every split edge, interior edges = parallel parent edge."""
    import torch

    from oracle import refine as R

    dgc = _dgc()
    rng = np.random.default_rng(3)
    par = rng.integers(0, 6, size=(1000, 3)).astype(np.int8)
    out = dgc.child_colors(torch.from_numpy(par).cuda()).cpu().numpy()
    for i in range(len(par)):
        for k in range(3):
            assert tuple(out[i, 2 * k:2 * k + 2]) == R.child_colors(int(par[i, k]))
            assert out[i, 6 + k] == par[i, k]
    # on a refined mesh: every split parent's three edges and its center child
    from oracle.coloring import color_faces

    m = synth.periodic_tri(12, jitter=0.0, seed=4)
    O = build_mesh(m["elem_vert"], m["elem_xyz"])
    col, _ = color_faces(O, seed=0)
    st = R.from_base(O, col)
    flags = synth.refine_flags(np.array([lf.xyz for lf in st.leaves]), np.zeros(O.K), 0, radius=0.3)
    st, _ = R.refine(st, flags)
    parents, expect = [], []
    for i in range(0, len(st.leaves) - 3):
        lf = st.leaves[i]
        if lf.level == 1 and i + 3 < len(st.leaves) and st.leaves[i + 3].level == 1:
            c0, c1, c2, ce = st.leaves[i:i + 4]
            if c0.edges[0].parent is None or ce.edges[0] is not c2.edges[0]:
                continue
            E = [c0.edges[0].parent, c1.edges[1].parent, c2.edges[2].parent]
            parents.append([e.color for e in E])
            expect.append([x for e in E for x in (e.children[0].color, e.children[1].color)]
                          + [ce.edges[k].color for k in range(3)])
    assert len(parents) > 10
    got = dgc.child_colors(torch.from_numpy(np.array(parents, dtype=np.int8)).cuda()).cpu().numpy()
    assert np.array_equal(got, np.array(expect, dtype=np.int8))
