"""The launch autotuner: it installs the fastest candidate, and the
installed configuration computes what the library default computes."""
import numpy as np
import pytest

import synth
from tests.helpers import make_input

pytestmark = pytest.mark.gpu


def _mesh(kind, size, seed, p):
    import torch

    import paper_1601_07613_amd as dgc

    m = make_input(kind, size, seed)
    M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    M.color(seed=seed)
    D = dgc.DeviceMesh(M, p)
    st = synth.density_wave_states(synth.element_centroid(m["elem_xyz"]), vel=(0.5, 0.3, 0.2)[:D.dim])
    U = synth.perturbed_dofs(synth.element_measure(m["elem_xyz"]), st, D.n_p, eps=0.01, seed=seed)
    print("tune case", kind, size, "K", D.K, flush=True)
    return D, torch.from_numpy(D.to_layout(U)).cuda()


@pytest.mark.parametrize("kind,size,p", [("delaunay", 6000, 2), ("tets", 6, 1), ("quads", 16, 2)])
def test_autotune_surface_launch(kind, size, p):
    import torch

    from paper_1601_07613_amd.tune import DEFAULT_CANDIDATES, autotune, candidates_for

    D, Ug = _mesh(kind, size, 31, p)
    cands = candidates_for(D)
    # tetrahedra at p = 1 also try the pair team
    assert len(cands) == len(DEFAULT_CANDIDATES) + (4 if kind == "tets" else 0)
    ref = torch.zeros_like(Ug)
    D.set_launch("default")
    D.surface_rhs(Ug, ref)
    rhs = torch.zeros_like(Ug)
    best, results = autotune(D, Ug, rhs, reps=3, warmup=1)
    assert best in cands and len(results) == len(cands)
    assert all(ms > 0 for _, ms in results)
    assert best == min(results, key=lambda r: r[1])[0]
    got = torch.zeros_like(Ug)
    D.surface_rhs(Ug, got)  # the installed launch
    torch.cuda.synchronize()
    # the same arithmetic up to the order of the trace sums (mode, pair and
    # variable teams for tetrahedra)
    scale = ref.abs().max().item()
    assert (got - ref).abs().max().item() <= 1e-12 * scale
    D.set_launch("default")


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_autotune_rk_step_form(precision):
    import torch

    from paper_1601_07613_amd.tune import RK_FORMS, autotune_rk

    D, Ug = _mesh("delaunay", 6000, 32, 2)
    U0 = Ug.clone()
    dt = 1e-4
    best, results = autotune_rk(D, Ug, dt, precision=precision)
    assert torch.equal(Ug, U0)  # the tuner steps a copy
    assert best in RK_FORMS and [f for f, _ in results] == list(RK_FORMS)
    ws = D.workspace("rk", "colored", precision)
    a = U0.clone()
    for _ in range(3):
        D.rk_step(a, dt, precision=precision, ws=ws)  # the installed form
    D.set_rk_form("separate")
    b = U0.clone()
    for _ in range(3):
        D.rk_step(b, dt, precision=precision, ws=ws)
    D.set_rk_form("default")
    torch.cuda.synchronize()
    change = (b - U0).abs().max().item()
    tol = 1e-11 if precision == "f64" else 1e-5
    assert (a - b).abs().max().item() <= tol * change
