"""Error budget of the reduced-precision forms (the f32 form, and why the
basis contractions do not run in bf16 / fp16).

The f32 form evaluates the right-hand side from an f32 copy of the stage
state and keeps the SSP-RK3 accumulation in f64.  Here the same scheme is
emulated with the oracle: each stage's right-hand side is evaluated from
the state rounded to f32, bf16 or fp16 (the operand the basis contraction
would read in that precision), the stages accumulate in f64.  After 100
steps of the 16 x 16 periodic vortex (p = 1, CFL 0.1) the relative L2 error
against the f64 run must stay within the 1e-6 budget for f32; bf16 and fp16
miss it by orders of magnitude (their 8- and 11-bit significands round each
stage input at ~4e-3 and ~5e-4 relative), so those contractions are not
built.  By orthonormality the L2 norm of a field is the Euclidean norm of
its DOFs."""
import numpy as np
import pytest

import synth
from oracle import dg
from oracle.mesh import build_mesh

BUDGET = 1e-6


def _run(d, U0, dt, n_steps, rnd):
    U = U0.copy()
    for _ in range(n_steps):
        U = dg.ssp_rk3(lambda V: dg.rhs(d, rnd(V)), U, dt)
    return U


def _round(dtype):
    import torch

    if dtype is None:
        return lambda V: V
    return lambda V: torch.from_numpy(V).to(dtype).to(torch.float64).numpy()


@pytest.fixture(scope="module")
def vortex():
    m = synth.periodic_tri(16, seed=1)
    M = build_mesh(m["elem_vert"], m["elem_xyz"])
    d = dg.Discretization(M, 1)
    U0 = dg.project(d, lambda X: synth.isentropic_vortex(X, 0.0))
    dt = dg.cfl_dt(d, U0, 0.1)
    ref = _run(d, U0, dt, 100, _round(None))
    return d, U0, dt, ref


def _rel_l2(U, ref):
    return np.sqrt(((U - ref) ** 2).sum(axis=(0, 2)) / (ref ** 2).sum(axis=(0, 2))).max()


@pytest.mark.parametrize("name,within", [("float32", True), ("float16", False), ("bfloat16", False)])
def test_stage_input_precision_against_budget(vortex, name, within):
    import torch

    d, U0, dt, ref = vortex
    U = _run(d, U0, dt, 100, _round(getattr(torch, name)))
    err = _rel_l2(U, ref)
    print("%s stage inputs: relative L2 error after 100 steps %.2e" % (name, err))
    assert np.isfinite(err)
    assert (err <= BUDGET) == within, err
