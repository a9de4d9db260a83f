"""Serving loop on the GPU: continuous batching gives every request the same
result as solving it alone; the f32 bulk form stays within the stated error."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _stream(n=8, steps=10):
    from synth.requests import request_stream

    from paper_1601_07613_amd.serve import Request

    rs = request_stream(n, rate=400.0, k_lo=300, k_hi=4000, seed=9, steps=steps)
    return [Request(rid=r["rid"], arrival=r["arrival"], p=r["p"], steps=r["steps"], spec=r) for r in rs]


def _alone(spec, precision):
    """The request solved alone: its own single-member batch (f64 or f32 form)."""
    import torch

    import paper_1601_07613_amd as dgc
    from paper_1601_07613_amd.serve import GPUExecutor, Request

    ex = GPUExecutor(precision=precision)
    r = Request(rid=spec["rid"], arrival=0.0, p=spec["p"], steps=spec["steps"], spec=spec)
    ex.prepare(r)
    ex.admit(r)
    B = dgc.Batch([r.dev], precision=precision)
    for _ in range(r.steps):
        B.rk_step()
    torch.cuda.synchronize()
    D, U, ws, dt = r.dev
    return D.from_layout(U.cpu().numpy()), r


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batched_serving_results_equal_alone(precision):
    from paper_1601_07613_amd.serve import GPUExecutor, Server

    reqs = _stream()
    st = Server(GPUExecutor(precision=precision), budget_bytes=6_000_000, prep_workers=2).run(reqs)
    print(st.summary())
    assert st.completed == len(reqs) and st.failed == 0
    assert st.max_used <= 6_000_000
    assert st.recaptures >= 2
    # some steps ran as graph replays, the others as eager batched launches
    assert st.graph_captures >= 1
    for r in reqs:
        ref, _ = _alone(r.spec, precision)
        assert np.array_equal(r.result, ref), r.rid


def test_f32_bulk_error_against_f64():
    """f32 form (batched) vs the f64 path for every request: relative L2 <= 1e-6."""
    from paper_1601_07613_amd.serve import GPUExecutor, Server

    reqs = _stream(steps=20)
    Server(GPUExecutor(precision="f32"), budget_bytes=1 << 40, prep_workers=2).run(reqs)
    for r in reqs:
        ref, _ = _alone(r.spec, "f64")
        rel = np.sqrt(((r.result - ref) ** 2).sum() / (ref ** 2).sum())
        assert rel <= 1e-6, (r.rid, rel)


def test_serving_f64_against_cpu_oracle_smallest():
    """The two smallest requests, served in the f64 batched form, against the
    CPU oracle advanced with the same dt."""
    from oracle import dg
    from oracle.mesh import build_mesh
    import synth.requests as sreq
    from paper_1601_07613_amd.serve import GPUExecutor, Server

    reqs = _stream(steps=5)
    Server(GPUExecutor(precision="f64"), budget_bytes=1 << 40, prep_workers=2).run(reqs)
    small = sorted(reqs, key=lambda r: r.spec["n"])[:2]
    for r in small:
        m, U0 = sreq.request_input(r.spec)
        O = build_mesh(m["elem_vert"], m["elem_xyz"])
        d = dg.Discretization(O, r.p)
        _, rr = _alone(r.spec, "f64")
        dt = rr.dev[3]
        U = U0.copy()
        for _ in range(r.steps):
            U = dg.rk3_step(d, U, dt)
        err = np.abs(r.result - U).max() / np.abs(U).max()
        assert err <= 1e-12, (r.rid, err)
