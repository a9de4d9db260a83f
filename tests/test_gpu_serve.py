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


def test_serving_memory_stays_within_budget():
    """Device memory held by the served requests (torch's allocated bytes
    after every iteration, minus what was allocated before) never exceeds the
    budget plus the batch descriptors: finished members are released before
    the next admission."""
    import torch

    from paper_1601_07613_amd.serve import GPUExecutor, Server

    class Watch(GPUExecutor):
        peak = 0

        def sync(self):
            super().sync()
            Watch.peak = max(Watch.peak, torch.cuda.memory_allocated() - base)

    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    budget = 6_000_000
    ex = Watch(precision="f32")
    st = Server(ex, budget_bytes=budget, prep_workers=2).run(_stream(steps=12))
    assert st.completed == 8
    descriptors = sum(B.dev.numel() for B in ex.batches.values()) + 3 * 65536
    print("peak allocated over the base", Watch.peak, "budget", budget)
    assert 0 < Watch.peak <= budget + descriptors


def test_serving_real_stream_smallest_eight_against_oracle():
    """The eight smallest requests of the 256-request stream (Poisson
    arrivals at 50/s, seed 5, 100 SSP-RK3 steps each, p in {1, 2, 3}), served
    together in the f64 batched form, against the CPU oracle advanced with
    each request's own time step (the oracle runs in a pool of host
    processes)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    from synth.requests import request_stream

    from paper_1601_07613_amd.serve import GPUExecutor, Request, Server
    from tests.helpers import oracle_serve_request

    rs = request_stream(256, rate=50.0, seed=5, steps=100)
    small = sorted(rs, key=lambda r: (r["n"], r["rid"]))[:8]
    assert {r["p"] for r in small} == {1, 2, 3}
    with cf.ProcessPoolExecutor(max_workers=8, mp_context=mp.get_context("spawn")) as pool:
        futs = [pool.submit(oracle_serve_request, r) for r in small]
        t0 = min(r["arrival"] for r in small)
        reqs = [Request(rid=r["rid"], arrival=(r["arrival"] - t0) * 0.01, p=r["p"], steps=r["steps"], spec=r)
                for r in small]
        st = Server(GPUExecutor(precision="f64"), budget_bytes=1 << 40, prep_workers=4).run(reqs)
        assert st.completed == 8
        refs = [f.result() for f in futs]
    for r, ref in zip(reqs, refs):
        assert np.isfinite(ref).all()
        err = np.abs(r.result - ref).max() / np.abs(ref).max()
        print("request", r.rid, "K", ref.shape[0], "p", r.p, "rel err", err, flush=True)
        assert err <= 1e-12, (r.rid, err)


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
        dt = sreq.request_dt(r.spec, m)
        U = U0.copy()
        for _ in range(r.steps):
            U = dg.rk3_step(d, U, dt)
        err = np.abs(r.result - U).max() / np.abs(U).max()
        assert err <= 1e-12, (r.rid, err)
