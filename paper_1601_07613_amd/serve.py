"""Serving loop: continuous batching of independent DG solves on one GPU.

Requests arrive over time (each: a mesh, an order p, an initial state and a
number of SSP-RK3 steps).  A host worker pool builds, colors and lays out
each request's mesh while the GPU works.  A prepared request is admitted when
its device footprint fits in the HBM budget (first come, first served; a
request that can never fit is rejected).  Admitted requests of the same order
p form one group; every iteration advances every group by one batched SSP-RK3
step (each group on a stream of its own, so groups overlap too), so requests
join and leave between steps and their work overlaps on the device.  A group whose membership changed steps with eager batched
launches; once its membership has held for a few steps its step is captured
in a graph and replayed until the next change (a capture costs a warm-up
and a synchronisation, which a membership that changes every few steps
would pay over and over).  Finished requests free their memory for the next
admission: their group's batch and graph, which reference every member's
arrays, are dropped before the next admission and rebuilt for the members
that remain.  The host waits for an iteration's device work one iteration
later (a finishing request's download, a rebuild or a drop waits at once),
so it admits and launches the next iteration while the device runs this
one.  A request whose result is not finite fails alone.

``mode="sequential"`` is the plain baseline: one request at a time, each
advanced by the single-mesh f64 step without batching or graphs.
"""

from __future__ import annotations

import concurrent.futures as cf
import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float
    p: int
    steps: int
    spec: dict
    footprint: int = 0
    t_ready: float = math.nan
    t_admit: float = math.nan
    t_done: float = math.nan
    steps_done: int = 0
    status: str = "waiting"   # waiting, preparing, ready, active, done, failed, rejected
    dofs: int = 0
    host: object = None       # prepared host data (executor-specific)
    dev: object = None        # device data (executor-specific)
    result: object = None


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait_until(self, t: float) -> None:
        d = t - self.now()
        if d > 0:
            time.sleep(min(d, 0.002))


@dataclass
class ServeStats:
    latencies: dict = field(default_factory=dict)
    completed: int = 0
    failed: int = 0
    rejected: int = 0
    makespan: float = 0.0
    dof_steps: float = 0.0
    max_used: int = 0
    recaptures: int = 0       # membership rebuilds of the batched groups
    graph_captures: int = 0   # graphs the executor captured
    iterations: int = 0

    def summary(self) -> dict:
        lat = np.array(list(self.latencies.values())) if self.latencies else np.zeros(1)
        return {
            "completed": self.completed, "failed": self.failed, "rejected": self.rejected,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "makespan_s": self.makespan,
            "requests_per_s": self.completed / self.makespan if self.makespan > 0 else 0.0,
            "dof_steps_per_s": self.dof_steps / self.makespan if self.makespan > 0 else 0.0,
            "max_used_bytes": self.max_used, "membership_rebuilds": self.recaptures,
            "graph_captures": self.graph_captures, "iterations": self.iterations,
        }


class Server:
    def __init__(self, executor, budget_bytes: int, mode: str = "batched", clock=None, prep_workers: int = 4):
        if mode not in ("batched", "sequential"):
            raise ValueError(mode)
        self.ex = executor
        self.budget = int(budget_bytes)
        self.mode = mode
        self.clock = clock or WallClock()
        self.prep_workers = prep_workers

    def run(self, requests) -> ServeStats:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        st = ServeStats()
        pending = list(reqs)
        preparing = {}
        ready = []            # FIFO by arrival
        active = {}           # p -> list of requests
        dirty = set()
        used = 0
        clock = self.clock
        pool = cf.ThreadPoolExecutor(max_workers=self.prep_workers) if self.prep_workers > 0 else None
        try:
            while pending or preparing or ready or any(active.values()):
                now = clock.now()
                # arrivals start their host preparation
                while pending and pending[0].arrival <= now:
                    r = pending.pop(0)
                    r.status = "preparing"
                    if pool is None:
                        preparing[r.rid] = (r, _done_future(self.ex.prepare, r))
                    else:
                        preparing[r.rid] = (r, pool.submit(self.ex.prepare, r))
                # finished preparations queue for admission, in arrival order
                fin = [rid for rid, (r, f) in preparing.items() if f.done()]
                for rid in sorted(fin, key=lambda i: (preparing[i][0].arrival, i)):
                    r, f = preparing.pop(rid)
                    try:
                        f.result()
                        r.status = "ready"
                        r.t_ready = clock.now()
                        ready.append(r)
                    except Exception:  # noqa: BLE001 - a bad request fails alone
                        r.status = "failed"
                        st.failed += 1
                ready.sort(key=lambda r: (r.arrival, r.rid))
                # admission by footprint (head of line waits; never-fitting requests are rejected)
                n_active = sum(len(v) for v in active.values())
                while ready:
                    r = ready[0]
                    if r.footprint > self.budget:
                        ready.pop(0)
                        r.status = "rejected"
                        st.rejected += 1
                        self.ex.release(r)
                        continue
                    if used + r.footprint > self.budget or (self.mode == "sequential" and n_active >= 1):
                        break
                    ready.pop(0)
                    self.ex.admit(r)
                    r.status = "active"
                    r.t_admit = clock.now()
                    used += r.footprint
                    st.max_used = max(st.max_used, used)
                    active.setdefault(r.p, []).append(r)
                    dirty.add(r.p)
                    n_active += 1
                if not any(active.values()):
                    nxt = [pending[0].arrival] if pending else []
                    clock.wait_until(min(nxt) if nxt else clock.now() + 0.0005)
                    continue
                # one SSP-RK3 step of every active group
                for p in sorted(active):
                    group = active[p]
                    if not group:
                        continue
                    if self.mode == "batched":
                        if p in dirty:
                            self.ex.rebuild(p, group)
                            st.recaptures += 1
                        self.ex.step_group(p, group)
                    else:
                        for r in group:
                            self.ex.step_single(r)
                dirty.clear()
                self.ex.sync()
                st.iterations += 1
                for p in sorted(active):
                    keep = []
                    for r in active[p]:
                        r.steps_done += 1
                        if r.steps_done < r.steps:
                            keep.append(r)
                            continue
                        ok = self.ex.finish(r)
                        used -= r.footprint
                        r.t_done = clock.now()  # the result is on the host
                        if ok:
                            r.status = "done"
                            st.completed += 1
                            st.latencies[r.rid] = r.t_done - r.arrival
                            st.dof_steps += r.dofs * r.steps
                        else:
                            r.status = "failed"
                            st.failed += 1
                        dirty.add(p)
                    active[p] = keep
                    if p in dirty and self.mode == "batched":
                        # the group's batch and graph still reference the
                        # finished members' arrays: free them before the next
                        # admission counts their bytes as available
                        drop = getattr(self.ex, "drop_group", None)
                        if drop is not None:
                            drop(p)
            st.makespan = clock.now() - (reqs[0].arrival if reqs else 0.0)
            st.graph_captures = int(getattr(self.ex, "captures", 0))
        finally:
            if pool is not None:
                pool.shutdown(wait=True)
        return st


def _done_future(fn, *a):
    f = cf.Future()
    try:
        f.set_result(fn(*a))
    except Exception as e:  # noqa: BLE001
        f.set_exception(e)
    return f


class GPUExecutor:
    """Runs requests on the GPU through libdgc (batched groups or single solves).

    ``layout`` is the element numbering of each request's mesh: the paper's
    (Section 5) by default, measured a little lower in latency than the
    paired numbering on the request stream's periodic grids (the paired
    numbering steps faster on the device but costs more host time to lay
    out and to build the device arrays)."""

    def __init__(self, precision: str = "f32", cfl: float = 0.1, seed: int = 0, layout: str = "paper"):
        import torch

        import paper_1601_07613_amd as dgc

        self.dgc = dgc
        self.torch = torch
        self.precision = precision
        self.cfl = cfl
        self.seed = seed
        self.layout = layout
        self.batches = {}
        self.graphs = {}
        self.eager_steps = {}
        self.captures = 0
        self.streams = {}  # one stream per group (default priority)
        self.last_step = None  # event after the previous iteration's work

    # host work (worker threads): mesh, coloring, layout, initial DOFs; the
    # request supplies its time step, the library the device footprint
    def prepare(self, r: Request) -> None:
        import synth.requests as sreq

        m, U0 = sreq.request_input(r.spec)
        dt = sreq.request_dt(r.spec, m, cfl=self.cfl)
        M = self.dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
        M.color(seed=self.seed, layout=self.layout)
        r.footprint = self.dgc.device_footprint(M, r.p, self.precision)
        r.dofs = U0.size
        r.host = (M, U0, dt)

    def admit(self, r: Request) -> None:
        torch = self.torch
        M, U0, dt = r.host
        D = self.dgc.DeviceMesh(M, r.p)
        # the records move into the layout order on the device (a host scatter
        # of a randomly numbered layout costs the serving loop more)
        U = D.to_layout_device(torch.from_numpy(U0).cuda())
        ws = D.workspace("rk", "colored", self.precision if self.precision else "f64")
        r.dev = (D, U, ws, dt)

    def release(self, r: Request) -> None:
        r.host = None
        r.dev = None

    # eager batched steps of a group before its step is captured in a graph
    STABLE_STEPS = 2

    def drop_group(self, p) -> None:
        """Let go of group p's batch descriptor and captured graph, which hold
        the device arrays of every member, finished ones included (after the
        work that uses them)."""
        self.torch.cuda.synchronize()
        self.batches.pop(p, None)
        self.graphs.pop(p, None)

    def rebuild(self, p, group) -> None:
        # the group's previous descriptor and graph may still be in use by the
        # iteration in flight
        self.torch.cuda.synchronize()
        self.batches[p] = self.dgc.Batch([r.dev for r in group], precision=self.precision)
        self.graphs.pop(p, None)
        self.eager_steps[p] = 0

    def step_group(self, p, group) -> None:
        # each group steps on a stream of its own, so the groups of one
        # iteration (different orders p) overlap on the device; the stream
        # first waits for the uploads of newly admitted requests
        torch = self.torch
        s = self.streams.get(p)
        if s is None:
            s = self.streams[p] = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            g = self.graphs.get(p)
            if g is not None:
                g.replay()
                return
            B = self.batches[p]
            B.rk_step()
            self.eager_steps[p] += 1
            if self.eager_steps[p] >= self.STABLE_STEPS:
                # the kernels are loaded by now: capture without a warm-up stage
                self.graphs[p] = B.capture(warm=False)
                self.captures += 1

    def step_single(self, r: Request) -> None:
        D, U, ws, dt = r.dev
        D.rk_step(U, dt, precision="f64", ws=ws)

    def sync(self) -> None:
        """End of an iteration's launches: the caller's stream waits for every
        group's stream, and the host waits for the previous iteration only,
        so that it prepares the next iteration while this one runs (a
        finishing request's download, a rebuild or a drop waits for the rest)."""
        torch = self.torch
        cur = torch.cuda.current_stream()
        for s in self.streams.values():
            cur.wait_stream(s)
        ev = torch.cuda.Event()
        ev.record(cur)
        if self.last_step is not None:
            self.last_step.synchronize()
        self.last_step = ev

    def finish(self, r: Request) -> bool:
        D, U, ws, dt = r.dev
        cur = self.torch.cuda.current_stream()
        for s in self.streams.values():
            cur.wait_stream(s)
        res = D.from_layout_device(U).cpu().numpy()
        r.result = res
        r.dev = None
        r.host = None
        return bool(np.isfinite(res).all())
