"""Benchmark of the colored DG surface pass on one MI355X.

Workload (default): Delaunay triangulation of ~500 k seeded Poisson-disc
points in the unit square (~1 M triangles, ~1.5 M edges), reflective walls,
2D Euler with p = 2 (N_p = 6, M = 4), shock-tube state with seeded noise in
the higher modes, float64.  One step = one full surface right-hand side over
all colors (3 launches, one per color, ordered on the stream).

Prints one JSON line with the metric (surface DOF-updates/s), the roofline
of the surface kernel (algorithmic HBM bytes / measured time vs 8 TB/s),
the same pass with the atomic and buffered-gather variants, the volume term
and one SSP-RK3 step for context, and the CPU oracle timed on the host.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ABLATION_ROUNDS = 5
PROFILES = {
    "delaunay": os.path.join(ROOT, "profiles", "surface_colored_team_prefetch_delaunay996k_p2_f64.md"),
    "tets": os.path.join(ROOT, "profiles", "surface_colored_mode_team_kuhn64_tets_p1_f64.md"),
}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1601_07613_amd", "csrc", "kernels", f)
                  for f in ("surface.hpp", "euler_dev.hpp", "team.hpp", "device_api.hip")]


def profiled_traffic(args, launch):
    """HBM bytes per launch measured by rocprofv3 counters for the committed
    kernel on the default configuration of this workload, or None when the
    kernel source changed since the profile (or the configuration differs)."""
    import hashlib
    import re

    same_launch = (launch.get("form") in ("default", "team_prefetch" if args.workload == "delaunay" else "default")
                   and launch.get("block") in (0, 256) and not launch.get("xcd_remap"))
    default = (same_launch and args.seed == 2 and args.layout == "paired" and
               ((args.workload == "delaunay" and args.points == 500_000 and args.p == 2) or
                (args.workload == "tets" and args.tet_n == 64 and args.p == 1)))
    if not default:
        return None
    try:
        text = open(PROFILES[args.workload]).read()
    except OSError:
        return None
    h = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SOURCES)).hexdigest()[:16]
    m_sha = re.search(r"kernel_source_sha256_16: ([0-9a-f]{16})", text)
    m_tr = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    if not m_sha or not m_tr or m_sha.group(1) != h:
        return None
    return int(m_tr.group(1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu() -> dict:
    """The host's CPU model string and logical CPU count (as the OS reports
    them; a container may be limited to fewer)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def algorithmic_bytes(n_face: int, n_interior: int, rec: int, elt: int, dim: int) -> int:
    """Bytes one colored pass must move: per face side, read the DOF record and
    read + write the RHS record; per face, its geometry (dim + 3 doubles),
    both element ids (2 x int32) and both table codes (2 x uint8)."""
    sides = n_face + n_interior
    return sides * 3 * rec * elt + n_face * ((dim + 3) * 8 + 8 + 2)


def compact_bytes(n_face: int, n_interior: int, n_elem: int, nvar: int, n_p: int, max_slots: int, n_qf: int,
                  elt: int, dim: int) -> int:
    """Bytes the compact buffered variant must move: the face pass reads both
    DOF records, the face geometry, ids and codes and writes one record of
    n_qf * nvar + 1 values; the element pass reads the element's slots and
    sqrt(det J), the records of its faces, and reads + writes its RHS."""
    rec = nvar * n_p * elt
    frec = (n_qf * nvar + 1) * elt
    face = (n_face + n_interior) * rec + n_face * ((dim + 3) * 8 + 8 + 2 + frec)
    elem = n_elem * (max_slots * 4 + 8 + 2 * rec) + (n_face + n_interior) * frec
    return face + elem


def timed(fn, steps, warmup, stream):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    t0.record(stream)
    for _ in range(steps):
        fn()
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    return t0.elapsed_time(t1) / steps, wall


def extra_workloads(dgc, synth, torch, steps, warmup, log):
    """The other configurations, reported beside the headline: small periodic
    mesh latency (c0), periodic Kuhn tetrahedra in f64 and f32 with the f32
    form's error (c2), the adaptively refined nonconforming mesh (c3)."""
    from paper_1601_07613_amd.tune import autotune, time_call

    out = {}
    stream = torch.cuda.current_stream()

    def surf_stats(D, K, E, nb, elt, precision, variants=(), tune=False):
        U = torch.zeros((K, D.n_var, D.n_p), dtype=torch.float64 if elt == 8 else torch.float32, device="cuda")
        U[:, 0, 0] = 1.0
        U[:, -1, 0] = 2.5
        rhs = torch.zeros_like(U)
        launch = None
        if tune:
            # the launch autotuner on this mesh, as for the headline
            launch, _ = autotune(D, U, rhs, precision=precision)
        ms = time_call(lambda: D.surface_rhs(U, rhs, "colored", precision), reps=steps, warmup=warmup)
        ab = algorithmic_bytes(E, E - nb, D.n_var * D.n_p, elt, D.dim)
        res = {"colored_us": ms * 1e3, "dof_updates_per_s": K * D.n_var * D.n_p / (ms * 1e-3),
               "algorithmic_GBs": ab / (ms * 1e-3) / 1e9, "frac_of_8TBs": ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "launch": launch or "default"}
        # the other variants of the same pass (Section 1's alternatives)
        for v in variants:
            ws = D.workspace("surface", v, precision) if v in ("gather", "compact") else None
            res[v + "_us"] = time_call(lambda: D.surface_rhs(U, rhs, v, precision, ws=ws), reps=steps,
                                       warmup=warmup) * 1e3
            del ws
        return res

    # c0: 16 x 16 x 2 periodic triangles, p = 1 (latency-bound)
    m = synth.periodic_tri(16, seed=1)
    M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    M.color(seed=1)
    D = dgc.DeviceMesh(M, 1)
    U = torch.zeros((D.K, 4, D.n_p), dtype=torch.float64, device="cuda")
    U[:, 0, 0] = 0.1
    U[:, 3, 0] = 0.25
    rhs = torch.zeros_like(U)
    ws = D.workspace("rk", "colored")
    B = dgc.Batch([(D, U, ws, 1e-9)])
    g = B.capture(steps=10)
    forms = {}
    for rf in ("block", "fused", "fused_volume", "separate"):
        D.set_rk_form(rf)
        forms[rf] = time_call(lambda: D.rk_step(U, 1e-9, ws=ws), reps=100, warmup=10) * 1e3
    D.set_rk_form("default")
    out["c0_periodic512_p1"] = {
        "surface_pass_us": time_call(lambda: D.surface_rhs(U, rhs), reps=200, warmup=20) * 1e3,
        "rk3_step_us": time_call(lambda: D.rk_step(U, 1e-9, ws=ws), reps=100, warmup=10) * 1e3,
        "rk3_step_by_form_us": forms,
        "rk3_step_graph_us": time_call(g.replay, reps=20, warmup=3) * 1e3 / 10,
    }
    del g, B
    log("c0: %s" % out["c0_periodic512_p1"])

    # c2: 64^3 x 6 periodic Kuhn tetrahedra, p = 1, f64 and f32
    t = synth.kuhn_tets(64, seed=3)
    T = dgc.Mesh.build(t["elem_vert"], t["elem_xyz"])
    cs = T.color(seed=0, layout="paired")
    DT = dgc.DeviceMesh(T, 1)
    info = DT.info
    # the variants in the default launch; then the colored pass autotuned
    r64d = surf_stats(DT, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64",
                      variants=("atomic", "gather", "compact"))
    r64 = surf_stats(DT, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64", tune=True)
    r32 = surf_stats(DT, info["n_elem"], info["n_face"], info["n_boundary"], 4, "f32", tune=True)
    DT.set_launch("pair_team")
    r64p = surf_stats(DT, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64")
    DT.set_launch("thread")
    r64t = surf_stats(DT, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64")
    DT.set_launch("team_prefetch")
    r64v = surf_stats(DT, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64")
    DT.set_launch("default")
    # f32 form error: 10 SSP-RK3 steps of the density wave from the same state
    meas = synth.element_measure(t["elem_xyz"])
    st = synth.density_wave_states(synth.element_centroid(t["elem_xyz"]))
    U0 = synth.perturbed_dofs(meas, st, DT.n_p, eps=0.0)
    h = 1.0 / 64
    dt = 0.1 * 0.2 * h / (3 ** 0.5 + 1.2)
    Ua = torch.from_numpy(DT.to_layout(U0)).cuda()
    Ub = Ua.clone()
    wa = DT.workspace("rk", "colored", "f64")
    wb = DT.workspace("rk", "colored", "f32")
    for _ in range(10):
        DT.rk_step(Ua, dt, precision="f64", ws=wa)
        DT.rk_step(Ub, dt, precision="f32", ws=wb)
    torch.cuda.synchronize()
    diff = ((Ub - Ua) ** 2).sum(dim=(0, 2)).sqrt() / (Ua ** 2).sum(dim=(0, 2)).sqrt()
    rk64 = time_call(lambda: DT.rk_step(Ua, dt, precision="f64", ws=wa), reps=20, warmup=3)
    rk32 = time_call(lambda: DT.rk_step(Ub, dt, precision="f32", ws=wb), reps=20, warmup=3)
    rk_forms = {}
    for rf in ("fused_volume", "fused", "separate"):
        DT.set_rk_form(rf)
        rk_forms["f64_" + rf] = time_call(lambda: DT.rk_step(Ua, dt, precision="f64", ws=wa), reps=20,
                                          warmup=3) * 1e3
        rk_forms["f32_form_" + rf] = time_call(lambda: DT.rk_step(Ub, dt, precision="f32", ws=wb), reps=20,
                                               warmup=3) * 1e3
    DT.set_rk_form("default")
    del DT, Ua, Ub, wa, wb
    # the paper's own layout of the same coloring (Section 5), autotuned too
    T.set_colors(T.export("color"), layout="paper")
    DTp = dgc.DeviceMesh(T, 1)
    r64paper = surf_stats(DTp, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64", tune=True)
    DTp.set_launch("default")
    r64paperd = surf_stats(DTp, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64")
    out["c2_kuhn64_tets_p1"] = {
        "n_elem": info["n_elem"], "n_face": info["n_face"], "n_colors": info["n_colors"], "layout": "paired",
        "color_ms": cs["color_ms"], "f64": r64, "f32": r32, "f64_default_launch": r64d, "f64_pair_team_form": r64p,
        "f64_thread_form": r64t, "f64_variable_team_form": r64v,
        "f64_paper_layout": r64paper, "f64_paper_layout_default_launch": r64paperd,
        "rk3_step_us": {"f64": rk64 * 1e3, "f32_form": rk32 * 1e3},
        "rk3_step_by_form_us": rk_forms,
        "f32_form_rel_L2_after_10_steps": [float(x) for x in diff.cpu()],
    }
    log("c2: %s" % out["c2_kuhn64_tets_p1"])
    del DTp, T

    # quadrilaterals: 1024 x 1024 periodic parallelograms, p = 2 (N_p = 9), four
    # colors, paired layout (the paper's layout of the same coloring beside it)
    g = synth.quad_grid(1024, jitter=0.1, seed=6)
    Qm = dgc.Mesh.build(g["elem_vert"], g["elem_xyz"])
    qs = Qm.color(seed=0)
    DQp = dgc.DeviceMesh(Qm, 2)
    info = DQp.info
    rqp = surf_stats(DQp, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64", tune=True)
    del DQp
    Qm.set_colors(Qm.export("color"), layout="paired")
    DQ = dgc.DeviceMesh(Qm, 2)
    rq = surf_stats(DQ, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64", tune=True)
    rq32 = surf_stats(DQ, info["n_elem"], info["n_face"], info["n_boundary"], 4, "f32", tune=True)
    Uq = torch.zeros((DQ.K, 4, DQ.n_p), dtype=torch.float64, device="cuda")
    Uq[:, 0, 0] = 1.0
    Uq[:, 3, 0] = 2.5
    wq = DQ.workspace("rk", "colored")
    out["quads_1024sq_p2"] = {
        "n_elem": info["n_elem"], "n_face": info["n_face"], "n_colors": info["n_colors"],
        "color_ms": qs["color_ms"], "conflicts_after_greedy": qs["conflicts_after_greedy"], "layout": "paired",
        "f64": rq, "f32": rq32, "f64_paper_layout": rqp,
        "rk3_step_us": time_call(lambda: DQ.rk_step(Uq, 1e-7, ws=wq), reps=10, warmup=2) * 1e3,
    }
    rk_forms = {}
    for rf in ("fused_volume", "fused"):
        DQ.set_rk_form(rf)
        rk_forms[rf] = time_call(lambda: DQ.rk_step(Uq, 1e-7, ws=wq), reps=10, warmup=2) * 1e3
    DQ.set_rk_form("default")
    wqc = DQ.workspace("rk", "compact")
    rk_forms["compact_variant"] = time_call(lambda: DQ.rk_step(Uq, 1e-7, variant="compact", ws=wqc), reps=10,
                                            warmup=2) * 1e3
    del wqc
    out["quads_1024sq_p2"]["rk3_step_by_form_us"] = rk_forms
    log("quads: %s" % out["quads_1024sq_p2"])
    del DQ, Qm, Uq, wq

    # the same grid numbered in a random order (an unstructured generator's
    # numbering, Table 2's conflict fraction), paper layout and its Morton and
    # paired extensions
    gs = synth.shuffle_elements(g, seed=7)
    Qs = dgc.Mesh.build(gs["elem_vert"], gs["elem_xyz"])
    qss = Qs.color(seed=0)
    res = {"color_ms": qss["color_ms"], "conflicts_after_greedy": qss["conflicts_after_greedy"],
           "conflict_fraction": qss["conflicts_after_greedy"] / Qs.info()["n_face"], "swaps": qss["swaps"],
           "loop_breaks": qss["loop_breaks"]}
    for lay in ("paper", "paper_sfc", "paired"):
        Qs.set_colors(Qs.export("color"), layout=lay)
        DS = dgc.DeviceMesh(Qs, 2)
        info = DS.info
        res["f64_" + lay] = surf_stats(DS, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64", tune=True)
        del DS
    out["quads_1024sq_random_numbering_p2"] = res
    log("quads, random numbering: %s" % res)
    del Qs, gs

    # mixed: the same grid with the cells within 0.3 of the center split into
    # triangles, p = 2, paired layout (the paper's layout beside it)
    g = synth.hybrid_grid(1024, jitter=0.1, seed=6, radius=0.3)
    Hm = dgc.Mesh.build(g["elem_vert"], g["elem_xyz"])
    hs = Hm.color(seed=0)
    DH = dgc.DeviceMesh(Hm, 2)
    info = DH.info
    rhp = surf_stats(DH, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64", tune=True)
    del DH
    Hm.set_colors(Hm.export("color"), layout="paired")
    DH = dgc.DeviceMesh(Hm, 2)
    rh = surf_stats(DH, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64", tune=True)
    out["mixed_1024sq_p2"] = {"n_elem": info["n_elem"], "n_tri": g["n_tri"], "n_quad": g["n_quad"],
                              "n_face": info["n_face"], "n_colors": info["n_colors"], "color_ms": hs["color_ms"],
                              "conflicts_after_greedy": hs["conflicts_after_greedy"], "layout": "paired", "f64": rh,
                              "f64_paper_layout": rhp}
    log("mixed: %s" % out["mixed_1024sq_p2"])
    del DH, Hm

    # c3: 128 x 128 x 2 periodic base refined to level 3 within r < 0.15, p = 2
    m = synth.periodic_tri(128, jitter=0.0, seed=4)
    A = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    A.color(seed=0)
    t0 = time.perf_counter()
    for lvl in range(1, 4):
        xyz = A.export("elem_xyz").reshape(-1, 3, 2)
        lev = A.export("elem_level")
        A, _ = A.refine(synth.refine_flags(xyz, lev, lvl - 1, radius=0.15))
    refine_s = time.perf_counter() - t0
    DA = dgc.DeviceMesh(A, 2)
    info = DA.info
    r = surf_stats(DA, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64", tune=True)
    # the same leaves and colors in the paired numbering
    A.set_colors(A.export("color"), layout="paired")
    DP = dgc.DeviceMesh(A, 2)
    rp = surf_stats(DP, info["n_elem"], info["n_face"], info["n_boundary"], 8, "f64", tune=True)
    del DP
    out["c3_amr_level3_p2"] = {"n_elem": info["n_elem"], "n_face": info["n_face"], "n_colors": info["n_colors"],
                               "refine_s": refine_s, "f64": r, "f64_paired_layout": rp}
    log("c3: %s" % out["c3_amr_level3_p2"])
    del DA, A

    # c3 dynamic: the same base, a feature moving across the torus; every 10
    # SSP-RK3 steps coarsen behind it and refine one level (up to 3) around it,
    # moving the solution on the device; 60 steps, p = 2
    from paper_1601_07613_amd.amr import AdaptiveRun

    A = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    A.color(seed=0)
    DA = dgc.DeviceMesh(A, 2)
    cen = synth.element_centroid(m["elem_xyz"])
    U0 = synth.perturbed_dofs(synth.element_measure(m["elem_xyz"]), synth.isentropic_vortex(cen, 0.0), DA.n_p,
                              eps=0.0)
    dt_dyn = 0.1 * (1.0 / 128 / 8) / 3.0

    def crit(xyz, lev, tt):
        return synth.adapt_flags(xyz, lev, (0.5 + 100.0 * tt, 0.5 + 60.0 * tt), 0.15, 0.2, max_level=3)

    run = AdaptiveRun(A, 2, torch.from_numpy(DA.to_layout(U0)).cuda(), dt_dyn, crit, every=10)
    t0 = time.perf_counter()
    run.run(60)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_us = time_call(lambda: run.D.rk_step(run.U, dt_dyn, ws=run.ws), reps=5, warmup=1) * 1e3
    log_ = run.log
    out["c3_dynamic_p2"] = {
        "adapt_cycles": len(log_), "steps": 60, "wall_s": wall,
        "n_elem_range": [min(r["n_elem"] for r in log_), max(r["n_elem"] for r in log_)],
        "merged_total": sum(r["merged"] for r in log_), "refined_total": sum(r["refined"] for r in log_),
        "max_colors": max(r["n_colors"] for r in log_),
        "host_adapt_ms_mean": sum(r["host_ms"] for r in log_) / len(log_),
        "device_transfer_us_mean": sum(r["transfer_us"] for r in log_) / len(log_),
        "rk3_step_us_final_mesh": step_us,
        "finite": bool(torch.isfinite(run.U).all()),
    }
    log("c3 dynamic: %s" % out["c3_dynamic_p2"])
    del run, DA, A

    # c4: serving -- 256 solves, Poisson arrivals at 50/s, 100 SSP-RK3 steps each
    from synth.requests import request_stream
    from paper_1601_07613_amd.serve import GPUExecutor, Request, Server

    def reqs(saturated=False):
        rs = request_stream(256, rate=50.0, seed=5, steps=100)
        return [Request(rid=r["rid"], arrival=0.0 if saturated else r["arrival"], p=r["p"], steps=r["steps"],
                        spec=r) for r in rs]

    serving = {}
    results = {}
    for name, prec, mode, budget, sat in (("batched_f32_budget512MB", "f32", "batched", 512 << 20, False),
                                          ("batched_f32_full", "f32", "batched", 200 << 30, False),
                                          ("plain_f64_sequential", "f64", "sequential", 200 << 30, False),
                                          ("batched_f32_saturated", "f32", "batched", 200 << 30, True),
                                          ("plain_f64_saturated", "f64", "sequential", 200 << 30, True)):
        rs = reqs(sat)
        st = Server(GPUExecutor(precision=prec), budget_bytes=budget, mode=mode, prep_workers=16).run(rs)
        serving[name] = st.summary()
        results[name] = {r.rid: r.result for r in rs if r.status == "done"}
        log("c4 %s: %s" % (name, serving[name]))
    # error of the served f32 bulk form against the plain f64 path, per request
    a, b = results["batched_f32_budget512MB"], results["plain_f64_sequential"]
    rel = np.array([np.sqrt(((a[i] - b[i]) ** 2).sum() / (b[i] ** 2).sum()) for i in sorted(set(a) & set(b))])
    serving["f32_served_rel_L2_vs_f64"] = {"requests": int(rel.size), "max": float(rel.max()),
                                           "median": float(np.median(rel)), "budget": 1e-6}
    log("c4 f32 served error: %s" % serving["f32_served_rel_L2_vs_f64"])
    out["c4_serving_256"] = serving
    return out


SWEEP_SIDES = {
    # side counts of the paper's meshes A-E (Table 1, Table 2, Table 3)
    "triangles": (14775, 59547, 236372, 942162, 3774165),
    "quadrilaterals": (8888, 35396, 141076, 563108, 2249162),
    "tetrahedra": (14937, 102438, 720736),
}


def coloring_sweep(dgc, synth, log):
    """Host coloring at sizes like the paper's meshes A-E (Figure 9, Table 8):
    for each element family and size, the conflicts left by the greedy stage,
    the coloring time and the renumbering + reordering time, against the
    number of sides.  Meshes: jittered-lattice Delaunay triangles, periodic
    parallelograms and periodic Kuhn tetrahedra (even grids, which have
    four-colorings), each numbered in a seeded random order (an unstructured
    generator's numbering; see shuffle_elements)."""
    out = {}
    for fam, sizes in SWEEP_SIDES.items():
        rows = []
        for sides in sizes:
            if fam == "triangles":
                m = synth.lattice_delaunay(sides // 3, seed=7)
            elif fam == "quadrilaterals":
                # an even periodic grid: an odd one has no four-coloring
                m = synth.quad_grid(2 * max(2, int(round((sides / 8) ** 0.5))), seed=6)
            else:
                m = synth.kuhn_tets(2 * max(1, int(round((sides / 96) ** (1 / 3)))), seed=3)
            m = synth.shuffle_elements(m, seed=1)
            t = time.perf_counter()
            Mx = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
            build_ms = (time.perf_counter() - t) * 1e3
            st = Mx.color(seed=0)
            E = Mx.info()["n_face"]
            rows.append({"sides": E, "elements": len(m["elem_vert"]), "conflicts_after_greedy": st["conflicts_after_greedy"],
                         "conflict_fraction": st["conflicts_after_greedy"] / E, "color_ms": st["color_ms"],
                         "layout_ms": st["layout_ms"], "build_ms": build_ms, "n_colors": st["n_colors"]})
            log("sweep %s: %s" % (fam, rows[-1]))
            del Mx, m
        out[fam] = rows
    return out


def oracle_pool(m, U, p, log):
    """The oracle's surface term over a pool of host processes, in a child
    interpreter that never touches the GPU; ``None`` if it fails."""
    import subprocess
    import tempfile

    workers = max(1, min(16, os.cpu_count() or 1))
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "input.npz")
        np.savez(path, elem_vert=m["elem_vert"], elem_xyz=m["elem_xyz"], U=U, p=p)
        try:
            r = subprocess.run([sys.executable, "-m", "oracle.pool_timing", path, str(workers), "2"], cwd=ROOT,
                               capture_output=True, text=True, timeout=300)
        except subprocess.TimeoutExpired:
            log("cpu oracle pool: timed out")
            return None
    if r.returncode != 0:
        log("cpu oracle pool failed: %s" % r.stderr[-500:])
        return None
    res = json.loads(r.stdout.strip().splitlines()[-1])
    dof = U.size
    log("cpu oracle pool: %.2f s per surface term on %d processes" % (res["seconds"], res["workers"]))
    return {"value": dof / res["seconds"], "unit": "DOF-updates/s", "cores": res["workers"], "kind": "oracle",
            "sample": "the same surface term split into %d element chunks over %d host processes (faces on chunk "
                      "borders evaluated by both sides), %d repetitions" % (4 * res["workers"], res["workers"],
                                                                             res["reps"]),
            "matches_single_process": res["matches_single_process"]}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=["delaunay", "tets", "quads"], default="delaunay",
                    help="delaunay: ~1M triangles, p=2 (the headline); tets: 64^3 x 6 Kuhn tetrahedra, p=1; "
                         "quads: 1024^2 periodic parallelograms, p=2")
    ap.add_argument("--points", type=int, default=500_000)
    ap.add_argument("--tet-n", type=int, default=64)
    ap.add_argument("--p", type=int, default=None)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--only", choices=["all", "colored", "volume", "rk", "batch", "sweep"], default="all",
                    help="'colored' times the colored pass only, 'volume' the volume-term forms only, 'rk' the "
                         "SSP-RK3 step forms only, 'batch' a batched SSP-RK3 step of 8 periodic meshes of "
                         "125k triangles (for profiling), 'sweep' the host coloring sweep only")
    ap.add_argument("--variant", choices=["colored", "atomic", "gather", "compact"], default="colored",
                    help="with --only colored: time this variant of the surface pass instead")
    ap.add_argument("--rk-form", choices=["default", "fused_volume", "fused", "separate"], default="default",
                    help="SSP-RK3 step form timed by --only rk")
    ap.add_argument("--form", choices=["auto", "default", "team", "team_prefetch", "thread", "team_stream", "mode_team",
                                       "pair_team"], default="auto",
                    help="face-kernel form; 'auto' runs the launch autotuner before timing")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--xcd-remap", action="store_true")
    ap.add_argument("--layout", choices=["paper", "paper_sfc", "paired", "renumber", "none"], default="paired",
                    help="element numbering and face order: the paper's (Section 5), or the paired extension "
                         "(first-color pairs in blocks of 16, Morton order; the default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-pool", action="store_true",
                    help="skip the oracle timed over a pool of host processes")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (HBM counter calibration)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        return 2

    import torch

    import paper_1601_07613_amd as dgc
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2

    if args.only == "sweep":
        print(json.dumps({"coloring_sweep": coloring_sweep(dgc, synth, log)}))
        return 0

    if args.calibrate_copy:
        # 1 GiB read + 1 GiB written per launch: the reference for FETCH_SIZE / WRITE_SIZE
        n = (1 << 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 5}))
        return 0

    from paper_1601_07613_amd.tune import autotune, time_call

    if args.only == "batch":
        # 8 periodic jittered meshes of 250 x 250 x 2 triangles, one batch
        p = 2 if args.p is None else args.p
        prec = "f32"
        members = []
        for i in range(8):
            mb = synth.periodic_tri(250, seed=10 + i)
            Mb = dgc.Mesh.build(mb["elem_vert"], mb["elem_xyz"])
            Mb.color(seed=i, layout="paired")
            Db = dgc.DeviceMesh(Mb, p)
            st = synth.density_wave_states(synth.element_centroid(mb["elem_xyz"]), vel=(0.5, 0.3))
            Ub = synth.perturbed_dofs(synth.element_measure(mb["elem_xyz"]), st, Db.n_p, eps=0.01, seed=i)
            members.append((Db, torch.from_numpy(Db.to_layout(Ub)).cuda(), Db.workspace("rk", "colored", prec),
                            1e-5))
        B = dgc.Batch(members, precision=prec)
        t_ms = timed(B.rk_step, args.steps, args.warmup, torch.cuda.current_stream())[0]
        K = sum(D.K for D, _, _, _ in members)
        log("batched %s step, %d meshes, %d triangles, p = %d: %.1f us" % (prec, len(members), K, p, t_ms * 1e3))
        print(json.dumps({"batched_rk3_step_us": t_ms * 1e3, "precision": prec, "n_mesh": len(members),
                          "n_elem": K, "p": p}))
        return 0

    t = time.perf_counter()
    if args.workload == "delaunay":
        m = synth.poisson_delaunay(args.points, seed=args.seed)
        p = 2 if args.p is None else args.p
    elif args.workload == "quads":
        m = synth.quad_grid(1024, jitter=0.1, seed=6)
        p = 2 if args.p is None else args.p
    else:
        m = synth.kuhn_tets(args.tet_n, seed=3)
        p = 1 if args.p is None else args.p
    args.p = p
    gen_s = time.perf_counter() - t
    log("mesh generated: K=%d in %.1fs" % (len(m["elem_vert"]), gen_s))
    t = time.perf_counter()
    M = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
    build_s = time.perf_counter() - t
    cst = M.color(seed=0, layout=args.layout)
    colors = M.export("color")
    meas = synth.element_measure(m["elem_xyz"])
    cen = synth.element_centroid(m["elem_xyz"])
    st = synth.shock_tube_states(cen) if args.workload == "delaunay" else synth.density_wave_states(cen)
    stream = torch.cuda.current_stream()
    log("host preprocessing: build %.2fs, color %.0f ms, layout %.0f ms" % (build_s, cst["color_ms"], cst["layout_ms"]))

    def device_mesh(layout):
        M.set_colors(colors, layout=layout)
        D = dgc.DeviceMesh(M, p)
        U = synth.perturbed_dofs(meas, st, D.n_p, eps=0.01, seed=args.seed + 100)
        Ug = torch.from_numpy(D.to_layout(U)).cuda()
        return D, U, Ug, torch.zeros_like(Ug)

    D, U, Ug, rhs = device_mesh(args.layout)
    info = D.info
    K, E, nb = info["n_elem"], info["n_face"], info["n_boundary"]
    rec = D.n_var * D.n_p
    ab = algorithmic_bytes(E, E - nb, rec, 8, D.dim)
    dof = K * D.n_var * D.n_p

    if args.only == "volume":
        # each volume-term form, back to back (for counter runs of one kernel)
        res = {}
        for vf in ("valu", "team", "mfma"):
            D.set_volume_form(vf)
            res[vf + "_us"] = timed(lambda: D.volume_rhs(Ug, rhs), args.steps, args.warmup, stream)[0] * 1e3
        log("volume forms: %s" % res)
        print(json.dumps({"volume_forms_us": res, "n_elem": K, "p": args.p}))
        return 0

    if args.only == "rk":
        # SSP-RK3 steps of one form and variant (for counter runs of the step's kernels)
        D.set_rk_form(args.rk_form)
        if args.form != "auto":
            D.set_launch(args.form, args.block, args.xcd_remap)
        rv = args.variant if args.variant in ("colored", "compact") else "colored"
        ws = D.workspace("rk", rv)
        Ur = Ug.clone()
        # clocks up: ~0.25 s of steps before the measurement
        time_call(lambda: D.rk_step(Ur, 1e-7, variant=rv, ws=ws), reps=200, warmup=5)
        t_ms = timed(lambda: D.rk_step(Ur, 1e-7, variant=rv, ws=ws), args.steps, args.warmup, stream)[0]
        log("rk3 step (%s, %s): %.1f us" % (args.rk_form, rv, t_ms * 1e3))
        print(json.dumps({"rk3_step_us": t_ms * 1e3, "rk_form": args.rk_form, "variant": rv, "n_elem": K,
                          "p": args.p}))
        return 0

    # clocks up: run the pass for ~0.5 s before any measurement
    time_call(lambda: D.surface_rhs(Ug, rhs, "colored"), reps=200, warmup=5)
    if args.form == "auto":
        best, sweep = autotune(D, Ug, rhs)
        log("autotuned launch: %s" % best)
    else:
        D.set_launch(args.form, args.block, args.xcd_remap)
        best, sweep = {"form": args.form, "block": args.block, "xcd_remap": args.xcd_remap}, []

    if args.variant != "colored":
        # another variant of the same pass (for counter runs of its kernels)
        wsv = D.workspace("surface", args.variant) if args.variant in ("gather", "compact") else None
        t_ms = timed(lambda: D.surface_rhs(Ug, rhs, args.variant, ws=wsv), args.steps, args.warmup, stream)[0]
        log("%s pass: %.1f us" % (args.variant, t_ms * 1e3))
        print(json.dumps({"variant": args.variant, "pass_us": t_ms * 1e3, "n_elem": K, "p": args.p}))
        return 0
    ms, wall = timed(lambda: D.surface_rhs(Ug, rhs, "colored"), args.steps, args.warmup, stream)
    log("colored pass: %.1f us (wall %.2fs for %d steps)" % (ms * 1e3, wall, args.steps))
    value = dof / (ms * 1e-3)
    achieved = ab / (ms * 1e-3) / 1e9

    extra = {}
    if args.only == "all":
        for cfg, t_ms in sweep:
            extra["colored_%s_b%d%s_us" % (cfg["form"], cfg["block"], "_xcd" if cfg["xcd_remap"] else "")] = t_ms * 1e3
        ws = D.workspace("surface", "gather")
        extra["atomic_us"] = timed(lambda: D.surface_rhs(Ug, rhs, "atomic"), args.steps, args.warmup, stream)[0] * 1e3
        extra["gather_us"] = timed(lambda: D.surface_rhs(Ug, rhs, "gather", ws=ws), args.steps, args.warmup,
                                   stream)[0] * 1e3
        del ws
        wsc = D.workspace("surface", "compact")
        extra["compact_us"] = timed(lambda: D.surface_rhs(Ug, rhs, "compact", ws=wsc), args.steps, args.warmup,
                                    stream)[0] * 1e3
        extra["compact_algorithmic_bytes"] = compact_bytes(E, E - nb, K, D.n_var, D.n_p, info["max_slots"],
                                                           D.tinfo["n_qf"], 8, D.dim)
        del wsc
        extra["volume_us"] = timed(lambda: D.volume_rhs(Ug, rhs), args.steps, args.warmup, stream)[0] * 1e3
        if D.dim == 2:
            for vf in ("valu", "mfma", "team"):
                D.set_volume_form(vf)
                extra["volume_%s_us" % vf] = timed(lambda: D.volume_rhs(Ug, rhs), args.steps, args.warmup,
                                                   stream)[0] * 1e3
            D.set_volume_form("default")
        wsr = D.workspace("rk", "colored")
        Ur = Ug.clone()
        extra["rk3_step_us"] = timed(lambda: D.rk_step(Ur, 1e-7, ws=wsr), max(args.steps // 5, 3), 2, stream)[0] * 1e3
        D.set_rk_form("separate")
        extra["rk3_step_separate_combine_us"] = timed(lambda: D.rk_step(Ur, 1e-7, ws=wsr), max(args.steps // 5, 3), 2,
                                                      stream)[0] * 1e3
        D.set_rk_form("fused")
        extra["rk3_step_fused_combine_us"] = timed(lambda: D.rk_step(Ur, 1e-7, ws=wsr), max(args.steps // 5, 3), 2,
                                                   stream)[0] * 1e3
        D.set_rk_form("fused_volume")
        extra["rk3_step_fused_volume_us"] = timed(lambda: D.rk_step(Ur, 1e-7, ws=wsr), max(args.steps // 5, 3), 2,
                                                  stream)[0] * 1e3
        wsrc = D.workspace("rk", "compact")
        extra["rk3_step_compact_us"] = timed(lambda: D.rk_step(Ur, 1e-7, variant="compact", ws=wsrc),
                                             max(args.steps // 5, 3), 2, stream)[0] * 1e3
        del wsrc
        from paper_1601_07613_amd.tune import autotune_rk

        best_rk, rk_res = autotune_rk(D, Ur, 1e-7, reps=max(args.steps // 5, 3))
        extra["rk3_step_autotuned"] = {"form": best_rk, "us": min(ms for _, ms in rk_res) * 1e3}
        D.set_rk_form("default")
        wsr32 = D.workspace("rk", "colored", "f32")
        for rf in ("separate", "fused_volume"):
            D.set_rk_form(rf)
            extra["rk3_step_f32_form_%s_us" % rf] = timed(lambda: D.rk_step(Ur, 1e-7, precision="f32", ws=wsr32),
                                                          max(args.steps // 5, 3), 2, stream)[0] * 1e3
        D.set_rk_form("default")
        del wsr32
        D.set_launch("thread", 256)
        extra["colored_thread_form_us"] = timed(lambda: D.surface_rhs(Ug, rhs, "colored"), args.steps, args.warmup,
                                                stream)[0] * 1e3
        D.set_launch(best["form"], best["block"], best["xcd_remap"])
        extra["colored_over_atomic"] = extra["atomic_us"] / (ms * 1e3)
        extra["colored_over_gather"] = extra["gather_us"] / (ms * 1e3)
        extra["colored_over_compact"] = extra["compact_us"] / (ms * 1e3)
        # the other layouts of the same coloring, same launch
        for lay in ("paper", "paper_sfc", "paired", "renumber", "none"):
            if lay == args.layout:
                continue
            D2, _, Ug2, rhs2 = device_mesh(lay)
            D2.set_launch(best["form"], best["block"], best["xcd_remap"])
            extra["colored_layout_%s_us" % lay] = timed(lambda: D2.surface_rhs(Ug2, rhs2, "colored"), args.steps,
                                                        args.warmup, stream)[0] * 1e3
            del D2, Ug2, rhs2
        M.set_colors(colors, layout=args.layout)
        # Table 7 shape: standard greedy (more colors) vs the paper's coloring,
        # each with no renumbering / renumbering / renumbering + reordering,
        # plus the headline pass itself; the seven passes are timed in turn,
        # round after round, so that slow drifts of the clock hit all alike
        G = dgc.Mesh.build(m["elem_vert"], m["elem_xyz"])
        gst = G.color(algorithm="greedy")
        gcol = G.export("color")
        cfgs = {"headline": (D, Ug, rhs)}
        for cname, Mx, col in (("greedy_%dcolors" % gst["n_colors"], G, gcol), ("paper_3colors", M, colors)):
            for lay in ("none", "renumber", "paper"):
                Mx.set_colors(col, layout=lay)
                Dx = dgc.DeviceMesh(Mx, p)
                Dx.set_launch(best["form"], best["block"], best["xcd_remap"])
                Ux = torch.from_numpy(Dx.to_layout(U)).cuda()
                cfgs["%s_%s" % (cname, lay)] = (Dx, Ux, torch.zeros_like(Ux))
        samples = {k: [] for k in cfgs}
        for _ in range(ABLATION_ROUNDS):
            for k, (Dx, Ux, rx) in cfgs.items():
                samples[k].append(time_call(lambda: Dx.surface_rhs(Ux, rx, "colored"), reps=args.steps,
                                            warmup=2) * 1e3)
        extra["table7_ablation_us"] = {
            k: {"median": float(np.median(v)), "min": float(min(v)), "max": float(max(v))} for k, v in samples.items()}
        extra["table7_ablation_us"]["rounds"] = ABLATION_ROUNDS
        del cfgs, samples
        M.set_colors(colors, layout=args.layout)
        del G
        # the f32 form of the same pass (f32 records, f64 geometry)
        U32 = Ug.float()
        r32 = torch.zeros_like(U32)
        ms32 = time_call(lambda: D.surface_rhs(U32, r32, "colored", "f32"), reps=args.steps, warmup=args.warmup)
        extra["colored_f32_us"] = ms32 * 1e3
        extra["colored_f32_algorithmic_GBs"] = algorithmic_bytes(E, E - nb, rec, 4, D.dim) / (ms32 * 1e-3) / 1e9
        del U32, r32
        # measured streaming reference: device copy of 1 GiB
        n = (1 << 30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        cms = time_call(lambda: b.copy_(a), reps=20, warmup=3)
        extra["copy_1GiB_GBs"] = 2 * n * 8 / (cms * 1e-3) / 1e9
        del a, b
        for k2, v in extra.items():
            log("%s: %s" % (k2, v))

    workloads = None
    if args.only == "all" and args.workload == "delaunay":
        workloads = extra_workloads(dgc, synth, torch, args.steps, args.warmup, log)
        workloads["coloring_sweep"] = coloring_sweep(dgc, synth, log)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import dg
        from oracle.mesh import build_mesh

        O = build_mesh(m["elem_vert"], m["elem_xyz"])
        d = dg.Discretization(O, args.p)
        d.face_basis(0)
        d.face_basis(1)
        reps = 2
        t = time.perf_counter()
        for _ in range(reps):
            dg.surface_rhs(d, U)
        cpu_s = (time.perf_counter() - t) / reps
        cpu = {"value": dof / cpu_s, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
               "sample": "the full surface term of this workload (%d elements, %d faces), %d repetitions, "
                         "numpy float64, single process" % (K, E, reps),
               "host": host_cpu()}
        log("cpu oracle: %.2f s per surface term" % cpu_s)
        if not args.no_cpu_pool:
            cpu["pool"] = oracle_pool(m, U, args.p, log)

    out = {
        "metric": "surface-integral DOF-updates/s",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("Delaunay triangulation of %d seeded Poisson-disc points in the unit square (%d triangles, "
                         "%d edges, %d wall edges), 2D Euler p=%d (N_p=%d, M=4), shock tube, colored surface pass, "
                         "%s layout" % (m["n_vert"], K, E, nb, args.p, D.n_p, args.layout))
            if args.workload == "delaunay" else
            ("periodic 1024^2 jittered parallelograms (%d cells, %d edges), 2D Euler p=%d (N_p=%d, M=4), density "
             "wave, colored surface pass, %s layout" % (K, E, args.p, D.n_p, args.layout))
            if args.workload == "quads" else
            ("periodic %d^3 cubes x 6 Kuhn tetrahedra (%d tets, %d faces), 3D Euler p=%d (N_p=%d, M=5), density "
             "wave, colored surface pass, %s layout" % (args.tet_n, K, E, args.p, D.n_p, args.layout)),
            "n_elem": K, "n_face": E, "p": args.p, "n_colors": info["n_colors"], "variant": "colored",
            "layout": args.layout, "launch": best,
        },
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": profiled_traffic(args, best),
                     "algorithmic_bytes_per_launch": ab // info["n_colors"],
                     "launches_per_pass": info["n_colors"],
                     "kernel": ("surface_mode_team_kernel" if args.workload == "tets" and best.get("form") in
                                ("default", "mode_team") else "surface_team_kernel") + " (colored), one launch per color"},
        "cpu_baseline": cpu,
        "host_preprocess": {"generate_s": gen_s, "build_s": build_s, "color_ms": cst["color_ms"],
                            "layout_ms": cst["layout_ms"], "conflicts_after_greedy": cst["conflicts_after_greedy"]},
        "variants_us": extra,
        "other_workloads": workloads,
    }
    print(json.dumps(out))
    reap_children(log)
    return 0


def reap_children(log):
    """Join every process this run started that is still alive (names it in
    the log first), so that nothing outlives the benchmark."""
    try:
        import psutil
    except ImportError:
        return
    kids = psutil.Process().children(recursive=True)
    for k in kids:
        try:
            log("child process still running at exit: pid %d %s" % (k.pid, " ".join(k.cmdline())))
            k.terminate()
        except psutil.Error:
            pass
    psutil.wait_procs(kids, timeout=10)


if __name__ == "__main__":
    sys.exit(main())
