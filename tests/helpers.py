"""Shared test helpers: build matching oracle / library meshes from one seeded input."""
from __future__ import annotations

import numpy as np

import synth


def make_input(kind: str, size: int, seed: int):
    if kind == "periodic":
        return synth.periodic_tri(size, seed=seed)
    if kind == "delaunay":
        return synth.poisson_delaunay(size, seed=seed)
    if kind == "tets":
        return synth.kuhn_tets(size, seed=seed)
    if kind == "tetbox":
        return synth.kuhn_tets(size, seed=seed, periodic=False)
    if kind == "quads":
        return synth.quad_grid(size, seed=seed)
    if kind == "quadbox":
        return synth.quad_grid(size, seed=seed, periodic=False)
    if kind == "quadshuf":
        # the grid numbered in a random order, as an unstructured generator would
        return synth.shuffle_elements(synth.quad_grid(size, seed=seed), seed=seed + 7)
    if kind == "hybrid":
        return synth.hybrid_grid(size, seed=seed)
    if kind == "hybridbox":
        return synth.hybrid_grid(size, seed=seed, periodic=False)
    raise ValueError(kind)


def rel_close(got, ref, scale, tol):
    """max |got - ref| / scale per conserved variable (scale: [K, M, Np] absolute sums)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    s = np.asarray(scale).max(axis=(0, 2)) if np.ndim(scale) == 3 else np.asarray(scale)
    err = np.abs(got - ref).max(axis=(0, 2)) / np.maximum(s, 1e-300)
    return err.max() <= tol, err


def oracle_serve_request(spec):
    """The CPU oracle's solution of one serving request: its mesh and initial
    DOFs, ``spec["steps"]`` SSP-RK3 steps with the time step the request
    supplies (runs in a worker process)."""
    import synth.requests as sreq
    from oracle import dg
    from oracle.mesh import build_mesh

    m, U = sreq.request_input(spec)
    dt = sreq.request_dt(spec, m)
    d = dg.Discretization(build_mesh(m["elem_vert"], m["elem_xyz"]), spec["p"])
    for _ in range(spec["steps"]):
        U = dg.rk3_step(d, U, dt)
    return U
