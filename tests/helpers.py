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
    if kind == "quads":
        return synth.quad_grid(size, seed=seed)
    if kind == "quadbox":
        return synth.quad_grid(size, seed=seed, periodic=False)
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
