"""Launch autotuner for the colored face kernels and the SSP-RK3 step.

Times every candidate launch configuration (kernel form, work-group size,
XCD remapping) of one device mesh on the caller's data with HIP events and
installs the fastest one; then, optionally, the fastest SSP-RK3 step
schedule (volume term and stage combination fused into the first and last
colors' launches, the combination only, or separate launches).  All
candidates compute the same result; only the rounding order of some sums
could differ between forms, and every form is bitwise deterministic.
"""

from __future__ import annotations

import itertools

# "default" is the library's choice for the element type, order, precision
# and size; "team" and "team_stream" are the alternatives that can win on a
# given mesh (the streaming team at large N_p x Q)
DEFAULT_CANDIDATES = [
    {"form": f, "block": b, "xcd_remap": x}
    for f, b, x in itertools.product(("default", "team", "team_stream"), (128, 256), (False, True))
]


def candidates_for(dmesh):
    """The launch candidates for this mesh: the common ones, and for
    tetrahedra at p = 1 the pair team too (the default there is the mode
    team)."""
    cands = list(DEFAULT_CANDIDATES)
    if dmesh.dim == 3 and dmesh.p == 1:
        cands += [{"form": "pair_team", "block": b, "xcd_remap": x}
                  for b, x in itertools.product((128, 256), (False, True))]
    return cands


def time_call(fn, reps: int = 20, warmup: int = 3) -> float:
    """Average milliseconds of ``fn()`` over ``reps`` calls on the current stream."""
    import torch

    for _ in range(warmup):
        fn()
    s = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(s)
    for _ in range(reps):
        fn()
    t1.record(s)
    t1.synchronize()
    return t0.elapsed_time(t1) / reps


def autotune(dmesh, U, rhs, variant: str = "colored", precision: str = "f64", candidates=None, reps: int = 20,
             warmup: int = 3):
    """Pick the fastest launch configuration of ``dmesh.surface_rhs`` for these
    arrays; returns ``(best, [(config, ms), ...])`` and leaves ``best`` installed."""
    cands = candidates or candidates_for(dmesh)
    ws = dmesh.workspace("surface", variant, precision) if variant in ("gather", "compact") else None
    results = []
    for c in cands:
        dmesh.set_launch(c["form"], c["block"], c.get("xcd_remap", False))
        ms = time_call(lambda: dmesh.surface_rhs(U, rhs, variant, precision, ws=ws), reps, warmup)
        results.append((dict(c), ms))
    best = min(results, key=lambda r: r[1])[0]
    dmesh.set_launch(best["form"], best["block"], best.get("xcd_remap", False))
    return best, results


RK_FORMS = ("fused_volume", "fused", "separate")


def autotune_rk(dmesh, U, dt: float, precision: str = "f64", forms=RK_FORMS, reps: int = 5, warmup: int = 2):
    """Pick the fastest SSP-RK3 step form of ``dmesh`` (with its installed face
    launch) for a state shaped like ``U``; the steps run on a copy, ``U`` is
    left unchanged.  Returns ``(best, [(form, ms), ...])`` and leaves ``best``
    installed.  A form whose conditions do not hold on this mesh runs as the
    next simpler one, so timing it is harmless."""
    work = U.clone()
    ws = dmesh.workspace("rk", "colored", precision)
    results = []
    for f in forms:
        dmesh.set_rk_form(f)
        ms = time_call(lambda: dmesh.rk_step(work, dt, precision=precision, ws=ws), reps, warmup)
        results.append((f, ms))
    best = min(results, key=lambda r: r[1])[0]
    dmesh.set_rk_form(best)
    return best, results
