"""Launch autotuner for the colored face kernels.

Times every candidate launch configuration (kernel form, work-group size,
XCD remapping) of one device mesh on the caller's data with HIP events and
installs the fastest one.  All candidates compute the same result; only the
rounding order of the accumulation could differ between forms, and the
colored update is bitwise deterministic for a fixed form.
"""

from __future__ import annotations

import itertools

# "default" is the library's choice for the element type and order (team
# with right-hand-side prefetch in 2D, mode team for tetrahedra at p = 1)
DEFAULT_CANDIDATES = [
    {"form": f, "block": b, "xcd_remap": x}
    for f, b, x in itertools.product(("default", "team"), (128, 256), (False, True))
]


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
    cands = candidates or DEFAULT_CANDIDATES
    ws = dmesh.workspace("surface", variant, precision) if variant == "gather" else None
    results = []
    for c in cands:
        dmesh.set_launch(c["form"], c["block"], c.get("xcd_remap", False))
        ms = time_call(lambda: dmesh.surface_rhs(U, rhs, variant, precision, ws=ws), reps, warmup)
        results.append((dict(c), ms))
    best = min(results, key=lambda r: r[1])[0]
    dmesh.set_launch(best["form"], best["block"], best.get("xcd_remap", False))
    return best, results
