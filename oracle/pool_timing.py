"""Timing of the oracle's surface term split over a pool of host processes.

Test infrastructure, like the rest of ``oracle/``: only the benchmark's CPU
baseline runs it, as a child process that never touches the GPU.  The
element set is cut into chunks; each worker evaluates the oracle's plain
face loop restricted to the faces of its chunk and returns the chunk's rows,
so faces on chunk borders are evaluated twice (once per side).  The result
is checked against the single-process oracle on the first chunks.

Usage: ``python -m oracle.pool_timing INPUT.npz WORKERS REPS`` where the
archive holds ``elem_vert``, ``elem_xyz``, ``U`` (original element order)
and ``p``; prints one JSON line.
"""

from __future__ import annotations

import json
import multiprocessing as mp
import sys
import time

import numpy as np

from oracle import dg
from oracle.mesh import build_mesh

_G: dict = {}


def _rows(chunk):
    r = dg.surface_rhs(_G["d"], _G["U"], elems=chunk)
    return chunk, r[chunk]


def main(argv) -> int:
    path, workers, reps = argv[0], int(argv[1]), int(argv[2])
    z = np.load(path)
    O = build_mesh(z["elem_vert"], z["elem_xyz"])
    d = dg.Discretization(O, int(z["p"]))
    d.face_basis(0)
    d.face_basis(1)
    U = z["U"]
    _G.update(d=d, U=U)
    chunks = np.array_split(np.arange(O.K), 4 * workers)
    # the workers inherit the discretisation from this process (no GPU here)
    with mp.get_context("fork").Pool(workers) as pool:
        pool.map(_rows, chunks[:workers])
        t = time.perf_counter()
        for _ in range(reps):
            rhs = np.empty_like(U)
            for chunk, rows in pool.imap_unordered(_rows, chunks):
                rhs[chunk] = rows
        sec = (time.perf_counter() - t) / reps
    probe = np.concatenate(chunks[:2])
    ref = dg.surface_rhs(d, U, elems=probe)[probe]
    ok = bool(np.array_equal(ref, rhs[probe]))
    print(json.dumps({"seconds": sec, "workers": workers, "reps": reps, "K": int(O.K), "E": int(O.E),
                      "matches_single_process": ok}))
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
