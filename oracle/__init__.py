"""CPU oracle for the edge-colored DG surface-integral path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64
implementation of what the GPU library computes, written from the paper
(Giuliani & Krivodonova, "Edge coloring in unstructured CFD codes") and,
where the paper is silent, from the readings listed in the project's design
notes.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path never does.  It shares no code
with the native library: the only common dependency is the ``synth`` input
generator package, which holds none of the method's arithmetic.

Parity status per module (what pins each function is listed in its header):

* ``quadrature``  -- pinned (monomial exactness).
* ``basis``       -- pinned (orthonormality, span, hand-derived p=1 modes).
* ``mesh``        -- pinned (counts, closure identities, periodic geometry).
* ``euler``       -- pinned (consistency, conservation, mirror symmetry).
* ``dg``          -- pinned (free stream, conservation, p=0 finite volume
  closed form, convergence order, SSP-RK3 amplification factor).
* ``coloring``    -- validity and count pinned exactly; the order of the
  resolution swaps is **parity unpinned** by the paper (its worked figures
  are not available), it is pinned only against the native library under
  one shared written specification.
* ``layout``      -- pinned (the paper's Table 5/6 properties).
* ``refine``      -- pinned (the paper's worked child-color example, the
  six-color bound, coarsening round trip).
"""
