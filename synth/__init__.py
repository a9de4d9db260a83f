"""Seeded synthetic inputs shared by the oracle-based tests and the GPU path.

This package generates *inputs only*: vertex coordinates, element-to-vertex
connectivity, per-element states and perturbations, refinement criteria and
request streams.  It contains none of the method's arithmetic (no face
table, no coloring, no basis, no flux), so both the CPU oracle and the
native library can consume its output without sharing any computation.
"""

from .meshes import (  # noqa: F401
    periodic_tri,
    lattice_delaunay,
    poisson_delaunay,
    kuhn_tets,
    element_measure,
    element_centroid,
    adapt_flags,
    hybrid_grid,
    quad_grid,
    refine_flags,
    shuffle_elements,
)
from .fields import (  # noqa: F401
    shock_tube_states,
    density_wave_states,
    uniform_states,
    perturbed_dofs,
    isentropic_vortex,
)
