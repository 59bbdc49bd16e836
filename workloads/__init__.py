"""Seeded synthetic workloads for the nodal DG elastic-wave solver.

This package only *generates inputs*: meshes (vertex coordinates, element to
vertex lists, boundary tags, periodic vertex identification), material models,
sponge-layer damping profiles, source and receiver positions, shot lists, and
plane-wave initial states. It holds none of the solver's arithmetic (no
operators, no fluxes, no time stepping) and is shared, as plain input data, by the CPU oracle, the tests and
the benchmark. The GPU library and the oracle never import each other.

All random draws use ``numpy.random.default_rng`` with fixed seeds so every
input is reproducible.
"""

from .mesh import kuhn_cube, kuhn_box, general_mesh, lattice_node_coords, element_centroids
from .medium import (layered_medium, blob_start_medium, homogeneous_medium,
                     lame_from_velocities, sponge_profile, pml_profile, pml_layer,
                     isotropic_stiffness, random_stiffness, stiffness_upper)
from .shots import (default_source, default_receivers, batched_shots,
                    ricker_f0)
from .planewave import plane_wave_state, anisotropic_plane_wave_state
from .configs import CONFIGS, get_config, build_workload

__all__ = [
    "kuhn_cube", "kuhn_box", "pml_profile", "pml_layer", "lattice_node_coords", "element_centroids",
    "layered_medium", "blob_start_medium", "homogeneous_medium",
    "lame_from_velocities", "sponge_profile", "isotropic_stiffness",
    "random_stiffness", "stiffness_upper", "anisotropic_plane_wave_state", "default_source", "default_receivers",
    "batched_shots", "ricker_f0", "plane_wave_state", "CONFIGS",
    "get_config", "build_workload",
]
