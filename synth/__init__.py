"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package holds no arithmetic of the boundary-integral method: it only
builds triangulated closed surfaces (geodesic icospheres and star-shaped
deformations of them) and point charges placed inside them.  These stand in
for the MSMS molecular surfaces and force-field partial charges of the
paper's protein workloads (Sec. 2.1, Tables 4 and 5), which are not
available.  Every draw uses ``numpy.random.default_rng`` (PCG64) in a fixed
order, so a seed names one input exactly.
"""
from .mesh import icosphere, star_radius, star_surface, real_sph_harm
from .charges import interior_charges, point_triangle_distance
from .workloads import (
    Workload,
    kirkwood_sphere,
    star_protein,
    large_star_protein,
    large_star_surface,
    batch_conformations,
    input_digest,
)

__all__ = [
    "icosphere",
    "star_radius",
    "star_surface",
    "real_sph_harm",
    "interior_charges",
    "point_triangle_distance",
    "Workload",
    "kirkwood_sphere",
    "star_protein",
    "large_star_protein",
    "large_star_surface",
    "batch_conformations",
    "input_digest",
]
