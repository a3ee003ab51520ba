"""Seeded synthetic inputs for the solid-angle labeling path.

This package only builds geometry and point sets: closed triangulated
surfaces (icospheres, geodesic spheres, spherical-harmonic perturbed shells,
ellipsoids) and query point sets (uniform boxes, near-surface offsets,
precision ladders).  It contains none of the labeling arithmetic; both the
FP64 oracle and the GPU library consume its arrays.

All coordinates are generated in float64 and rounded once to float32 at the
end, so every consumer reads identical bits.
"""
from .meshes import (icosahedron, icosphere, geodesic_sphere, real_sph_harm,
                     sh_shell, ellipsoid, random_rotation, signed_volume,
                     check_closed_oriented)
from .configs import (Surface, Lattice, Config, config_small, config_c1, config_c2, c4_instance,
                      config_c3, config_c4, config_c5, SEED_BASE)
from .points import (uniform_box, near_surface_points, precision_ladder,
                     face_centroids_on_surface)

__all__ = [
    "icosahedron", "icosphere", "geodesic_sphere", "real_sph_harm", "sh_shell",
    "ellipsoid", "random_rotation", "signed_volume", "check_closed_oriented",
    "Surface", "Lattice", "Config", "c4_instance", "config_small", "config_c1", "config_c2", "config_c3",
    "config_c4", "config_c5", "SEED_BASE", "uniform_box", "near_surface_points",
    "precision_ladder", "face_centroids_on_surface",
]
