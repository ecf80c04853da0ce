"""Seeded synthetic inputs (ray tables, receivers, coefficients) for beam summation.

Input generation only: nothing here evaluates a beam.  The oracle and the HIP
library both consume what these functions return.
"""
from .tracer import (RayTable, City, fibonacci_fan, theta_phi_fan, trace_open_plane, trace_city,
                     receiver_grid, grid_city, inside_buildings, normal_frame, face_normal_axis,
                     transported_frame, rotate_table)
from .configs import (Scene, C_AIR, GATE_G, OCTAVES_8, eps_rule, eps_literal, open_plane, open_plane_2k,
                      open_plane_100k, city_scene, city_10x10, city_5x5_panels, city_batched,
                      perturbed_gamma, receiver_subsample)

__all__ = [
    "RayTable", "City", "fibonacci_fan", "theta_phi_fan", "trace_open_plane", "trace_city", "receiver_grid",
    "grid_city", "inside_buildings", "Scene", "C_AIR", "GATE_G", "OCTAVES_8", "eps_rule", "eps_literal",
    "open_plane", "open_plane_2k", "open_plane_100k", "city_scene", "city_10x10", "city_5x5_panels",
    "city_batched", "perturbed_gamma", "receiver_subsample", "normal_frame", "face_normal_axis", "transported_frame", "rotate_table",
]
