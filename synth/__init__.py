"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package holds no arithmetic of the compression method: it only draws
point clouds on surfaces, their quadrature weights and random vectors.  Every
generator is deterministic in its arguments (numpy ``default_rng`` seeds).
"""
from .surfaces import (
    fibonacci_sphere,
    sphere_normals,
    ellipsoid,
    ellipsoid_normals,
    cube_surface,
    random_rotation,
    batch_instances,
    complex_gaussian,
    workload,
)

__all__ = [
    "fibonacci_sphere",
    "sphere_normals",
    "ellipsoid",
    "ellipsoid_normals",
    "cube_surface",
    "random_rotation",
    "batch_instances",
    "complex_gaussian",
    "workload",
]
