"""Point sets on closed surfaces with per-point quadrature weights.

The paper's experiments discretise the Helmholtz single-layer operator on the
unit sphere with about n points and a wave number chosen so that kappa*h is
constant (Section 7, numerical experiments, Table of the single-layer
potential).  These generators stand in for that mesh: golden-spiral
(Fibonacci) points on the sphere, the same spiral mapped to a rotated
ellipsoid, and uniform random points on the surface of the cube [-1,1]^3.
Each point carries a weight w_i approximating the surface area it represents.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))


def fibonacci_sphere(n: int):
    """Golden-spiral points on the unit sphere, z_i = 1-(2i+1)/n.

    Returns (points (n,3) float64 C-contiguous, weights (n,) = 4*pi/n).
    """
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * GOLDEN_ANGLE
    pts = np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)
    w = np.full(n, 4.0 * math.pi / n)
    return np.ascontiguousarray(pts), w


def random_rotation(seed: int) -> np.ndarray:
    """A proper rotation (det=+1) from the QR factor of a seeded 3x3 Gaussian."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def ellipsoid(n: int, axes=(1.0, 0.5, 0.25), seed: int = 3):
    """Golden-spiral points mapped to a rotated ellipsoid.

    x = Rot * diag(a,b,c) * u for the unit-sphere spiral point u.  The weight
    is the sphere weight times the area-stretch factor of that map,
    abc * sqrt(u1^2/a^2 + u2^2/b^2 + u3^2/c^2); it reduces to 4*pi/n for a=b=c=1.
    """
    u, w0 = fibonacci_sphere(n)
    a, b, c = (float(v) for v in axes)
    rot = random_rotation(seed)
    x = (u * np.array([a, b, c])) @ rot.T
    stretch = a * b * c * np.sqrt(
        (u[:, 0] / a) ** 2 + (u[:, 1] / b) ** 2 + (u[:, 2] / c) ** 2
    )
    return np.ascontiguousarray(x), w0 * stretch


def sphere_normals(points) -> np.ndarray:
    """Outward unit normals of the unit sphere at the given points."""
    p = np.asarray(points, dtype=np.float64)
    return np.ascontiguousarray(p / np.linalg.norm(p, axis=1)[:, None])


def ellipsoid_normals(n: int, axes=(1.0, 0.5, 0.25), seed: int = 3) -> np.ndarray:
    """Outward unit normals at the points of ``ellipsoid(n, axes, seed)``.

    The surface is {Rot diag(a,b,c) u : |u| = 1}; its normal at the image of
    u is Rot diag(1/a,1/b,1/c) u, normalised.
    """
    u, _ = fibonacci_sphere(n)
    a, b, c = (float(v) for v in axes)
    rot = random_rotation(seed)
    g = (u / np.array([a, b, c])) @ rot.T
    return np.ascontiguousarray(g / np.linalg.norm(g, axis=1)[:, None])


def cube_surface(n: int, seed: int):
    """Uniform random points on the surface of [-1,1]^3, weight 24/n each."""
    rng = np.random.default_rng(seed)
    face = rng.integers(0, 6, size=n)
    uv = rng.uniform(-1.0, 1.0, size=(n, 2))
    pts = np.empty((n, 3))
    axis = face // 2
    sign = np.where(face % 2 == 0, 1.0, -1.0)
    for a in range(3):
        sel = axis == a
        other = [d for d in range(3) if d != a]
        pts[sel, a] = sign[sel]
        pts[sel, other[0]] = uv[sel, 0]
        pts[sel, other[1]] = uv[sel, 1]
    return np.ascontiguousarray(pts), np.full(n, 24.0 / n)


def complex_gaussian(n: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Seeded complex Gaussian vector (or n x nrhs block), complex128."""
    rng = np.random.default_rng(seed)
    shape = (n,) if nrhs is None else (n, nrhs)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@dataclass
class Instance:
    """One synthetic compression problem: points, weights, wave number."""

    name: str
    points: np.ndarray
    weights: np.ndarray
    kappa: float


def batch_instances(count: int = 48, seed: int = 4, nmin: int = 2048, nmax: int = 16384):
    """Independent instances: sphere, random rotated ellipsoid or cube surface.

    n_i is uniform in [nmin, nmax]; kappa_i = sqrt(n_i)/5.66 keeps kappa*h fixed
    as in the paper's experiment series.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        kind = int(rng.integers(0, 3))
        kappa = math.sqrt(n) / 5.66
        if kind == 0:
            p, w = fibonacci_sphere(n)
            name = "sphere"
        elif kind == 1:
            axes = tuple(rng.uniform(0.3, 1.0, size=3))
            p, w = ellipsoid(n, axes, seed=int(rng.integers(0, 2**31)))
            name = "ellipsoid"
        else:
            p, w = cube_surface(n, seed=int(rng.integers(0, 2**31)))
            name = "cube"
        out.append(Instance(name, p, w, kappa))
    return out


def workload(name: str):
    """Named workloads: (points, weights, kappa, leaf_size, eps).

    sphere2048   : n=2048 spiral sphere, kappa=8, leaf 32, eps 1e-4
    sphere32768  : n=32768 spiral sphere, kappa=32, leaf 64, eps 1e-6
    ellip32768   : n=32768 rotated ellipsoid (1,.5,.25), kappa=32, leaf 64, eps 1e-4
    ellip32768e6 : the same ellipsoid at eps 1e-6
    sphere131072 : n=131072 spiral sphere, kappa=64, leaf 64, eps 1e-4
    """
    if name == "sphere2048":
        p, w = fibonacci_sphere(2048)
        return p, w, 8.0, 32, 1e-4
    if name == "sphere32768":
        p, w = fibonacci_sphere(32768)
        return p, w, 32.0, 64, 1e-6
    if name == "ellip32768":
        p, w = ellipsoid(32768)
        return p, w, 32.0, 64, 1e-4
    if name == "ellip32768e6":
        p, w = ellipsoid(32768)
        return p, w, 32.0, 64, 1e-6
    if name == "sphere131072":
        p, w = fibonacci_sphere(131072)
        return p, w, 64.0, 64, 1e-4
    if name.startswith("sphere"):
        n = int(name[len("sphere"):])
        p, w = fibonacci_sphere(n)
        return p, w, math.sqrt(n) / 5.66, 64, 1e-4
    raise KeyError(name)
