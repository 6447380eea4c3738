"""Pins for the oracle's double-layer entries and their compression.

* every entry against a central difference of the single-layer kernel in
  the normal direction at the column point (the definition of the DLP
  kernel as the normal derivative);
* on the unit sphere <x - y, y> = -|x - y|^2 / 2, so the entries reduce to
  -w_j (1 - i kappa r) exp(i kappa r) / (8 pi r), checked entry by entry;
* the compressed double-layer matrix meets the global error bound.
"""
import cmath
import math

import numpy as np

import synth
from oracle import compress as C
from oracle import dh2 as D
from oracle import matrix as Mx
from oracle import plan as P


def _slp(x, y, kappa):
    r = math.sqrt(sum((x[a] - y[a]) ** 2 for a in range(3)))
    return cmath.exp(1j * kappa * r) / (4 * math.pi * r)


def test_dlp_is_normal_derivative():
    x, w = synth.ellipsoid(300)
    nv = synth.ellipsoid_normals(300)
    kappa = 7.0
    M = Mx.HelmholtzDLPMatrix(x, nv, w, kappa)
    rng = np.random.default_rng(2)
    h = 1e-5
    for _ in range(40):
        i, j = rng.choice(300, 2, replace=False)
        blk = M.block(np.array([i]), np.array([j]))[0, 0]
        fd = (_slp(x[i], x[j] + h * nv[j], kappa) - _slp(x[i], x[j] - h * nv[j], kappa)) / (2 * h)
        assert abs(blk - w[j] * fd) <= 1e-7 * abs(blk) + 1e-12, (i, j)
    assert np.all(np.diag(M.dense()) == 0.5)


def test_dlp_on_the_sphere_closed_form():
    p, w = synth.fibonacci_sphere(200)
    kappa = 5.0
    G = Mx.dlp_dense_original(p, synth.sphere_normals(p), w, kappa)
    d = p[:, None, :] - p[None, :, :]
    r = np.sqrt(np.sum(d ** 2, axis=2))
    np.fill_diagonal(r, 1.0)
    ref = -w[None, :] * (1 - 1j * kappa * r) * np.exp(1j * kappa * r) / (8 * math.pi * r)
    np.fill_diagonal(ref, 0.5)
    assert np.allclose(G, ref, rtol=1e-12, atol=1e-15)


def test_dlp_compression_error():
    x, w = synth.ellipsoid(1024)
    nv = synth.ellipsoid_normals(1024)
    pl = P.build_plan(x, 8.0, 32)
    M = Mx.HelmholtzDLPMatrix(x, nv, w, 8.0, pl.tree.perm)
    cp = C.compress(M, pl, 1e-4)
    G = Mx.dlp_dense_original(x, nv, w, 8.0)
    err = np.linalg.norm(G - D.reconstruct(cp), 2) / np.linalg.norm(G, 2)
    assert 1e-8 < err <= 1e-4


def test_normals_are_outward_unit_vectors():
    """The synthetic normals are unit vectors pointing away from the centre
    (both surfaces are star-shaped about the origin)."""
    x, _ = synth.ellipsoid(500)
    for p_, n_ in ((x, synth.ellipsoid_normals(500)),
                   (synth.fibonacci_sphere(500)[0], synth.sphere_normals(synth.fibonacci_sphere(500)[0]))):
        assert np.allclose(np.linalg.norm(n_, axis=1), 1.0, atol=1e-15)
        assert np.all(np.sum(p_ * n_, axis=1) > 0)
