"""Oracle: matrix entries of the point-Nystroem Helmholtz single layer.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's matrix is the Galerkin discretisation of the single-layer operator
with the kernel g(x,y) = exp(i kappa |x-y|) / (4 pi |x-y|) (Section 1, the
Helmholtz kernel and the matrix definition).  The workloads here replace the
Galerkin integrals by point evaluation with surface weights:

    G_ij = w_j g(x_i, x_j)                          for i != j,
    G_ii = sqrt(w_i/pi)/2 + i kappa w_i / (4 pi),

the diagonal being the integral of g over a flat disk of area w_i around x_i
(to first order in kappa).  All functions address rows and columns by
positions in the permuted order of a cluster tree, through ``perm``.

The double-layer workload (Section 7, the DLP matrix: G = M/2 + G_dlp with
the kernel's normal derivative at y) is read the same way, for a second-kind
operator in collocation form:

    G_ij = w_j (1 - i kappa r) exp(i kappa r) <x_i - x_j, n_j> / (4 pi r^3),
    G_ii = 1/2,

the self-contribution of a flat disk being zero (<x - y, n(y)> = 0 on it).
"""
from __future__ import annotations

import math

import numpy as np


class HelmholtzMatrix:
    """Entries generated from points, weights and the wave number."""

    def __init__(self, points, weights, kappa: float, perm=None):
        pts = np.asarray(points, dtype=np.float64)
        w = np.asarray(weights, dtype=np.float64)
        if perm is None:
            perm = np.arange(len(pts))
        self.perm = np.asarray(perm)
        self.p = pts[self.perm]
        self.w = w[self.perm]
        self.kappa = float(kappa)
        self.n = len(pts)

    def block(self, rows, cols) -> np.ndarray:
        """G restricted to permuted positions rows x cols (complex128)."""
        rows = np.asarray(rows)
        cols = np.asarray(cols)
        d = self.p[rows][:, None, :] - self.p[cols][None, :, :]
        r = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2 + d[..., 2] ** 2)
        same = rows[:, None] == cols[None, :]
        rr = np.where(same, 1.0, r)
        g = np.exp(1j * self.kappa * rr) / (4.0 * math.pi * rr)
        out = self.w[cols][None, :] * g
        if same.any():
            wi = np.broadcast_to(self.w[rows][:, None], same.shape)
            diag = 0.5 * np.sqrt(wi / math.pi) + 1j * self.kappa * wi / (4.0 * math.pi)
            out = np.where(same, diag, out)
        return out

    def dense(self) -> np.ndarray:
        """The whole matrix in permuted order."""
        idx = np.arange(self.n)
        return self.block(idx, idx)


class HelmholtzDLPMatrix:
    """Double-layer entries from points, unit normals, weights and kappa."""

    def __init__(self, points, normals, weights, kappa: float, perm=None):
        pts = np.asarray(points, dtype=np.float64)
        nrm = np.asarray(normals, dtype=np.float64)
        w = np.asarray(weights, dtype=np.float64)
        if perm is None:
            perm = np.arange(len(pts))
        self.perm = np.asarray(perm)
        self.p = pts[self.perm]
        self.nv = nrm[self.perm]
        self.w = w[self.perm]
        self.kappa = float(kappa)
        self.n = len(pts)

    def block(self, rows, cols) -> np.ndarray:
        """G restricted to permuted positions rows x cols (complex128)."""
        rows = np.asarray(rows)
        cols = np.asarray(cols)
        d = self.p[rows][:, None, :] - self.p[cols][None, :, :]
        r = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2 + d[..., 2] ** 2)
        same = rows[:, None] == cols[None, :]
        rr = np.where(same, 1.0, r)
        dn = np.einsum("ijk,jk->ij", d, self.nv[cols])
        k = self.kappa
        g = (1.0 - 1j * k * rr) * np.exp(1j * k * rr) * dn / (4.0 * math.pi * rr ** 3)
        out = self.w[cols][None, :] * g
        return np.where(same, 0.5 + 0.0j, out)

    def dense(self) -> np.ndarray:
        idx = np.arange(self.n)
        return self.block(idx, idx)


def dlp_dense_original(points, normals, weights, kappa: float) -> np.ndarray:
    """Dense double-layer G in the ORIGINAL point order."""
    return HelmholtzDLPMatrix(points, normals, weights, kappa).dense()


class DenseMatrix:
    """Entries read from a dense matrix given in the original index order."""

    def __init__(self, G, perm=None):
        self.G = np.asarray(G, dtype=np.complex128)
        self.n = self.G.shape[0]
        self.perm = np.arange(self.n) if perm is None else np.asarray(perm)

    def block(self, rows, cols) -> np.ndarray:
        return self.G[np.ix_(self.perm[np.asarray(rows)], self.perm[np.asarray(cols)])]

    def dense(self) -> np.ndarray:
        return self.G[np.ix_(self.perm, self.perm)]


class AdjointMatrix:
    """Entries of G^* from entries of G: (G^*)|_{r x c} = (G|_{c x r})^*."""

    def __init__(self, base):
        self.base = base
        self.n = base.n

    def block(self, rows, cols) -> np.ndarray:
        return self.base.block(cols, rows).conj().T


def helmholtz_dense_original(points, weights, kappa: float) -> np.ndarray:
    """Dense G in the ORIGINAL point order (the dense-input workload)."""
    return HelmholtzMatrix(points, weights, kappa).dense()
