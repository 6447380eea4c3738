"""Oracle: construction of orthogonal directional cluster bases, coupling
matrices and near field (Section 6 of the paper).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the paper's order and notation:

* block weights omega_b = ||G|_b|| for b in L+ (remark "Error control", with
  the Frobenius norm; ``weight_norm='2'`` selects the spectral norm;
  ``weight_norm='global'`` gives every block the same weight, the Frobenius
  norm of G restricted to the admissible blocks, for a global-relative
  tolerance; ``weight_norm='one'`` the unit weights of the unweighted
  algorithm);
* weighted block rows G^w_tc: the columns of F_tc coming from the admissible
  block b=(t+,s) of an ancestor-or-self t+ are divided by
  omega_b * zeta^(level(t)-level(t+)) (remark "Error control": local accuracy
  eps_r ~ zeta^(level(r)-level(t)); the experiments use zeta = 2/3);
* leaf clusters: Q_tc = first k left singular vectors of G^w_tc, where k is the
  number of singular values above eps (absolute threshold on the weighted
  matrix; truncation error in the spectral norm <= eps);
* non-leaf clusters: G_hat_tc = [Q_{t1c'}^* G^w_tc|t1 ; Q_{t2c'}^* G^w_tc|t2]
  formed BY DEFINITION from the expanded son bases and the matrix itself
  (equation hatQ_hatG) -- deliberately not through the R recursion, so that
  the recursion used elsewhere can be checked against it; Q_hat = first k left
  singular vectors, split into E_{t1c}, E_{t2c};
* R_tc = Q_tc^* G^w_tc (optional; kept for checking a recursion);
* the column basis is the same construction applied to G^* with every block
  transposed, keeping c_b and omega_b (the paragraph after the Frobenius-best
  projection);
* coupling matrices S_b = V_{t c_b}^* G|_b W_{s c_b} (best approximation in the
  Frobenius norm for orthogonal bases);
* near field: G|_b copied for every inadmissible leaf b.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .matrix import AdjointMatrix
from .plan import Plan, ColumnSets


@dataclass
class Basis:
    """Directional cluster basis with transfer matrices, plus diagnostics."""

    k: dict = field(default_factory=dict)        # (t,c) -> rank
    sigma: dict = field(default_factory=dict)    # (t,c) -> all singular values
    Q: dict = field(default_factory=dict)        # leaf (t,c) -> #t x k
    E: dict = field(default_factory=dict)        # (t',c) -> k_{t'c'} x k_tc, c on father level
    Qhat: dict = field(default_factory=dict)     # non-leaf (t,c) -> r x k
    Qexp: dict = field(default_factory=dict)     # (t,c) -> expanded #t x k
    R: dict = field(default_factory=dict)        # (t,c) -> k x N_tc (optional)
    Ghat: dict = field(default_factory=dict)     # non-leaf (t,c) -> r x N_tc (optional)
    G: dict = field(default_factory=dict)        # (t,c) -> G^w_tc (optional, small n)


def block_weights(M, plan: Plan, norm: str = "fro") -> np.ndarray:
    """omega_b = ||G|_{t x s}|| for every admissible block (norm 'fro' or '2'),
    the same (sum_b ||G|_b||_F^2)^(1/2) for all blocks ('global'), or 1
    ('one')."""
    tr, bt = plan.tree, plan.blocks
    nb = len(bt.adm_t)
    if norm == "one":
        return np.ones(nb)
    if norm not in ("fro", "2", "global"):
        raise ValueError(f"unknown weight norm {norm!r}")
    om = np.empty(nb)
    for b in range(nb):
        blk = M.block(tr.rows(bt.adm_t[b]), tr.rows(bt.adm_s[b]))
        om[b] = np.linalg.norm(blk, 2 if norm == "2" else "fro")
    if norm == "global":
        om = np.full(nb, np.sqrt(np.sum(om ** 2)))
    return om


def weighted_block_row(M, plan: Plan, sets: ColumnSets, t: int, c: int,
                       omega: np.ndarray, zeta: float) -> np.ndarray:
    """G^w_tc: rows t, columns F_tc in set order, each block rescaled."""
    tr = plan.tree
    rows = tr.rows(t)
    parts = []
    for (b, s, d) in sets.F[t][c]:
        parts.append(M.block(rows, tr.rows(s)) / (omega[b] * zeta ** d))
    return np.hstack(parts)


def truncated_left_singular(A: np.ndarray, eps: float):
    """Left singular vectors whose singular values exceed eps."""
    if A.shape[0] == 0:
        return np.zeros((0, 0), dtype=np.complex128), np.zeros(0), 0
    U, sig, _ = np.linalg.svd(A, full_matrices=False)
    k = int(np.count_nonzero(sig > eps))
    return U[:, :k], sig, k


def build_basis(M, plan: Plan, sets: ColumnSets, omega: np.ndarray, eps: float,
                zeta: float, keep_R: bool = False, keep_G: bool = False) -> Basis:
    """Algorithm 'basis' of Section 6, levels from the deepest to the root."""
    tr, dr = plan.tree, plan.dirs
    B = Basis()
    order = sorted(range(tr.nc), key=lambda t: -tr.level[t])
    for t in order:
        if not sets.F[t]:
            continue
        rows_t = tr.rows(t)
        for c in sets.used(t):
            A = weighted_block_row(M, plan, sets, t, c, omega, zeta)
            if keep_G:
                B.G[(t, c)] = A
            if tr.son1[t] < 0:
                Q, sig, k = truncated_left_singular(A, eps)
                B.Q[(t, c)] = Q
                B.Qexp[(t, c)] = Q
            else:
                cp = int(dr.sd[tr.level[t]][c])
                blocks, sizes, sons_q = [], [], []
                for ts in tr.sons(t):
                    Qs = B.Qexp[(ts, cp)]
                    loc = tr.rows(ts) - tr.off[t]
                    blocks.append(Qs.conj().T @ A[loc, :])
                    sizes.append(Qs.shape[1])
                    sons_q.append((ts, Qs))
                Ghat = np.vstack(blocks)
                if keep_G:
                    B.Ghat[(t, c)] = Ghat
                Qh, sig, k = truncated_left_singular(Ghat, eps)
                B.Qhat[(t, c)] = Qh
                parts, o = [], 0
                for (ts, Qs), kk in zip(sons_q, sizes):
                    Es = Qh[o:o + kk, :]
                    o += kk
                    B.E[(ts, c)] = Es
                    parts.append(Qs @ Es)
                B.Qexp[(t, c)] = np.vstack(parts) if parts else np.zeros((len(rows_t), 0))
            B.k[(t, c)] = k
            B.sigma[(t, c)] = sig
            if keep_R:
                B.R[(t, c)] = B.Qexp[(t, c)].conj().T @ A
    return B


@dataclass
class Compressed:
    plan: Plan
    eps: float
    zeta: float
    omega: np.ndarray
    V: Basis
    W: Basis
    S: list                     # per admissible block: k_t x k_s
    near: list                  # per inadmissible block: dense block


def compress(M, plan: Plan, eps: float, zeta: float = 2.0 / 3.0,
             weight_norm: str = "fro", keep_R: bool = False,
             keep_G: bool = False) -> Compressed:
    """Full compression: row basis, column basis, coupling, near field."""
    tr, bt = plan.tree, plan.blocks
    omega = block_weights(M, plan, weight_norm)
    V = build_basis(M, plan, plan.rowsets, omega, eps, zeta, keep_R, keep_G)
    W = build_basis(AdjointMatrix(M), plan, plan.colsets, omega, eps, zeta, keep_R, keep_G)
    S = []
    for b in range(len(bt.adm_t)):
        t, s, c = int(bt.adm_t[b]), int(bt.adm_s[b]), int(bt.adm_c[b])
        Gb = M.block(tr.rows(t), tr.rows(s))
        S.append(V.Qexp[(t, c)].conj().T @ Gb @ W.Qexp[(s, c)])
    near = [M.block(tr.rows(t), tr.rows(s)) for t, s in zip(bt.near_t, bt.near_s)]
    return Compressed(plan, eps, zeta, omega, V, W, S, near)
