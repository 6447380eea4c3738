"""Oracle: the DH2 representation in use -- matrix-vector product, dense
reconstruction, error measures and storage statistics.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* matvec: forward transformation x_sc = W_sc^* x|s through the transfer
  matrices, coupling y_tc = sum_b S_b x_{s c_b}, backward transformation
  y|t += V_tc y_tc through the transfer matrices, and the near field
  (Section 4, equations mvm1-mvm3 and the forward/backward procedures; the
  backward procedure's leaf loop runs over the directions of t).
* reconstruct: the dense matrix V_tc S_b W_sc^* / G|_b, block by block.
* rel_error_2: ||G - G~||_2 / ||G||_2, exact for small n (dense SVD) and by
  a power iteration otherwise (Section 7 measures the relative spectral
  error with a power iteration).
"""
from __future__ import annotations

import numpy as np

from .compress import Compressed


def _forward(cp: Compressed, basis, sets, x):
    """x_hat[(s,c)] for every used (s,c), leaves up."""
    tr, dr = cp.plan.tree, cp.plan.dirs
    xh = {}
    for s in sorted(range(tr.nc), key=lambda t: -tr.level[t]):
        for c in sets.used(s):
            if tr.son1[s] < 0:
                xh[(s, c)] = basis.Q[(s, c)].conj().T @ x[tr.rows(s)]
            else:
                cp_ = int(dr.sd[tr.level[s]][c])
                acc = 0
                for ss in tr.sons(s):
                    acc = acc + basis.E[(ss, c)].conj().T @ xh[(ss, cp_)]
                xh[(s, c)] = acc
    return xh


def _backward(cp: Compressed, basis, sets, yh, y):
    tr, dr = cp.plan.tree, cp.plan.dirs
    for t in sorted(range(tr.nc), key=lambda t: tr.level[t]):
        for c in sets.used(t):
            if (t, c) not in yh:
                continue
            if tr.son1[t] < 0:
                y[tr.rows(t)] += basis.Q[(t, c)] @ yh[(t, c)]
            else:
                cp_ = int(dr.sd[tr.level[t]][c])
                for ts in tr.sons(t):
                    add = basis.E[(ts, c)] @ yh[(t, c)]
                    if (ts, cp_) in yh:
                        yh[(ts, cp_)] = yh[(ts, cp_)] + add
                    else:
                        yh[(ts, cp_)] = add


def matvec(cp: Compressed, x: np.ndarray, adjoint: bool = False) -> np.ndarray:
    """y = G~ x (or G~^* x) for x in the ORIGINAL index order."""
    tr, bt = cp.plan.tree, cp.plan.blocks
    perm = tr.perm
    xp = np.asarray(x, dtype=np.complex128)[perm]
    y = np.zeros_like(xp)
    if not adjoint:
        src, dst, src_sets, dst_sets = cp.W, cp.V, cp.plan.colsets, cp.plan.rowsets
    else:
        src, dst, src_sets, dst_sets = cp.V, cp.W, cp.plan.rowsets, cp.plan.colsets
    xh = _forward(cp, src, src_sets, xp)
    yh = {}
    for b in range(len(bt.adm_t)):
        t, s, c = int(bt.adm_t[b]), int(bt.adm_s[b]), int(bt.adm_c[b])
        if adjoint:
            t, s = s, t
            contrib = cp.S[b].conj().T @ xh[(s, c)]
        else:
            contrib = cp.S[b] @ xh[(s, c)]
        yh[(t, c)] = yh[(t, c)] + contrib if (t, c) in yh else contrib
    _backward(cp, dst, dst_sets, yh, y)
    for (t, s), blk in zip(zip(bt.near_t, bt.near_s), cp.near):
        if adjoint:
            y[tr.rows(s)] += blk.conj().T @ xp[tr.rows(t)]
        else:
            y[tr.rows(t)] += blk @ xp[tr.rows(s)]
    out = np.empty_like(y)
    out[perm] = y
    return out


def reconstruct(cp: Compressed) -> np.ndarray:
    """Dense G~ in the ORIGINAL index order."""
    tr, bt = cp.plan.tree, cp.plan.blocks
    n = tr.n
    Gp = np.zeros((n, n), dtype=np.complex128)
    for b in range(len(bt.adm_t)):
        t, s, c = int(bt.adm_t[b]), int(bt.adm_s[b]), int(bt.adm_c[b])
        Gp[np.ix_(tr.rows(t), tr.rows(s))] = cp.V.Qexp[(t, c)] @ cp.S[b] @ cp.W.Qexp[(s, c)].conj().T
    for (t, s), blk in zip(zip(bt.near_t, bt.near_s), cp.near):
        Gp[np.ix_(tr.rows(t), tr.rows(s))] = blk
    out = np.empty_like(Gp)
    out[np.ix_(tr.perm, tr.perm)] = Gp
    return out


def spectral_norm_power(apply, apply_adj, n: int, iters: int = 50, seed: int = 1,
                        rtol: float = 1e-4) -> float:
    """Largest singular value of an operator by the power method on A^*A."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x /= np.linalg.norm(x)
    lam_old = 0.0
    lam = 0.0
    for _ in range(iters):
        y = apply_adj(apply(x))
        lam = float(np.real(np.vdot(x, y)))
        nrm = np.linalg.norm(y)
        if nrm == 0.0:
            return 0.0
        x = y / nrm
        if lam_old > 0.0 and abs(lam - lam_old) <= rtol * lam:
            break
        lam_old = lam
    return float(np.sqrt(max(lam, 0.0)))


def rel_error_2(cp: Compressed, G: np.ndarray | None = None, M=None, iters: int = 50,
                seed: int = 1) -> float:
    """||G - G~||_2 / ||G||_2; exact when the dense G is given."""
    if G is not None:
        Gt = reconstruct(cp)
        return float(np.linalg.norm(G - Gt, 2) / np.linalg.norm(G, 2))
    n = cp.plan.tree.n
    idx = np.arange(n)
    perm = cp.plan.tree.perm

    def gx(x, adj=False):
        # direct product with the generated matrix, in row chunks
        xp = x[perm]
        y = np.empty(n, dtype=np.complex128)
        step = 1024
        for a in range(0, n, step):
            rows = idx[a:a + step]
            if adj:
                y[rows] = M.block(idx, rows).conj().T @ xp
            else:
                y[rows] = M.block(rows, idx) @ xp
        out = np.empty_like(y)
        out[perm] = y
        return out

    diff = lambda x: gx(x) - matvec(cp, x)
    diff_a = lambda x: gx(x, True) - matvec(cp, x, adjoint=True)
    num = spectral_norm_power(diff, diff_a, n, iters, seed)
    den = spectral_norm_power(gx, lambda x: gx(x, True), n, iters, seed)
    return num / den


def storage_stats(cp: Compressed) -> dict:
    """k_max and storage in KiB per degree of freedom (complex128 = 16 B)."""
    tr = cp.plan.tree
    words = 0
    for Q in cp.V.Q.values():
        words += Q.size
    for Q in cp.W.Q.values():
        words += Q.size
    for E in list(cp.V.E.values()) + list(cp.W.E.values()):
        words += E.size
    for S in cp.S:
        words += S.size
    for blk in cp.near:
        words += blk.size
    kmax = max([0] + list(cp.V.k.values()) + list(cp.W.k.values()))
    return dict(k_max=kmax, mem_per_n_kib=words * 16 / 1024 / tr.n)
