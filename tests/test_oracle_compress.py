"""Pins for the oracle's basis construction, coupling matrices and matvec.

The oracle is checked against what the paper and the mathematics fix: brute
force on small inputs, the exact Pythagoras identity behind the non-leaf step,
the error theorem, orthogonality and nestedness, Frobenius optimality of the
coupling matrices, a matrix that is directional-H2 by construction, and the
complex symmetry of the single-layer matrix.
"""
import cmath
import math

import numpy as np
import pytest

import synth
from oracle import compress as C
from oracle import dh2 as D
from oracle import matrix as Mx
from oracle import plan as P

EPS = 1e-4
ZETA = 2.0 / 3.0


@pytest.fixture(scope="module")
def sphere():
    p, w = synth.fibonacci_sphere(2048)
    pl = P.build_plan(p, 8.0, 32)
    M = Mx.HelmholtzMatrix(p, w, 8.0, pl.tree.perm)
    cp = C.compress(M, pl, EPS, ZETA, keep_R=True, keep_G=True)
    G = Mx.helmholtz_dense_original(p, w, 8.0)
    return p, w, pl, M, cp, G


def _entry(p, w, kappa, i, j):
    """One matrix entry written out with scalar complex arithmetic."""
    if i == j:
        return 0.5 * math.sqrt(w[i] / math.pi) + 1j * kappa * w[i] / (4 * math.pi)
    r = math.sqrt(sum((p[i][a] - p[j][a]) ** 2 for a in range(3)))
    return w[j] * cmath.exp(1j * kappa * r) / (4 * math.pi * r)


def test_leaf_block_rows_bruteforce(sphere):
    """Weights, weighted block rows and their singular values rebuilt entry by
    entry with scalar loops; ranks = #{sigma > eps}."""
    p, w, pl, M, cp, G = sphere
    tr = pl.tree
    leaf_items = [(t, c) for (t, c) in cp.V.Q][:4]
    for (t, c) in leaf_items:
        rows = [int(tr.perm[i]) for i in tr.rows(t)]
        cols, scale = [], []
        for (b, s, d) in pl.rowsets.F[t][c]:
            tb, sb = int(pl.blocks.adm_t[b]), int(pl.blocks.adm_s[b])
            om2 = 0.0
            for i in tr.rows(tb):
                for j in tr.rows(sb):
                    om2 += abs(_entry(p, w, 8.0, int(tr.perm[i]), int(tr.perm[j]))) ** 2
            assert math.isclose(math.sqrt(om2), cp.omega[b], rel_tol=1e-12)
            for j in tr.rows(s):
                cols.append(int(tr.perm[j]))
                scale.append(1.0 / (math.sqrt(om2) * ZETA ** d))
        A = np.array([[_entry(p, w, 8.0, i, j) * sc for j, sc in zip(cols, scale)] for i in rows])
        sig = np.linalg.svd(A, compute_uv=False)
        assert np.allclose(sig, cp.V.sigma[(t, c)], rtol=1e-12, atol=1e-14 * sig[0])
        assert cp.V.k[(t, c)] == int(np.sum(sig > EPS))


def _positions_in_son(pl, sets, t, c, ts):
    """Column positions of F_tc inside F_{ts,sd(c)} (matched by block id)."""
    tr, dr = pl.tree, pl.dirs
    cp_ = int(dr.sd[tr.level[t]][c])
    son_cols = []
    for (b, s, d) in sets.F[ts][cp_]:
        son_cols += [(b, int(j)) for j in tr.rows(s)]
    where = {key: i for i, key in enumerate(son_cols)}
    out = []
    for (b, s, d) in sets.F[t][c]:
        out += [where[(b, int(j))] for j in tr.rows(s)]
    return np.array(out)


def test_R_recursion_equals_definition(sphere):
    """G_hat_tc formed by definition equals zeta*[R_t1c'|F_tc ; R_t2c'|F_tc]
    (the R recursion of Section 6), and R_tc = Q_hat^* G_hat_tc."""
    p, w, pl, M, cp, G = sphere
    tr, dr = pl.tree, pl.dirs
    checked = 0
    for (t, c), Gh in cp.V.Ghat.items():
        cp_ = int(dr.sd[tr.level[t]][c])
        parts = []
        for ts in tr.sons(t):
            pos = _positions_in_son(pl, pl.rowsets, t, c, ts)
            parts.append(ZETA * cp.V.R[(ts, cp_)][:, pos])
        rec = np.vstack(parts)
        assert np.allclose(rec, Gh, rtol=0, atol=1e-12 * max(1.0, np.abs(Gh).max()))
        assert np.allclose(cp.V.Qhat[(t, c)].conj().T @ Gh, cp.V.R[(t, c)], atol=1e-12)
        checked += 1
    assert checked > 10


def test_error_nonleaf_identity(sphere):
    """Equation error_nonleaf: for every non-leaf (t,c) the Frobenius error
    splits exactly into the sons' errors plus the error of G_hat."""
    p, w, pl, M, cp, G = sphere
    tr, dr = pl.tree, pl.dirs
    for (t, c), Gh in cp.V.Ghat.items():
        A = cp.V.G[(t, c)]
        Q = cp.V.Qexp[(t, c)]
        lhs = np.linalg.norm(A - Q @ (Q.conj().T @ A)) ** 2
        cp_ = int(dr.sd[tr.level[t]][c])
        rhs = 0.0
        for ts in tr.sons(t):
            loc = tr.rows(ts) - tr.off[t]
            Qs = cp.V.Qexp[(ts, cp_)]
            As = A[loc, :]
            rhs += np.linalg.norm(As - Qs @ (Qs.conj().T @ As)) ** 2
        Qh = cp.V.Qhat[(t, c)]
        rhs += np.linalg.norm(Gh - Qh @ (Qh.conj().T @ Gh)) ** 2
        assert math.isclose(lhs, rhs, rel_tol=1e-9, abs_tol=1e-24)


def _desc_bound(pl, t, eps, zeta):
    """sum over r in desc(t) of (eps zeta^(level(r)-level(t)))^2."""
    tr = pl.tree
    tot, stack = 0.0, [t]
    while stack:
        r = stack.pop()
        tot += (eps * zeta ** (tr.level[r] - tr.level[t])) ** 2
        stack += list(tr.sons(r))
    return tot


def test_error_theorem_and_quasi_optimality(sphere):
    """Theorem 'Error estimate' in the weighted form, and the lower bound
    sigma_{k+1} <= ||(I-QQ^*)G_tc|| from the Eckart-Young theorem."""
    p, w, pl, M, cp, G = sphere
    for (t, c), A in cp.V.G.items():
        Q = cp.V.Qexp[(t, c)]
        err = np.linalg.norm(A - Q @ (Q.conj().T @ A), 2)
        assert err ** 2 <= _desc_bound(pl, t, EPS, ZETA) * (1 + 1e-9)
        sig = np.linalg.svd(A, compute_uv=False)
        k = Q.shape[1]
        if k < len(sig):
            assert sig[k] <= err * (1 + 1e-9) + 1e-15


def test_orthonormal_and_nested(sphere):
    """Definition 'Orthogonality' and equation 'nested'."""
    p, w, pl, M, cp, G = sphere
    tr, dr = pl.tree, pl.dirs
    for basis in (cp.V, cp.W):
        for (t, c), Q in basis.Qexp.items():
            k = Q.shape[1]
            assert np.allclose(Q.conj().T @ Q, np.eye(k), atol=1e-13)
            if tr.son1[t] >= 0:
                cp_ = int(dr.sd[tr.level[t]][c])
                for ts in tr.sons(t):
                    loc = tr.rows(ts) - tr.off[t]
                    assert np.allclose(Q[loc, :], basis.Qexp[(ts, cp_)] @ basis.E[(ts, c)],
                                       atol=1e-13)


def test_coupling_frobenius_optimal(sphere):
    """S_b = V^* G_b W minimises ||G_b - V S W^*||_F over S (Section 6)."""
    p, w, pl, M, cp, G = sphere
    tr, bt = pl.tree, pl.blocks
    rng = np.random.default_rng(7)
    for b in range(0, len(bt.adm_t), 97):
        t, s, c = int(bt.adm_t[b]), int(bt.adm_s[b]), int(bt.adm_c[b])
        V, W = cp.V.Qexp[(t, c)], cp.W.Qexp[(s, c)]
        Gb = M.block(tr.rows(t), tr.rows(s))
        base = np.linalg.norm(Gb - V @ cp.S[b] @ W.conj().T)
        for _ in range(3):
            Dl = 1e-3 * (rng.standard_normal(cp.S[b].shape) + 1j * rng.standard_normal(cp.S[b].shape))
            assert np.linalg.norm(Gb - V @ (cp.S[b] + Dl) @ W.conj().T) >= base


def test_block_error_bound(sphere):
    """Per block: ||G_b - V S W^*||_2 <= sqrt(2) * eps * omega_b / sqrt(1-2 zeta^2)
    (error-control remark summed over a binary tree, both bases)."""
    p, w, pl, M, cp, G = sphere
    tr, bt = pl.tree, pl.blocks
    bound = math.sqrt(2.0) * EPS / math.sqrt(1.0 - 2.0 * ZETA ** 2)
    for b in range(0, len(bt.adm_t), 13):
        t, s, c = int(bt.adm_t[b]), int(bt.adm_s[b]), int(bt.adm_c[b])
        Gb = M.block(tr.rows(t), tr.rows(s))
        err = np.linalg.norm(Gb - cp.V.Qexp[(t, c)] @ cp.S[b] @ cp.W.Qexp[(s, c)].conj().T, 2)
        assert err <= bound * cp.omega[b]


def test_global_error_and_matvec(sphere):
    """Relative spectral error below eps (the paper observes about eps/10),
    and the tree matvec (forward, coupling, backward, near field) equals the
    dense reconstruction."""
    p, w, pl, M, cp, G = sphere
    Gt = D.reconstruct(cp)
    err = np.linalg.norm(G - Gt, 2) / np.linalg.norm(G, 2)
    assert err <= EPS
    assert err >= EPS / 1000  # the compression really truncates
    x = synth.complex_gaussian(2048, 5)
    assert np.allclose(D.matvec(cp, x), Gt @ x, rtol=0, atol=1e-13 * np.abs(Gt @ x).max())
    assert np.allclose(D.matvec(cp, x, adjoint=True), Gt.conj().T @ x,
                       rtol=0, atol=1e-13 * np.abs(Gt.conj().T @ x).max())
    # the power iteration used for large n agrees with the exact 2-norm
    est = D.rel_error_2(cp, M=M, iters=60)
    assert est <= err * (1 + 1e-6)
    assert est >= 0.5 * err


def test_complex_symmetry(sphere):
    """Constant weights make G symmetric, so the column block row (s,c) of G^*
    and the row block row (s,-c) of G have the same singular values."""
    p, w, pl, M, cp, G = sphere
    assert np.allclose(G, G.T, atol=1e-15)
    tr, dr = pl.tree, pl.dirs
    n_checked = 0
    for (s, c), sig in cp.W.sigma.items():
        Dl = dr.dirs[tr.level[s]]
        neg = int(np.argmin(np.linalg.norm(Dl + Dl[c], axis=1)))
        sig2 = cp.V.sigma[(s, neg)]
        assert np.allclose(sig, sig2, rtol=1e-10, atol=1e-13 * sig[0])
        n_checked += 1
    assert n_checked > 50


def _random_dh2(pl, k0, rng):
    """A matrix that is a DH2 matrix by construction on plan pl."""
    tr, dr, bt = pl.tree, pl.dirs, pl.blocks

    def orth(rows, cols):
        a = rng.standard_normal((rows, cols)) + 1j * rng.standard_normal((rows, cols))
        q, _ = np.linalg.qr(a)
        return q[:, :cols]

    def basis(sets):
        Qexp = {}
        for t in sorted(range(tr.nc), key=lambda t: -tr.level[t]):
            for c in sets.used(t):
                if tr.son1[t] < 0:
                    Qexp[(t, c)] = orth(tr.size[t], min(k0, tr.size[t]))
                else:
                    cp_ = int(dr.sd[tr.level[t]][c])
                    sons = [Qexp[(ts, cp_)] for ts in tr.sons(t)]
                    r = sum(q.shape[1] for q in sons)
                    Qh = orth(r, min(k0, r))
                    parts, o = [], 0
                    for q in sons:
                        parts.append(q @ Qh[o:o + q.shape[1]])
                        o += q.shape[1]
                    Qexp[(t, c)] = np.vstack(parts)
        return Qexp

    V, W = basis(pl.rowsets), basis(pl.colsets)
    Gp = np.zeros((tr.n, tr.n), dtype=np.complex128)
    for t, s, c in zip(bt.adm_t, bt.adm_s, bt.adm_c):
        kt, ks = V[(t, c)].shape[1], W[(s, c)].shape[1]
        S = rng.standard_normal((kt, ks)) + 1j * rng.standard_normal((kt, ks))
        Gp[np.ix_(tr.rows(t), tr.rows(s))] = V[(t, c)] @ S @ W[(s, c)].conj().T
    for t, s in zip(bt.near_t, bt.near_s):
        shp = (tr.size[t], tr.size[s])
        Gp[np.ix_(tr.rows(t), tr.rows(s))] = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    G = np.empty_like(Gp)
    G[np.ix_(tr.perm, tr.perm)] = Gp
    return G


def test_exact_recovery_of_dh2_matrix():
    """A matrix that is directional-H2 with rank k0 by construction is
    recovered to rounding accuracy with ranks <= k0."""
    p, w = synth.fibonacci_sphere(1024)
    pl = P.build_plan(p, 8.0, 32)
    rng = np.random.default_rng(11)
    k0 = 6
    G = _random_dh2(pl, k0, rng)
    cp = C.compress(Mx.DenseMatrix(G, pl.tree.perm), pl, 1e-10)
    assert max(list(cp.V.k.values()) + list(cp.W.k.values())) <= k0
    Gt = D.reconstruct(cp)
    assert np.linalg.norm(G - Gt, 2) / np.linalg.norm(G, 2) <= 1e-9


def test_kappa_zero_ranks_bounded():
    """kappa = 0: one direction per level, a standard H2 matrix whose ranks do
    not grow with n (complexity theorem with kappa = 0)."""
    kmax = []
    for n in (512, 2048):
        p, w = synth.fibonacci_sphere(n)
        pl = P.build_plan(p, 0.0, 32)
        M = Mx.HelmholtzMatrix(p, w, 0.0, pl.tree.perm)
        cp = C.compress(M, pl, EPS)
        assert all(c == 0 for (_, c) in cp.V.k)
        kmax.append(max(cp.V.k.values()))
        if n == 512:
            G = M.dense()
            Gt = D.reconstruct(cp)[np.ix_(pl.tree.perm, pl.tree.perm)]
            assert np.linalg.norm(G - Gt, 2) / np.linalg.norm(G, 2) <= EPS
    assert kmax[1] <= kmax[0] + 4


@pytest.fixture(scope="module")
def small_sphere():
    p, w = synth.fibonacci_sphere(1024)
    pl = P.build_plan(p, 8.0, 32)
    M = Mx.HelmholtzMatrix(p, w, 8.0, pl.tree.perm)
    G = Mx.helmholtz_dense_original(p, w, 8.0)
    return p, w, pl, M, G


def test_global_weight_is_admissible_frobenius_norm(small_sphere):
    """The global weight is ||G restricted to the admissible blocks||_F, here
    computed from the dense matrix through a mask of the block list."""
    p, w, pl, M, G = small_sphere
    tr, bt = pl.tree, pl.blocks
    mask = np.zeros(G.shape, dtype=bool)
    for t, s in zip(bt.adm_t, bt.adm_s):
        rows = tr.perm[tr.rows(int(t))]
        cols = tr.perm[tr.rows(int(s))]
        mask[np.ix_(rows, cols)] = True
    om = C.block_weights(M, pl, "global")
    ref = np.linalg.norm(G[mask])
    assert np.allclose(om, ref, rtol=1e-13, atol=0)


def test_global_weights_equal_unit_weights_at_scaled_eps(small_sphere):
    """Constant weights omega only rescale the weighted block rows, so the
    global-relative compression at eps equals the unweighted one at
    eps * omega: same ranks, same subspaces (remark "Error control")."""
    p, w, pl, M, G = small_sphere
    cg = C.compress(M, pl, EPS, ZETA, weight_norm="global")
    og = float(cg.omega[0])
    c1 = C.compress(M, pl, EPS * og, ZETA, weight_norm="one")
    for bg, b1 in ((cg.V, c1.V), (cg.W, c1.W)):
        assert bg.k.keys() == b1.k.keys()
        for key in bg.k:
            s1 = b1.sigma[key]
            if np.any(np.abs(s1 - EPS * og) <= 1e-10 * EPS * og):
                continue
            assert bg.k[key] == b1.k[key], key
            assert np.allclose(bg.sigma[key] * og, s1, rtol=1e-12, atol=1e-14 * og)
            Qg, Q1 = bg.Qexp[key], b1.Qexp[key]
            if Qg.shape[1]:
                assert np.linalg.norm(Qg @ Qg.conj().T - Q1 @ Q1.conj().T, 2) <= 1e-9


def test_global_weights_block_bound(small_sphere):
    """With one weight for all blocks every admissible block obeys the
    bound of the error-control remark with that weight, and the global
    relative error stays below eps * omega / ||G||_2 times the same factor."""
    p, w, pl, M, G = small_sphere
    cp = C.compress(M, pl, EPS, ZETA, weight_norm="global")
    tr, bt = pl.tree, pl.blocks
    om = float(cp.omega[0])
    bound = math.sqrt(2.0) * EPS * om / math.sqrt(1.0 - 2.0 * ZETA ** 2)
    worst = 0.0
    for b in range(len(bt.adm_t)):
        t, s, c = int(bt.adm_t[b]), int(bt.adm_s[b]), int(bt.adm_c[b])
        Gb = M.block(tr.rows(t), tr.rows(s))
        err = np.linalg.norm(Gb - cp.V.Qexp[(t, c)] @ cp.S[b] @ cp.W.Qexp[(s, c)].conj().T, 2)
        worst = max(worst, err / bound)
    assert worst <= 1.0
    # the weights are larger than the block norms, so the compression is
    # coarser than the block-relative one
    cb = C.compress(M, pl, EPS, ZETA)
    assert sum(cp.V.k.values()) <= sum(cb.V.k.values())


def test_spectral_weights_block_bound(small_sphere):
    """Spectral weights omega_b = ||G|_b||_2 <= ||G|_b||_F: every block obeys
    the bound of the error-control remark with its spectral weight, and the
    bases are at least as large as with Frobenius weights."""
    p, w, pl, M, G = small_sphere
    tr, bt = pl.tree, pl.blocks
    cs = C.compress(M, pl, EPS, ZETA, weight_norm="2")
    cf = C.compress(M, pl, EPS, ZETA)
    assert np.all(cs.omega <= cf.omega * (1 + 1e-14))
    bound = math.sqrt(2.0) * EPS / math.sqrt(1.0 - 2.0 * ZETA ** 2)
    for b in range(len(bt.adm_t)):
        t, s, c = int(bt.adm_t[b]), int(bt.adm_s[b]), int(bt.adm_c[b])
        Gb = M.block(tr.rows(t), tr.rows(s))
        err = np.linalg.norm(Gb - cs.V.Qexp[(t, c)] @ cs.S[b] @ cs.W.Qexp[(s, c)].conj().T, 2)
        assert err <= bound * cs.omega[b]
        # the weight is the block's largest singular value
        assert abs(np.linalg.svd(Gb, compute_uv=False)[0] - cs.omega[b]) <= 1e-13 * cs.omega[b]
    assert sum(cs.V.k.values()) >= sum(cf.V.k.values())


def _words_from_ranks(pl, cp):
    """Storage in complex words counted from the ranks and block lists only:
    leaf bases #t x k, transfer matrices (sum of the sons' ranks) x k,
    couplings k_t x k_s, near-field blocks #t x #s."""
    tr, dr, bt = pl.tree, pl.dirs, pl.blocks
    words = 0
    for basis in (cp.V, cp.W):
        for (t, c), k in basis.k.items():
            if tr.son1[t] < 0:
                words += int(tr.size[t]) * k
            else:
                cp_ = int(dr.sd[tr.level[t]][c])
                words += sum(basis.k[(ts, cp_)] for ts in tr.sons(t)) * k
    for b in range(len(bt.adm_t)):
        t, s, c = int(bt.adm_t[b]), int(bt.adm_s[b]), int(bt.adm_c[b])
        words += cp.V.k[(t, c)] * cp.W.k[(s, c)]
    for t, s in zip(bt.near_t, bt.near_s):
        words += int(tr.size[t]) * int(tr.size[s])
    return words


def test_storage_stats_word_count(sphere):
    """storage_stats (k_max, Mem/n in KiB per degree of freedom, the paper's
    storage column) equals the count from the ranks and the block lists."""
    p, w, pl, M, cp, G = sphere
    st = D.storage_stats(cp)
    words = _words_from_ranks(pl, cp)
    assert math.isclose(st["mem_per_n_kib"], words * 16 / 1024 / pl.tree.n, rel_tol=1e-14)
    assert st["k_max"] == max(list(cp.V.k.values()) + list(cp.W.k.values()))
    assert st["k_max"] > 0


def test_storage_stats_closed_forms():
    """Two closed forms on the 512-point sphere: with a threshold above every
    singular value all ranks are 0 and only the near field is stored; with
    an admissibility parameter so small that no block is admissible the near
    field is the whole matrix, n^2 words, i.e. 16 n / 1024 KiB per point."""
    p, w = synth.fibonacci_sphere(512)
    pl = P.build_plan(p, 6.0, 16)
    M = Mx.HelmholtzMatrix(p, w, 6.0, pl.tree.perm)
    cp = C.compress(M, pl, 1e10, ZETA)
    st = D.storage_stats(cp)
    tr, bt = pl.tree, pl.blocks
    near = sum(int(tr.size[t]) * int(tr.size[s]) for t, s in zip(bt.near_t, bt.near_s))
    assert len(bt.adm_t) > 0 and st["k_max"] == 0
    assert math.isclose(st["mem_per_n_kib"], near * 16 / 1024 / 512, rel_tol=1e-14)
    pl0 = P.build_plan(p, 6.0, 16, eta2=1e-9)
    assert len(pl0.blocks.adm_t) == 0
    cp0 = C.compress(Mx.HelmholtzMatrix(p, w, 6.0, pl0.tree.perm), pl0, EPS, ZETA)
    st0 = D.storage_stats(cp0)
    assert st0["k_max"] == 0
    assert math.isclose(st0["mem_per_n_kib"], 16 * 512 / 1024, rel_tol=1e-14)
