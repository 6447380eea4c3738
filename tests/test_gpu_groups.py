"""Subtree batches (opts.groups = 2 and 3) against the FP64 oracle, both forms.

The sweep can run the subtrees below the first admissible level in several
groups, one after the other (the FP64 form does so by itself at the largest
size).  Here the groups are forced on the 2048-point sphere (kappa 8, leaf
32) and the 4096-point rotated ellipsoid (kappa sqrt(n)/5.66, leaf 32), both
at eps 1e-4, and every step of the basis construction is checked against
what the paper defines:

* leaf (t,c): singular values and rank of the weighted block row G^w_tc
  (the oracle's LAPACK SVD) and the projector Q Q^* (Davis-Kahan);
* other (t,c): G_hat_tc formed BY DEFINITION from the library's own expanded
  son bases and the oracle's weighted block row, [V_t1^* G^w|t1; V_t2^* G^w|t2]
  (Section 6), its singular values and rank against the library's, and the
  projector of the library's [E_t1c; E_t2c] against its left singular
  vectors;
* coupling matrices: S_b = V_tc^* G|_b W_sc with the library's expanded
  bases and the oracle's matrix block (projection step);
* per block: V S W^* of the library against the oracle's, bounded by the
  measured differences of the expanded projectors (a provable inequality);
* global relative error <= 1.1 eps and within 10 % of the oracle's, matvec
  N and C against the dense reconstruction of the exported representation
  to 1e-10, and the group count in the statistics.

Tolerances are those derived in test_gpu_parity: FP64 |sigma^2 - s^2| <=
1e-13 ||A||_F^2 + 1e-10 s^2 + max(1e-4 eps^2, 64 u r ||A||_F^2) (the last
term is the pivoted Cholesky's stop: the Schur complement it leaves is
positive semidefinite with diagonal below tau = max(1e-4 eps^2 / r,
64 u max_i M_ii), so its norm is at most its trace r tau, and by Weyl's
theorem no eigenvalue of the Gram matrix moves by more); mixed
|sigma - s| <= 2e-7 ||A||_F.  Coupling matrices: FP64
1e-11 omega_b (a few hundred roundings of the R recursion and the products
at unit relative size), mixed 4e-6 omega_b (complex FP32 entries and
R-products, at most 128-term FP32 sums per level and up to four levels:
about 60 roundings of 2^-24).
"""
import math

import numpy as np
import pytest

import synth
from oracle import compress as OC
from oracle import dh2 as OD
from oracle import matrix as OM
from oracle import plan as OP

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = 1e-4
ZETA = 2.0 / 3.0
MIXED_SIGMA = 2e-7
S_TOL = {"fp64": 1e-11, "mixed": 4e-6}

PROBLEMS = {
    "sphere2048": lambda: (*synth.fibonacci_sphere(2048), 8.0),
    "ellip4096": lambda: (*synth.ellipsoid(4096), math.sqrt(4096) / 5.66),
}
_cache = {}


def _problem(name):
    if name not in _cache:
        p, w, kappa = PROBLEMS[name]()
        plan = OP.build_plan(p, kappa, 32)
        M = OM.HelmholtzMatrix(p, w, kappa, plan.tree.perm)
        ref = OC.compress(M, plan, EPS, ZETA)
        G = OM.helmholtz_dense_original(p, w, kappa)
        _cache[name] = dict(p=p, w=w, kappa=kappa, plan=plan, M=M, ref=ref, G=G)
    return _cache[name]


def _sigma_check(sig_gpu, sig_ref, form):
    """Assert the singular values agree within the form's band; returns
    (tie, worst relative deviation)."""
    fro = float(np.sqrt(np.sum(sig_ref ** 2)))
    n_ = min(len(sig_gpu), len(sig_ref))
    g, s = sig_gpu[:n_], sig_ref[:n_]
    big = s > EPS
    if form == "mixed":
        d = np.abs(g[big] - s[big]) / max(fro, 1e-300)
        assert np.all(d <= MIXED_SIGMA), d.max()
        tie = bool(np.any(np.abs(sig_ref - EPS) <= MIXED_SIGMA * fro))
    else:
        tl = 1e-13 * fro ** 2 + _chol_cut(len(sig_ref), fro)
        d = np.abs(g[big] ** 2 - s[big] ** 2)
        assert np.all(d <= tl + 1e-10 * s[big] ** 2), d.max()
        d = d / max(fro ** 2, 1e-300)
        tie = bool(np.any(np.abs(sig_ref ** 2 - EPS ** 2) <= tl + 1e-10 * EPS ** 2))
    return tie, float(d.max()) if d.size else 0.0


def _chol_cut(r, fro):
    """Largest eigenvalue change from the pivoted Cholesky's stop: it leaves a
    positive semidefinite Schur complement whose diagonal is below
    tau = max(1e-4 eps^2 / r, 64 u max_i M_ii), so its norm is at most its
    trace, r tau, and max_i M_ii <= ||A||_F^2."""
    return max(1e-4 * EPS ** 2, 64 * 2.220446049250313e-16 * r * fro ** 2)


def _tol_lambda(sig_ref, form):
    fro2 = float(np.sum(sig_ref ** 2))
    if form == "mixed":
        return 2.0 * float(sig_ref[0]) * MIXED_SIGMA * np.sqrt(fro2) + 1e-13 * fro2
    return 1e-13 * fro2 + _chol_cut(len(sig_ref), np.sqrt(fro2))


def _projector_check(Qg, U, sig, k, form):
    if k == 0:
        return
    gap = sig[k - 1] ** 2 - (sig[k] ** 2 if k < len(sig) else 0.0)
    P = Qg @ Qg.conj().T - U @ U.conj().T
    assert np.linalg.norm(P, 2) <= 10 * _tol_lambda(sig, form) / gap + 1e-10


def _stepwise(pr, m, form):
    """Every item of both bases, leaf and other, against its definition."""
    from dh2_export import exported_bases
    plan, M, ref = pr["plan"], pr["M"], pr["ref"]
    tr, dr = plan.tree, plan.dirs
    counts = dict(leaf=0, inner=0, tie=0)
    worst = 0.0
    exp = {}
    for side in (0, 1):
        sets = plan.rowsets if side == 0 else plan.colsets
        basis_ref = ref.V if side == 0 else ref.W
        Mo = M if side == 0 else OM.AdjointMatrix(M)
        data, Qexp = exported_bases(m, plan, side)
        exp[side] = Qexp
        for (t, c), (k, mat, sig) in data.items():
            A = OC.weighted_block_row(Mo, plan, sets, t, c, ref.omega, ZETA)
            if tr.son1[t] < 0:
                U, s, kr = OC.truncated_left_singular(A, EPS)
                assert np.allclose(s, basis_ref.sigma[(t, c)], rtol=1e-12,
                                   atol=1e-14 * (s[0] if len(s) else 1.0))
                counts["leaf"] += 1
            else:
                cp = int(dr.sd[tr.level[t]][c])
                parts = []
                for ts in tr.sons(t):
                    loc = tr.rows(ts) - tr.off[t]
                    parts.append(Qexp[(ts, cp)].conj().T @ A[loc, :])
                Ghat = np.vstack(parts)
                U, s, kr = OC.truncated_left_singular(Ghat, EPS)
                counts["inner"] += 1
            tie, dw = _sigma_check(sig, s, form)
            worst = max(worst, dw)
            if tie:
                counts["tie"] += 1
                assert abs(k - kr) <= 1, (side, t, c)
                continue
            assert k == kr, (side, t, c, k, kr)
            _projector_check(mat, U, s, k, form)
    return counts, worst, exp


CASES = [(p, g, f) for p in PROBLEMS for g in (2, 3) for f in ("fp64", "mixed")]


@pytest.mark.parametrize("name,groups,form", CASES)
def test_subtree_groups(name, groups, form):
    from dh2_export import exported_dense
    from paper_1510_07087_amd import dh2
    pr = _problem(name)
    plan, ref, G = pr["plan"], pr["ref"], pr["G"]
    tr, bt = plan.tree, plan.blocks
    n = tr.n
    print(f"[gpu groups] {name} groups={groups} {form}", flush=True)
    o = dh2.opts(leaf_size=32, groups=groups,
                 precision=dh2.MIXED if form == "mixed" else dh2.FP64)
    b = dh2.blocks_build(dh2.tree_build(pr["p"], pr["kappa"], o), o)
    m = dh2.compress_helmholtz(b, pr["w"], EPS, o)
    torch.cuda.synchronize()
    st = dh2.stats(m)
    assert st["groups"] == groups

    counts, worst, exp = _stepwise(pr, m, form)
    assert counts["inner"] > 0 and counts["leaf"] > 0
    assert counts["tie"] < (counts["leaf"] + counts["inner"]) // 20
    print(f"[gpu groups] {name} g{groups} {form}: {counts}, worst sigma dev {worst:.2e}",
          flush=True)

    # coupling matrices against their definition with the library's bases, and
    # V S W^* against the oracle's per block
    Gt, V, W, S = exported_dense(m, plan)
    Gp = G[np.ix_(tr.perm, tr.perm)]
    s_worst, blk_worst = 0.0, 0.0
    for q in range(len(bt.adm_t)):
        t, s, c = int(bt.adm_t[q]), int(bt.adm_s[q]), int(bt.adm_c[q])
        Gb = Gp[np.ix_(tr.rows(t), tr.rows(s))]
        om = ref.omega[q]
        Vg, Wg = V[(t, c)], W[(s, c)]
        Sdef = Vg.conj().T @ Gb @ Wg
        ds = np.linalg.norm(S[q] - Sdef, 2) / om if S[q].size else 0.0
        s_worst = max(s_worst, ds)
        assert ds <= S_TOL[form], (q, ds)
        Vo, Wo = ref.V.Qexp[(t, c)], ref.W.Qexp[(s, c)]
        approx_g = Vg @ S[q] @ Wg.conj().T
        approx_o = Vo @ ref.S[q] @ Wo.conj().T
        diff = np.linalg.norm(approx_g - approx_o, 2)
        dP = np.linalg.norm(Vg @ Vg.conj().T - Vo @ Vo.conj().T, 2)
        dQ = np.linalg.norm(Wg @ Wg.conj().T - Wo @ Wo.conj().T, 2)
        g2 = np.linalg.norm(Gb, 2)
        assert diff <= (dP + dQ) * g2 + (S_TOL[form] + 1e-12) * om, (q, diff / om)
        blk_worst = max(blk_worst, diff / om)
    print(f"[gpu groups] {name} g{groups} {form}: |S - V^*GW| <= {s_worst:.1e} omega, "
          f"|VSW^* - oracle| <= {blk_worst:.1e} omega", flush=True)

    err = np.linalg.norm(G - Gt, 2) / np.linalg.norm(G, 2)
    err_ref = np.linalg.norm(G - OD.reconstruct(ref), 2) / np.linalg.norm(G, 2)
    print(f"[gpu groups] {name} g{groups} {form}: rel err {err:.3e} oracle {err_ref:.3e}",
          flush=True)
    assert err <= 1.1 * EPS
    assert 0.9 * err_ref <= err <= 1.1 * err_ref + 1e-3 * EPS

    x = synth.complex_gaussian(n, 5)
    xd = torch.from_numpy(x).to("cuda")
    for op, A in (("N", Gt), ("C", Gt.conj().T)):
        yd = torch.empty_like(xd)
        dh2.matvec(m, op, xd, yd)
        refy = A @ x
        assert np.linalg.norm(yd.cpu().numpy() - refy) <= 1e-10 * np.linalg.norm(refy), op
