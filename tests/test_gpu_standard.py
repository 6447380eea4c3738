"""Standard admissibility (condition (c) alone, as in the paper's comparison
with cross approximation) at the sizes where the ranks grow large: the
32768-point sphere (kappa 32) in both forms and the 131072-point sphere
(kappa 64) in the FP64 form, leaf 64, eps 1e-4.  Transfer factors reach
r = k1 + k2 well above 128 rows there, so the factorisations and transfer
R-products of the largest block rows run on the kernels that stage their
operands in device memory.

Checks against the FP64 oracle, with the tolerances of test_gpu_large:
* sampled leaf block rows (singular values, ranks, projectors);
* sampled block rows one level above the leaves, G_hat formed by definition
  from the library's son bases;
* sampled block rows with r > 128: G_hat formed by definition from the
  library's expanded son bases and the oracle's weighted block row;
* sampled admissible blocks against the error theorem's per-block bound
  ||G|_b - V S W^*||_2 <= sqrt(2) eps omega_b / sqrt(1 - 2 zeta^2) (the
  bound the paper proves; V, W expanded from the library's export, G|_b
  from the oracle);
* 16 rows against the direct FP64 sum, and the relative spectral error by
  power iteration: <= 1.1 eps at n = 32768; at n = 131072 the paper gives
  no global bound for block-relative tolerances (the blocks of one block
  row add their errors, and standard admissibility puts a few large blocks
  in every row), so the global error is reported and held below 2 eps as a
  regression guard.
"""
import numpy as np
import pytest

import synth
from oracle import compress as OC
from oracle import matrix as OM
from oracle import plan as OP
from test_gpu_large import _sampled_inner_rows, _sampled_leaf_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ZETA = 2.0 / 3.0
_cache = {}


def _problem(name):
    if name not in _cache:
        p, w, kappa, leaf, eps = synth.workload(name)
        eps = 1e-4
        plan = OP.build_plan(p, kappa, leaf, standard_only=True)
        M = OM.HelmholtzMatrix(p, w, kappa, plan.tree.perm)
        _cache[name] = dict(p=p, w=w, kappa=kappa, leaf=leaf, eps=eps, plan=plan, M=M)
    return _cache[name]


def _sampled_big_rows(pr, m, form, nsample, seed):
    """Block rows whose factor has more than 128 rows (k1 + k2 > 128):
    G_hat = [V_t1^* G^w|t1; V_t2^* G^w|t2] with the library's expanded son
    bases V (expanded from its exported leaf factors and transfer matrices)
    against the library's singular values, rank and projector."""
    from paper_1510_07087_amd import dh2
    plan, M, eps = pr["plan"], pr["M"], pr["eps"]
    tr, bt, dr = plan.tree, plan.blocks, plan.dirs
    rng = np.random.default_rng(seed)
    nbig = done = 0
    for side in (0, 1):
        sets = plan.rowsets if side == 0 else plan.colsets
        ex = dh2.basis_export(m, side)
        index = {(int(t), int(c)): i for i, (t, c) in enumerate(zip(ex["item_t"], ex["item_c"]))}

        def mat(i):
            r, k, mo = int(ex["item_r"][i]), int(ex["item_k"][i]), int(ex["mat_off"][i])
            return ex["mat"][mo:mo + r * k].reshape(r, k)

        memo = {}

        def expanded(t, c):
            if (t, c) not in memo:
                F = mat(index[(t, c)])
                if tr.son1[t] < 0:
                    memo[(t, c)] = F
                else:
                    cp = int(dr.sd[tr.level[t]][c])
                    parts, o = [], 0
                    for ts in tr.sons(t):
                        Vs = expanded(ts, cp)
                        parts.append(Vs @ F[o:o + Vs.shape[1], :])
                        o += Vs.shape[1]
                    memo[(t, c)] = np.vstack(parts)
            return memo[(t, c)]

        big = [(t, c) for (t, c), i in index.items() if int(ex["item_r"][i]) > 128]
        nbig += len(big)
        if not big:
            continue
        # the smallest clusters first (cheapest by definition), then random
        big.sort(key=lambda tc: (tr.size[tc[0]], tc))
        cand = big[:4 * nsample]
        pick = rng.choice(len(cand), size=min(nsample, len(cand)), replace=False)
        Mo = M if side == 0 else OM.AdjointMatrix(M)
        for q in pick:
            t, c = cand[q]
            omega = {}
            for (b, s, d) in sets.F[t][c]:
                if b not in omega:
                    omega[b] = np.linalg.norm(M.block(tr.rows(bt.adm_t[b]), tr.rows(bt.adm_s[b])))
            A = OC.weighted_block_row(Mo, plan, sets, t, c, omega, ZETA)
            cp = int(dr.sd[tr.level[t]][c])
            parts = []
            for ts in tr.sons(t):
                loc = tr.rows(ts) - tr.off[t]
                parts.append(expanded(ts, cp).conj().T @ A[loc, :])
            Ghat = np.vstack(parts)
            U, sig, k = OC.truncated_left_singular(Ghat, eps)
            i = index[(t, c)]
            r, kg = int(ex["item_r"][i]), int(ex["item_k"][i])
            assert r == Ghat.shape[0] and r > 128
            so = int(ex["sig_off"][i])
            sg = ex["sigma"][so:so + r]
            fro = float(np.sqrt(np.sum(sig ** 2)))
            n_ = min(len(sg), len(sig))
            big_ = sig[:n_] > eps
            if form == "mixed":
                d = np.abs(sg[:n_][big_] - sig[:n_][big_]) / fro
                assert np.all(d <= 2e-7), (side, t, c, d.max())
                tie = np.any(np.abs(sig - eps) <= 2e-7 * fro)
                tl = 2.0 * sig[0] * 2e-7 * fro + 1e-13 * fro ** 2
            else:
                tl = 1e-13 * fro ** 2 + max(1e-4 * eps ** 2,
                                            64 * 2.220446049250313e-16 * r * fro ** 2)
                d = np.abs(sg[:n_][big_] ** 2 - sig[:n_][big_] ** 2)
                assert np.all(d <= tl + 1e-10 * sig[:n_][big_] ** 2), (side, t, c)
                tie = np.any(np.abs(sig ** 2 - eps ** 2) <= tl + 1e-10 * eps ** 2)
            done += 1
            if tie:
                assert abs(kg - k) <= 1
                continue
            assert kg == k, (side, t, c, kg, k)
            if k:
                P = mat(i) @ mat(i).conj().T - U[:, :k] @ U[:, :k].conj().T
                gap = sig[k - 1] ** 2 - (sig[k] ** 2 if k < len(sig) else 0.0)
                assert np.linalg.norm(P, 2) <= 10 * tl / gap + 1e-10, (side, t, c)
    return nbig, done


def _sampled_block_bounds(pr, m, nsample, seed):
    """Admissible blocks between small clusters: ||G|_b - V S W^*||_2 against
    the per-block bound of the error theorem; returns the largest ratio."""
    from paper_1510_07087_amd import dh2
    plan, M, eps = pr["plan"], pr["M"], pr["eps"]
    tr, bt, dr = plan.tree, plan.blocks, plan.dirs
    bound = np.sqrt(2.0) * eps / np.sqrt(1.0 - 2.0 * ZETA ** 2)
    ex = [dh2.basis_export(m, side) for side in (0, 1)]
    idx = [{(int(t), int(c)): i for i, (t, c) in enumerate(zip(e["item_t"], e["item_c"]))}
           for e in ex]

    def expanded(side, t, c):
        e, i = ex[side], idx[side][(t, c)]
        r, k, mo = int(e["item_r"][i]), int(e["item_k"][i]), int(e["mat_off"][i])
        F = e["mat"][mo:mo + r * k].reshape(r, k)
        if tr.son1[t] < 0:
            return F
        cp = int(dr.sd[tr.level[t]][c])
        parts, o = [], 0
        for ts in tr.sons(t):
            Vs = expanded(side, ts, cp)
            parts.append(Vs @ F[o:o + Vs.shape[1], :])
            o += Vs.shape[1]
        return np.vstack(parts)

    nadm = len(bt.adm_t)
    soff, S = dh2.coupling_export(m, nadm)
    small = [b for b in range(nadm) if tr.size[bt.adm_t[b]] * tr.size[bt.adm_s[b]] <= 256 * 256]
    rng = np.random.default_rng(seed)
    worst = 0.0
    for b in rng.choice(len(small), size=min(nsample, len(small)), replace=False):
        b = small[b]
        t, s_, c = int(bt.adm_t[b]), int(bt.adm_s[b]), int(bt.adm_c[b])
        V, W = expanded(0, t, c), expanded(1, s_, c)
        kt, ks = V.shape[1], W.shape[1]
        Sb = S[soff[b]:soff[b + 1]].reshape(ks, kt).T if kt * ks else np.zeros((kt, ks))
        Gb = M.block(tr.rows(t), tr.rows(s_))
        om = np.linalg.norm(Gb)
        ratio = np.linalg.norm(Gb - V @ Sb @ W.conj().T, 2) / (bound * om)
        assert ratio <= 1.0, (b, ratio)
        worst = max(worst, ratio)
    return worst


CASES = [("sphere32768", "fp64"), ("sphere32768", "mixed"), ("sphere131072", "fp64")]


@pytest.mark.parametrize("name,form", CASES)
def test_standard_admissibility_large(name, form):
    from paper_1510_07087_amd import dh2
    pr = _problem(name)
    eps, n = pr["eps"], len(pr["p"])
    print(f"[gpu standard] {name} {form}: n={n} kappa={pr['kappa']}", flush=True)
    o = dh2.opts(leaf_size=pr["leaf"], standard_only=1,
                 precision=dh2.MIXED if form == "mixed" else dh2.FP64)
    b = dh2.blocks_build(dh2.tree_build(pr["p"], pr["kappa"], o), o)
    m = dh2.compress_helmholtz(b, pr["w"], eps, o)
    torch.cuda.synchronize()
    st = dh2.stats(m)
    print(f"[gpu standard] {name} {form}: k_max {st['k_max']}, {st['mem_per_n_kib']:.1f} KiB "
          f"per point, {st['t_total']:.3f} s, groups {st['groups']}", flush=True)
    nbig, done = _sampled_big_rows(pr, m, form, 3, 11)
    print(f"[gpu standard] {name} {form}: {nbig} block rows with r > 128, {done} checked",
          flush=True)
    assert nbig > 0 and done > 0
    w1 = _sampled_leaf_rows(pr, m, form, 8, 7)
    w2 = _sampled_inner_rows(pr, m, form, 4, 8)
    print(f"[gpu standard] {name} {form}: sampled rows agree ({w1:.2e}, {w2:.2e})", flush=True)
    worst = _sampled_block_bounds(pr, m, 6, 13)
    print(f"[gpu standard] {name} {form}: sampled blocks within the per-block bound "
          f"(worst {worst:.2f} of it)", flush=True)
    err = dh2.error_estimate(m, None, iters=8, seed=1)
    rows = np.random.default_rng(5).choice(n, 16, replace=False)
    x = torch.from_numpy(synth.complex_gaussian(n, 6)).to("cuda")
    _, _, rows_rel = dh2.rows_check(m, rows, x)
    print(f"[gpu standard] {name} {form}: rel err {err:.3e}, 16 rows {rows_rel:.3e}", flush=True)
    assert err <= (1.1 if n <= 32768 else 2.0) * eps
    assert rows_rel <= 10 * eps
