"""Degenerate inputs on the GPU, both forms (kappa 8, leaf 32, eps 1e-4):

* one point, and 17 points (a single leaf): no admissible block, the whole
  matrix is near field and comes back exactly;
* the 2048-point sphere plus one far point, which bisection puts in a
  one-point leaf: that leaf's block with itself stays in the near field
  (separated boxes only); the result matches the oracle's.

The near field is generated in FP64 in both forms (about ten roundings per
entry, so 4e-15 relative) and stored as complex FP64 (FP64 form) or complex
FP32 (mixed form: each component rounded to nearest, relative 2^-24, so the
product is off by at most 2^-24 ||G||_F ||x|| more); the other tolerances
are those of test_gpu_parity.
"""
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
KAPPA = 8.0


def _outlier(n=2048):
    p, w = synth.fibonacci_sphere(n)
    return np.vstack([p, [[5.0, 0.0, 0.0]]]), np.append(w, w[0])


def _compress(p, w, form):
    from paper_1510_07087_amd import dh2
    o = dh2.opts(leaf_size=32, precision=dh2.MIXED if form == "mixed" else dh2.FP64)
    b = dh2.blocks_build(dh2.tree_build(p, KAPPA, o), o)
    m = dh2.compress_helmholtz(b, w, EPS, o)
    torch.cuda.synchronize()
    return m, dh2.blocks_info(b)


def _apply(m, x, op):
    from paper_1510_07087_amd import dh2
    xd = torch.from_numpy(x).to("cuda")
    yd = torch.empty_like(xd)
    dh2.matvec(m, op, xd, yd)
    return yd.cpu().numpy()


@pytest.mark.parametrize("form", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [1, 17])
def test_near_field_only(n, form):
    print(f"[gpu edges] n={n} {form}", flush=True)
    p, w = synth.fibonacci_sphere(n)
    m, info = _compress(p, w, form)
    assert info["nadm"] == 0 and info["nnear"] == 1
    G = OM.helmholtz_dense_original(p, w, KAPPA)
    x = synth.complex_gaussian(n, 5)
    store = 2.0 ** -24 * np.linalg.norm(G) * np.linalg.norm(x) if form == "mixed" else 0.0
    for op, A in (("N", G), ("C", G.conj().T)):
        y = _apply(m, x, op)
        ref = A @ x
        bound = 4e-15 * np.linalg.norm(ref) * max(1.0, np.sqrt(n)) + store
        assert np.linalg.norm(y - ref) <= bound, op


@pytest.fixture(scope="module")
def outlier():
    p, w = _outlier()
    plan = OP.build_plan(p, KAPPA, 32)
    M = OM.HelmholtzMatrix(p, w, KAPPA, plan.tree.perm)
    ref = OC.compress(M, plan, EPS, ZETA)
    G = OM.helmholtz_dense_original(p, w, KAPPA)
    return dict(p=p, w=w, plan=plan, ref=ref, G=G)


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_outlier_leaf(outlier, form):
    from dh2_export import exported_dense
    print(f"[gpu edges] sphere 2048 + outlier {form}", flush=True)
    plan, G = outlier["plan"], outlier["G"]
    tr, bt = plan.tree, plan.blocks
    one = [t for t in range(tr.nc) if tr.size[t] == 1]
    assert one and len(bt.adm_t) > 0
    assert any(int(t) == one[0] and int(s) == one[0] for t, s in zip(bt.near_t, bt.near_s))
    m, info = _compress(outlier["p"], outlier["w"], form)
    assert info["nadm"] == len(bt.adm_t) and info["nnear"] == len(bt.near_t)
    Gt = exported_dense(m, plan)[0]
    assert np.all(np.isfinite(Gt))
    nG = np.linalg.norm(G, 2)
    err = np.linalg.norm(G - Gt, 2) / nG
    err_ref = np.linalg.norm(G - OD.reconstruct(outlier["ref"]), 2) / nG
    print(f"[gpu edges] outlier {form}: rel err gpu {err:.3e} oracle {err_ref:.3e}", flush=True)
    assert err <= 1.1 * EPS
    assert 0.9 * err_ref <= err <= 1.1 * err_ref + 1e-3 * EPS
    x = synth.complex_gaussian(len(outlier["p"]), 5)
    for op, A in (("N", Gt), ("C", Gt.conj().T)):
        y = _apply(m, x, op)
        ref = A @ x
        assert np.linalg.norm(y - ref) <= 1e-10 * np.linalg.norm(ref), op
