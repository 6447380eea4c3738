"""The double-layer workload (Section 7, the DLP matrix) on the GPU, with
entries generated on the device from points and normals (FP64 and mixed
form) and through the dense input (FP64), against the oracle's compression
of the same entries: 2048 points on the sphere and on the rotated ellipsoid
(kappa 8, leaf 32, eps 1e-4).  Mixed form: |sigma_gpu - sigma| <= 2e-7
||A||_F (the FP32 rounding of each entry and the FP32 R-products, as in
test_gpu_parity).

Checks and tolerances as in test_gpu_parity: singular values and ranks of
every block row (|sigma_gpu^2 - sigma^2| <= 1e-13 ||A||_F^2 + 1e-10 sigma^2
plus the pivoted Cholesky's cut 1e-4 eps^2), global relative spectral error
<= 1.1 eps and within 10 % of the oracle's, matrix-vector products against
the dense reconstruction of the exported representation to 1e-10.
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
N = 2048


def _surface(name):
    if name == "sphere":
        p, w = synth.fibonacci_sphere(N)
        return p, synth.sphere_normals(p), w
    p, w = synth.ellipsoid(N)
    return p, synth.ellipsoid_normals(N), w


@pytest.fixture(scope="module", params=["sphere", "ellipsoid"])
def surface(request):
    p, nv, w = _surface(request.param)
    plan = OP.build_plan(p, KAPPA, 32)
    M = OM.HelmholtzDLPMatrix(p, nv, w, KAPPA, plan.tree.perm)
    ref = OC.compress(M, plan, EPS, ZETA)
    G = OM.dlp_dense_original(p, nv, w, KAPPA)
    return dict(name=request.param, p=p, nv=nv, w=w, plan=plan, ref=ref, G=G)


@pytest.fixture(scope="module", params=["generated", "dense", "mixed"])
def dlp(request, surface):
    from paper_1510_07087_amd import dh2
    from dh2_export import exported_bases, exported_dense
    print(f"[gpu dlp] {surface['name']}: {request.param}", flush=True)
    o = dh2.opts(leaf_size=32, precision=dh2.MIXED if request.param == "mixed" else dh2.FP64)
    b = dh2.blocks_build(dh2.tree_build(surface["p"], KAPPA, o), o)
    if request.param == "dense":
        Gd = torch.from_numpy(surface["G"]).to("cuda")
        m = dh2.compress_dense(b, Gd, EPS, o)
    else:
        m = dh2.compress_helmholtz_dlp(b, surface["w"], surface["nv"], EPS, o)
    torch.cuda.synchronize()
    plan = surface["plan"]
    Gt = exported_dense(m, plan)[0]
    dv, _ = exported_bases(m, plan, 0)
    dw, _ = exported_bases(m, plan, 1)
    return dict(name=surface["name"], mode=request.param, ref=surface["ref"], G=surface["G"],
                m=m, Gt=Gt, dv=dv, dw=dw, p=surface["p"])


def test_singular_values_and_ranks(dlp):
    ref = dlp["ref"]
    mixed = dlp["mode"] == "mixed"
    n_checked = n_tie = 0
    for basis_ref, data in ((ref.V, dlp["dv"]), (ref.W, dlp["dw"])):
        assert set(basis_ref.sigma) == set(data)
        for key, sig_ref in basis_ref.sigma.items():
            k, _, sig = data[key]
            fro2 = float(np.sum(sig_ref ** 2))
            # rounding band plus the pivoted Cholesky's cut: the Schur
            # complement it leaves has diagonal below tau = max(1e-4 eps^2 / r,
            # 64 u max M_ii) and norm at most its trace r tau (Weyl's theorem)
            tl = 1e-13 * fro2 + max(1e-4 * EPS ** 2,
                                    64 * 2.220446049250313e-16 * len(sig_ref) * fro2)
            s_ref = np.zeros(len(sig))
            s_ref[:min(len(sig_ref), len(sig))] = sig_ref[:len(sig)]
            big = s_ref > EPS
            if mixed:
                d = np.abs(sig[big] - s_ref[big]) / np.sqrt(fro2)
                assert np.all(d <= 2e-7), (key, d.max())
                tie = np.any(np.abs(sig_ref - EPS) <= 2e-7 * np.sqrt(fro2))
            else:
                d = np.abs(sig[big] ** 2 - s_ref[big] ** 2)
                assert np.all(d <= tl + 1e-10 * s_ref[big] ** 2), (key, d.max(), tl)
                tie = np.any(np.abs(sig_ref ** 2 - EPS ** 2) <= tl + 1e-10 * EPS ** 2)
            if tie:
                n_tie += 1
                assert abs(k - basis_ref.k[key]) <= 1
            else:
                assert k == basis_ref.k[key], (key, k, basis_ref.k[key])
            n_checked += 1
    assert n_checked >= 200
    assert n_tie < n_checked // 20


def test_global_error(dlp):
    G = dlp["G"]
    nG = np.linalg.norm(G, 2)
    err = np.linalg.norm(G - dlp["Gt"], 2) / nG
    err_ref = np.linalg.norm(G - OD.reconstruct(dlp["ref"]), 2) / nG
    print(f"[gpu dlp] {dlp['name']} {dlp['mode']}: rel err gpu {err:.3e} oracle {err_ref:.3e}",
          flush=True)
    assert err <= 1.1 * EPS
    assert 0.9 * err_ref <= err <= 1.1 * err_ref + 1e-3 * EPS


def test_matvec(dlp):
    from paper_1510_07087_amd import dh2
    Gt = dlp["Gt"]
    x = synth.complex_gaussian(N, 5)
    xd = torch.from_numpy(x).to("cuda")
    for op, A in (("N", Gt), ("C", Gt.conj().T)):
        yd = torch.empty_like(xd)
        dh2.matvec(dlp["m"], op, xd, yd)
        y = yd.cpu().numpy()
        ref = A @ x
        assert np.linalg.norm(y - ref) <= 1e-10 * np.linalg.norm(ref), op


def test_error_estimate_and_rows(dlp):
    """Entries regenerated on the device for the error estimate and the
    direct rows agree with the dense matrix.  The estimate is a ratio of two
    power iterations; with G = I/2 + K the largest singular values of G
    cluster near 1/2, so the denominator converges slowly from below and the
    ratio may exceed the exact one by a little (observed 0.2 %)."""
    from paper_1510_07087_amd import dh2
    if dlp["mode"] == "dense":
        pytest.skip("regeneration from points needs the generated input")
    G = dlp["G"]
    exact = np.linalg.norm(G - dlp["Gt"], 2) / np.linalg.norm(G, 2)
    est = dh2.error_estimate(dlp["m"], None, iters=60, seed=1)
    assert 0.5 * exact <= est <= 1.05 * exact
    x = synth.complex_gaussian(N, 6)
    rows = np.random.default_rng(5).choice(N, 16, replace=False)
    direct, approx, _ = dh2.rows_check(dlp["m"], rows, torch.from_numpy(x).to("cuda"))
    assert np.allclose(direct, (G @ x)[rows], rtol=0, atol=1e-12 * np.abs(G @ x).max())

