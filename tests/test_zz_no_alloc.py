"""The allocation-free matrix-vector product (dh2_matvec_noalloc) against
dh2_matvec, called through the C ABI on two calls in a row: first the
2048-point sphere with three right-hand sides, then a smaller matrix (the
1024-point sphere, one right-hand side) reusing the same static scratch array.
Both products run the same kernels in the same order, so the results must be
identical; the FP64 matvec tolerance of the parity tests (1e-10 relative)
would be the bar otherwise.  Also: the refusal before the product's index
lists exist."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _matrix(n, kappa, leaf, eps=1e-4):
    from paper_1510_07087_amd import dh2
    p, w = synth.fibonacci_sphere(n)
    o = dh2.opts(leaf_size=leaf)
    b = dh2.blocks_build(dh2.tree_build(p, kappa, o), o)
    m = dh2.compress_helmholtz(b, w, eps, o)
    torch.cuda.synchronize()
    return m


def _columns(x):
    """(n, nrhs) complex128 on the device, column-major as the ABI expects."""
    return torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda").T


def test_noalloc_matches_matvec_on_two_calls():
    from paper_1510_07087_amd import dh2
    print("[no-alloc] n=2048 nrhs=3 then n=1024 nrhs=1", flush=True)
    big = _matrix(2048, 8.0, 32)
    small = _matrix(1024, 6.0, 32)
    x3 = _columns(synth.complex_gaussian(2048, 21, 3))
    x1 = torch.from_numpy(synth.complex_gaussian(1024, 22)).to("cuda")
    # before any dh2_matvec on the matrix the plan is missing: refused
    with pytest.raises(dh2.DH2Error) as ei:
        dh2.matvec_noalloc(big, "N", x3, torch.empty_like(x3))
    assert ei.value.code == -1
    for op in ("N", "C"):
        ref3 = torch.empty_like(x3)
        ref1 = torch.empty_like(x1)
        dh2.matvec(big, op, x3, ref3)
        dh2.matvec(small, op, x1, ref1)
        y3 = torch.full_like(x3, complex(np.nan, np.nan))
        y1 = torch.full_like(x1, complex(np.nan, np.nan))
        dh2.matvec_noalloc(big, op, x3, y3)
        dh2.matvec_noalloc(small, op, x1, y1)
        torch.cuda.synchronize()
        for y, ref in ((y3, ref3), (y1, ref1)):
            a, b = y.cpu().numpy(), ref.cpu().numpy()
            assert np.all(np.isfinite(a))
            assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b), op
            assert np.array_equal(a, b), op
