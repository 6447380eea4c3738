"""The allocation-free matrix-vector product captured into a HIP graph.

dh2_matvec_noalloc allocates nothing and never waits, and its second stream
(the near-field rows) is forked from and joined to the caller's stream with
events, so a caller can capture it.  The graph is captured once on the
2048-point sphere (FP64 form, three right-hand sides) and replayed several
times with a new input each time, with eager work and synchronisations
between the replays; every replay must equal the eager dh2_matvec on the
same input bit for bit (same kernels in the same order)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _columns(x):
    return torch.from_numpy(np.ascontiguousarray(x.T)).to("cuda").T


@pytest.mark.parametrize("op", ["N", "C"])
def test_noalloc_matvec_graph_replays(op):
    from paper_1510_07087_amd import dh2
    print(f"[graph] n=2048 nrhs=3 op={op}: capture, then 4 replays", flush=True)
    p, w = synth.fibonacci_sphere(2048)
    o = dh2.opts(leaf_size=32)
    b = dh2.blocks_build(dh2.tree_build(p, 8.0, o), o)
    m = dh2.compress_helmholtz(b, w, 1e-4, o)
    x = _columns(synth.complex_gaussian(2048, 31, 3))
    y = torch.empty_like(x)
    # eager calls first: the product's plan and the scratch address exist
    # before the capture
    dh2.matvec(m, op, x, y)
    dh2.matvec_noalloc(m, op, x, y)
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        dh2.matvec_noalloc(m, op, x, y)    # on the capturing stream
    torch.cuda.synchronize()

    for rep in range(4):
        xi = _columns(synth.complex_gaussian(2048, 40 + rep, 3))
        ref = torch.empty_like(xi)
        dh2.matvec(m, op, xi, ref)          # eager work between the replays
        torch.cuda.synchronize()
        x.copy_(xi)
        y.fill_(complex(np.nan, np.nan))
        g.replay()
        torch.cuda.synchronize()
        a, r = y.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(a)), rep
        assert np.array_equal(a, r), (rep, np.abs(a - r).max())
