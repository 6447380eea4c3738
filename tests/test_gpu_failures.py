"""Failure paths of the compression, forced from the host so that every
kernel still ends normally: a device-memory cap below what the compression
needs (DH2_ENOMEM) and a Jacobi sweep limit of one (DH2_ENOTCONV).  On
failure the output handle is left untouched, the message names the cause,
and the library stays usable: the next compression of the same blocks
succeeds and equals the one before the failures."""
import ctypes as C

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SENTINEL = 0x5A5A5A5A


def _raw_compress(dh2, b, w, eps, o):
    h = C.c_void_p(SENTINEL)
    wa = np.ascontiguousarray(w, dtype=np.float64)
    code = dh2.lib().dh2_compress_helmholtz(
        b.h, wa.ctypes.data_as(C.POINTER(C.c_double)), float(eps), C.byref(o),
        C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(h))
    return code, h.value, dh2.lib().dh2_last_error().decode()


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_failures_leave_output_untouched(form):
    from paper_1510_07087_amd import dh2
    print(f"[gpu failures] {form}: n=2048", flush=True)
    p, w = synth.fibonacci_sphere(2048)
    prec = dh2.MIXED if form == "mixed" else dh2.FP64
    o = dh2.opts(leaf_size=32, precision=prec)
    b = dh2.blocks_build(dh2.tree_build(p, 8.0, o), o)
    before = dh2.compress_helmholtz(b, w, 1e-4, o)
    torch.cuda.synchronize()
    x = torch.from_numpy(synth.complex_gaussian(2048, 9)).to("cuda")
    y0 = torch.empty_like(x)
    dh2.matvec(before, "N", x, y0)

    # device-memory cap of 1 MiB: the point data alone need more
    code, h, msg = _raw_compress(dh2, b, w, 1e-4, dh2.opts(leaf_size=32, precision=prec,
                                                              max_device_bytes=1 << 20))
    assert code == -2 and h == SENTINEL, (code, msg)
    assert "cap" in msg
    # one Jacobi sweep: the small SVDs still rotate after it
    code, h, msg = _raw_compress(dh2, b, w, 1e-4, dh2.opts(leaf_size=32, precision=prec,
                                                              max_sweeps=1))
    assert code == -4 and h == SENTINEL, (code, msg)
    assert "Jacobi" in msg

    after = dh2.compress_helmholtz(b, w, 1e-4, o)
    torch.cuda.synchronize()
    y1 = torch.empty_like(x)
    dh2.matvec(after, "N", x, y1)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    # a generous sweep limit is no failure
    ok = dh2.compress_helmholtz(b, w, 1e-4, dh2.opts(leaf_size=32, precision=prec,
                                                     max_sweeps=200))
    torch.cuda.synchronize()
    assert dh2.stats(ok)["k_max"] == dh2.stats(before)["k_max"]
