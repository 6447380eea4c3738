"""The C-ABI library loads and exports every symbol include/dh2.h declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dh2.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(dh2_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("dh2_tree_build", "dh2_blocks_build", "dh2_compress_dense",
                 "dh2_compress_helmholtz", "dh2_matvec", "dh2_error_estimate",
                 "dh2_rows_check", "dh2_get_stats", "dh2_basis_export"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1510_07087_amd import dh2
    L = dh2.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(dh2.EXPORTED)


def test_no_oracle_import_in_product():
    """The product path never imports or reads the oracle."""
    pkg = os.path.join(ROOT, "paper_1510_07087_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f


def test_missing_library_fails_loudly(monkeypatch):
    """No CPU fallback: without the built library every call raises."""
    from paper_1510_07087_amd import dh2
    monkeypatch.setattr(dh2, "_lib", None)
    monkeypatch.setattr(dh2, "LIB_PATH", os.path.join(ROOT, "no_such_libdh2.so"))
    with pytest.raises(RuntimeError, match="native library missing"):
        dh2.lib()


def test_opts_layout_matches_library():
    """dh2_opts_default fills exactly the binding's structure (no write past
    it) with the documented defaults."""
    import ctypes as C
    from paper_1510_07087_amd import dh2
    n = C.sizeof(dh2.Opts)
    buf = (C.c_ubyte * (n + 64))(*([0xA5] * (n + 64)))
    dh2.lib().dh2_opts_default(C.cast(buf, C.POINTER(dh2.Opts)))
    assert all(b == 0xA5 for b in bytes(buf)[n:])
    o = dh2.Opts.from_buffer(buf)
    assert (o.leaf_size, o.eta1, o.eta2, o.precision, o.weights) == (32, 20.0, 5.0, dh2.FP64,
                                                                      dh2.WEIGHTS_BLOCK)
    assert abs(o.zeta - 2.0 / 3.0) < 1e-16 and o.max_device_bytes == 0 and o.groups == 0
    assert o.max_sweeps == 0


def test_invalid_options_rejected():
    """Options are checked before any work: unknown weights, bad eta and zeta."""
    import numpy as np
    from paper_1510_07087_amd import dh2
    pts = np.random.default_rng(0).standard_normal((8, 3))
    for kw in (dict(weights=7), dict(eta2=0.0), dict(zeta=0.8), dict(leaf_size=0),
               dict(max_sweeps=-1)):
        with pytest.raises(dh2.DH2Error) as e:
            dh2.tree_build(pts, 1.0, dh2.opts(**kw))
        assert e.value.code == -1, kw  # DH2_EINVAL
