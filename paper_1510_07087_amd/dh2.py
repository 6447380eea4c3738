"""Python binding of the C ABI in include/dh2.h (argument marshalling only).

Every computation happens in libdh2.so (host plan in C++, compression and
products in gfx950 kernels).  Device arrays are torch tensors on the current
HIP device; streams are torch streams.  The module fails loudly when the
native library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DH2_LIBRARY may name another build of the same library (the sanitizer
# build of build.py); by default the in-tree libdh2.so
LIB_PATH = os.environ.get("DH2_LIBRARY") or os.path.join(_HERE, "libdh2.so")

FP64, MIXED = 0, 1
WEIGHTS_BLOCK, WEIGHTS_GLOBAL, WEIGHTS_SPECTRAL = 0, 1, 2
_STATUS = {0: "DH2_OK", -1: "DH2_EINVAL", -2: "DH2_ENOMEM", -3: "DH2_EDEVICE",
           -4: "DH2_ENOTCONV", -5: "DH2_EUNSUPPORTED"}


class DH2Error(RuntimeError):
    """A non-zero dh2_status; ``code`` holds it."""

    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class Opts(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("eta1", C.c_double), ("eta2", C.c_double),
                ("zeta", C.c_double), ("precision", C.c_int32),
                ("lowfreq_zero_dir", C.c_int32), ("standard_only", C.c_int32),
                ("groups", C.c_int32), ("max_device_bytes", C.c_int64),
                ("weights", C.c_int32), ("max_sweeps", C.c_int32)]


class TreeInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("nclusters", C.c_int32), ("depth", C.c_int32),
                ("ndirs_total", C.c_int32), ("kappa", C.c_double)]


class BlocksInfo(C.Structure):
    _fields_ = [("nadm", C.c_int64), ("nnear", C.c_int64), ("near_entries", C.c_int64),
                ("items", C.c_int32 * 2), ("entries", C.c_int64 * 2)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("nadm", C.c_int64), ("nnear", C.c_int64),
                ("k_max", C.c_int32), ("items", C.c_int32 * 2), ("mem_bytes", C.c_double),
                ("mem_per_n_kib", C.c_double), ("t_row", C.c_double), ("t_col", C.c_double),
                ("t_prj", C.c_double), ("t_near", C.c_double), ("t_total", C.c_double),
                ("flops_row", C.c_double), ("flops_col", C.c_double),
                ("flops_prj", C.c_double), ("flops_gram", C.c_double),
                ("flops_rprod", C.c_double), ("t_gram_kernel", C.c_double),
                ("groups", C.c_int32), ("precision", C.c_int32),
                ("flops_gram_leaf", C.c_double), ("t_gram_leaf", C.c_double),
                ("n_gram_leaf", C.c_int32), ("pad", C.c_int32),
                ("flops_rprod_leaf", C.c_double), ("ops_gram_leaf_i8", C.c_double),
                ("repr_bytes", C.c_double)]


EXPORTED = [
    "dh2_opts_default", "dh2_last_error", "dh2_tree_build", "dh2_tree_free",
    "dh2_tree_get_info", "dh2_tree_export", "dh2_tree_directions", "dh2_blocks_build",
    "dh2_blocks_free", "dh2_blocks_get_info", "dh2_blocks_export", "dh2_blocks_colsets",
    "dh2_compress_dense", "dh2_compress_helmholtz", "dh2_compress_helmholtz_dlp",
    "dh2_compress_batch", "dh2_matrix_free",
    "dh2_matvec", "dh2_matvec_noalloc",
    "dh2_error_estimate", "dh2_rows_check", "dh2_get_stats", "dh2_basis_export",
    "dh2_coupling_export", "dh2_near_export", "dh2_release_cached_memory",
]

_lib = None


def lib():
    """Load libdh2.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"native library missing: {LIB_PATH} "
                           "(build it with: python -m paper_1510_07087_amd.build)")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D, VP = C.POINTER, C.c_int32, C.c_int64, C.c_double, C.c_void_p
    sig = {
        "dh2_opts_default": (None, [P(Opts)]),
        "dh2_last_error": (C.c_char_p, []),
        "dh2_tree_build": (I32, [P(D), I64, D, P(Opts), P(VP)]),
        "dh2_tree_free": (None, [VP]),
        "dh2_tree_get_info": (I32, [VP, P(TreeInfo)]),
        "dh2_tree_export": (I32, [VP, P(I64), P(I64), P(I64), P(I32), P(I32), P(I32), P(D),
                                  P(D), P(D), P(D)]),
        "dh2_tree_directions": (I32, [VP, I32, P(I32), P(D), P(I32)]),
        "dh2_blocks_build": (I32, [VP, P(Opts), P(VP)]),
        "dh2_blocks_free": (None, [VP]),
        "dh2_blocks_get_info": (I32, [VP, P(BlocksInfo)]),
        "dh2_blocks_export": (I32, [VP, P(I32), P(I32), P(I32), P(I32), P(I32)]),
        "dh2_blocks_colsets": (I32, [VP, I32, P(I32), P(I32), P(I64), P(I32), P(I32), P(I32)]),
        "dh2_compress_dense": (I32, [VP, VP, I64, D, P(Opts), VP, P(VP)]),
        "dh2_compress_helmholtz": (I32, [VP, P(D), D, P(Opts), VP, P(VP)]),
        "dh2_compress_helmholtz_dlp": (I32, [VP, P(D), P(D), D, P(Opts), VP, P(VP)]),
        "dh2_compress_batch": (I32, [I32, P(VP), P(P(D)), D, P(Opts), VP, P(VP)]),
        "dh2_matrix_free": (None, [VP]),
        "dh2_matvec": (I32, [VP, C.c_char, I64, VP, VP, VP]),
        "dh2_matvec_noalloc": (I32, [VP, C.c_char, I64, VP, VP, VP]),
        "dh2_error_estimate": (I32, [VP, VP, I64, I32, C.c_uint64, P(D), VP]),
        "dh2_rows_check": (I32, [VP, P(I64), I32, VP, P(D), P(D), P(D), VP]),
        "dh2_get_stats": (I32, [VP, P(Stats)]),
        "dh2_basis_export": (I32, [VP, I32, P(I32), P(I64), P(I64), P(I32), P(I32), P(I32),
                                   P(I32), P(I64), P(D), P(I64), P(D)]),
        "dh2_coupling_export": (I32, [VP, P(I64), P(D)]),
        "dh2_near_export": (I32, [VP, P(I64), P(D)]),
        "dh2_release_cached_memory": (None, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(code):
    if code != 0:
        raise DH2Error(code, lib().dh2_last_error().decode())


def _p(a, ct):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


def opts(**kw) -> Opts:
    """dh2_opts with the library defaults, overridden by keyword arguments."""
    o = Opts()
    lib().dh2_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


class _Handle:
    _free = None

    def __init__(self, h, keep=None):
        self.h = h
        self._keep = keep

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            getattr(_lib, self._free)(self.h)
            self.h = None


class Tree(_Handle):
    _free = "dh2_tree_free"


class Blocks(_Handle):
    _free = "dh2_blocks_free"


class Matrix(_Handle):
    _free = "dh2_matrix_free"


# ---------------------------------------------------------------------------
def tree_build(points, kappa: float, o: Opts) -> Tree:
    pts = np.ascontiguousarray(points, dtype=np.float64)
    h = C.c_void_p()
    _check(lib().dh2_tree_build(_p(pts, C.c_double), pts.shape[0], float(kappa), C.byref(o),
                                C.byref(h)))
    return Tree(h)


def tree_info(t: Tree) -> dict:
    info = TreeInfo()
    _check(lib().dh2_tree_get_info(t.h, C.byref(info)))
    return {f: getattr(info, f) for f, _ in TreeInfo._fields_}


def tree_export(t: Tree) -> dict:
    info = tree_info(t)
    n, nc, depth = info["n"], info["nclusters"], info["depth"]
    out = dict(perm=np.empty(n, np.int64), off=np.empty(nc, np.int64),
               size=np.empty(nc, np.int64), level=np.empty(nc, np.int32),
               son1=np.empty(nc, np.int32), son2=np.empty(nc, np.int32),
               lo=np.empty((nc, 3)), hi=np.empty((nc, 3)), diam=np.empty(nc),
               delta=np.empty(depth + 1))
    I64, I32, D = C.c_int64, C.c_int32, C.c_double
    _check(lib().dh2_tree_export(t.h, _p(out["perm"], I64), _p(out["off"], I64),
                                 _p(out["size"], I64), _p(out["level"], I32),
                                 _p(out["son1"], I32), _p(out["son2"], I32),
                                 _p(out["lo"], D), _p(out["hi"], D), _p(out["diam"], D),
                                 _p(out["delta"], D)))
    return out


def tree_directions(t: Tree, level: int):
    nd = C.c_int32()
    _check(lib().dh2_tree_directions(t.h, level, C.byref(nd), None, None))
    dirs = np.empty((nd.value, 3))
    sd = np.empty(nd.value, np.int32)
    _check(lib().dh2_tree_directions(t.h, level, C.byref(nd), _p(dirs, C.c_double),
                                     _p(sd, C.c_int32)))
    return dirs, sd


def blocks_build(t: Tree, o: Opts) -> Blocks:
    h = C.c_void_p()
    _check(lib().dh2_blocks_build(t.h, C.byref(o), C.byref(h)))
    return Blocks(h, keep=t)


def blocks_info(b: Blocks) -> dict:
    info = BlocksInfo()
    _check(lib().dh2_blocks_get_info(b.h, C.byref(info)))
    return dict(nadm=info.nadm, nnear=info.nnear, near_entries=info.near_entries,
                items=list(info.items), entries=list(info.entries))


def blocks_export(b: Blocks) -> dict:
    info = blocks_info(b)
    na, nn = info["nadm"], info["nnear"]
    out = {k: np.empty(na, np.int32) for k in ("adm_t", "adm_s", "adm_c")}
    out.update({k: np.empty(nn, np.int32) for k in ("near_t", "near_s")})
    I32 = C.c_int32
    _check(lib().dh2_blocks_export(b.h, _p(out["adm_t"], I32), _p(out["adm_s"], I32),
                                   _p(out["adm_c"], I32), _p(out["near_t"], I32),
                                   _p(out["near_s"], I32)))
    return out


def blocks_colsets(b: Blocks, side: int) -> dict:
    info = blocks_info(b)
    ni, ne = info["items"][side], info["entries"][side]
    out = dict(item_t=np.empty(ni, np.int32), item_c=np.empty(ni, np.int32),
               item_begin=np.empty(ni + 1, np.int64), ent_b=np.empty(ne, np.int32),
               ent_s=np.empty(ne, np.int32), ent_d=np.empty(ne, np.int32))
    I32, I64 = C.c_int32, C.c_int64
    _check(lib().dh2_blocks_colsets(b.h, side, _p(out["item_t"], I32), _p(out["item_c"], I32),
                                    _p(out["item_begin"], I64), _p(out["ent_b"], I32),
                                    _p(out["ent_s"], I32), _p(out["ent_d"], I32)))
    return out


def compress_helmholtz(b: Blocks, w, eps: float, o: Opts, stream=None) -> Matrix:
    wa = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    h = C.c_void_p()
    _check(lib().dh2_compress_helmholtz(b.h, _p(wa, C.c_double), float(eps), C.byref(o),
                                        _stream(stream), C.byref(h)))
    return Matrix(h, keep=b)


def compress_helmholtz_dlp(b: Blocks, w, normals, eps: float, o: Opts, stream=None) -> Matrix:
    """Double-layer operator generated from points, weights and unit normals
    (n x 3, original order); either form (o.precision)."""
    wa = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    na = np.ascontiguousarray(normals, dtype=np.float64)
    h = C.c_void_p()
    _check(lib().dh2_compress_helmholtz_dlp(b.h, _p(wa, C.c_double), _p(na, C.c_double),
                                            float(eps), C.byref(o), _stream(stream),
                                            C.byref(h)))
    return Matrix(h, keep=b)


def compress_batch(blocks, ws, eps: float, o: Opts, stream=None):
    """Independent Helmholtz instances in one call: blocks[i] with weights
    ws[i] (None: 4 pi / n_i).  Returns the list of matrices."""
    count = len(blocks)
    hb = (C.c_void_p * max(1, count))(*[b.h for b in blocks])
    arrs = [None if w is None else np.ascontiguousarray(w, dtype=np.float64) for w in ws]
    wp = (C.POINTER(C.c_double) * max(1, count))(
        *[C.POINTER(C.c_double)() if a is None else a.ctypes.data_as(C.POINTER(C.c_double))
          for a in arrs])
    outs = (C.c_void_p * max(1, count))()
    _check(lib().dh2_compress_batch(count, hb, wp, float(eps), C.byref(o), _stream(stream), outs))
    return [Matrix(C.c_void_p(outs[i]), keep=blocks[i]) for i in range(count)]


def compress_dense(b: Blocks, G, eps: float, o: Opts, stream=None) -> Matrix:
    """G: torch complex128 tensor (n x n, row-major) on the GPU, original order."""
    assert G.dtype.is_complex and G.element_size() == 16 and G.is_cuda
    assert G.stride(1) == 1
    h = C.c_void_p()
    _check(lib().dh2_compress_dense(b.h, C.c_void_p(G.data_ptr()), G.stride(0), float(eps),
                                    C.byref(o), _stream(stream), C.byref(h)))
    return Matrix(h, keep=b)


def matvec(m: Matrix, op: str, x, y, stream=None):
    """y = G~ x (op 'N') or G~^* x (op 'C'); x, y: torch complex128 (n,) or (n, nrhs)
    column-major, i.e. contiguous (nrhs, n) transposed."""
    n = x.shape[0]
    nrhs = 1 if x.dim() == 1 else x.shape[1]
    if x.dim() == 2:
        assert x.stride(0) == 1 and y.stride(0) == 1
    _check(lib().dh2_matvec(m.h, op.encode(), nrhs, C.c_void_p(x.data_ptr()),
                            C.c_void_p(y.data_ptr()), _stream(stream)))
    return y


def matvec_noalloc(m: Matrix, op: str, x, y, stream=None):
    """dh2_matvec_noalloc: as matvec, with the library's static scratch array
    (no device allocation); only enqueued on the stream."""
    n = x.shape[0]
    nrhs = 1 if x.dim() == 1 else x.shape[1]
    if x.dim() == 2:
        assert x.stride(0) == 1 and y.stride(0) == 1
    _check(lib().dh2_matvec_noalloc(m.h, op.encode(), nrhs, C.c_void_p(x.data_ptr()),
                                    C.c_void_p(y.data_ptr()), _stream(stream)))
    return y


def error_estimate(m: Matrix, G=None, iters: int = 50, seed: int = 1, stream=None) -> float:
    err = C.c_double()
    gp = C.c_void_p(G.data_ptr()) if G is not None else None
    ld = G.stride(0) if G is not None else 0
    _check(lib().dh2_error_estimate(m.h, gp, ld, iters, seed, C.byref(err), _stream(stream)))
    return err.value


def rows_check(m: Matrix, rows, x, stream=None):
    r = np.ascontiguousarray(rows, dtype=np.int64)
    direct = np.empty(2 * len(r))
    approx = np.empty(2 * len(r))
    mr = C.c_double()
    _check(lib().dh2_rows_check(m.h, _p(r, C.c_int64), len(r), C.c_void_p(x.data_ptr()),
                                _p(direct, C.c_double), _p(approx, C.c_double), C.byref(mr),
                                _stream(stream)))
    return (direct.view(np.complex128), approx.view(np.complex128), mr.value)


def stats(m: Matrix) -> dict:
    s = Stats()
    _check(lib().dh2_get_stats(m.h, C.byref(s)))
    out = {}
    for f, _ in Stats._fields_:
        v = getattr(s, f)
        out[f] = list(v) if hasattr(v, "__len__") else v
    return out


def basis_export(m: Matrix, side: int) -> dict:
    ni, ns, nm = C.c_int32(), C.c_int64(), C.c_int64()
    L = lib()
    _check(L.dh2_basis_export(m.h, side, C.byref(ni), C.byref(ns), C.byref(nm), None, None, None,
                              None, None, None, None, None))
    n_i, n_s, n_m = ni.value, ns.value, nm.value
    out = dict(item_t=np.empty(n_i, np.int32), item_c=np.empty(n_i, np.int32),
               item_k=np.empty(n_i, np.int32), item_r=np.empty(n_i, np.int32),
               sig_off=np.empty(n_i, np.int64), sigma=np.empty(max(1, n_s)),
               mat_off=np.empty(n_i, np.int64), mat=np.empty(max(1, 2 * n_m)))
    I32, I64, D = C.c_int32, C.c_int64, C.c_double
    _check(L.dh2_basis_export(m.h, side, C.byref(ni), C.byref(ns), C.byref(nm),
                              _p(out["item_t"], I32), _p(out["item_c"], I32),
                              _p(out["item_k"], I32), _p(out["item_r"], I32),
                              _p(out["sig_off"], I64), _p(out["sigma"], D),
                              _p(out["mat_off"], I64), _p(out["mat"], D)))
    out["mat"] = out["mat"][:2 * n_m].view(np.complex128)
    out["sigma"] = out["sigma"][:n_s]
    return out


def coupling_export(m: Matrix, nadm: int):
    off = np.empty(nadm + 1, np.int64)
    _check(lib().dh2_coupling_export(m.h, _p(off, C.c_int64), None))
    S = np.empty(max(1, 2 * int(off[-1])))
    _check(lib().dh2_coupling_export(m.h, _p(off, C.c_int64), _p(S, C.c_double)))
    return off, S[:2 * int(off[-1])].view(np.complex128)


def near_export(m: Matrix, nnear: int):
    off = np.empty(nnear + 1, np.int64)
    _check(lib().dh2_near_export(m.h, _p(off, C.c_int64), None))
    N = np.empty(max(1, 2 * int(off[-1])))
    _check(lib().dh2_near_export(m.h, _p(off, C.c_int64), _p(N, C.c_double)))
    return off, N[:2 * int(off[-1])].view(np.complex128)


def release_cached_memory():
    """Return the library's cached device memory to the driver."""
    lib().dh2_release_cached_memory()
