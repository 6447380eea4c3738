"""The library's host plan (C++) equals the oracle's plan exactly.

Cluster tree (permutation, ranges, levels, sons, boxes), directions and son
maps, block lists with block directions, and the column sets of both bases
are compared element by element; floating-point values bit for bit.  These
run on the CPU (no GPU needed): only the plan entry points are called.
"""
import math

import numpy as np
import pytest

import synth
from oracle import plan as P

dh2 = pytest.importorskip("paper_1510_07087_amd.dh2")


def _lib_available():
    try:
        dh2.lib()
        return True
    except Exception:
        return False


pytestmark = pytest.mark.skipif(not _lib_available(), reason="libdh2.so not built")

def _sphere_with_outlier(n=2048):
    """The sphere plus one far point: bisection puts it in a one-point leaf."""
    p, w = synth.fibonacci_sphere(n)
    return np.vstack([p, [[5.0, 0.0, 0.0]]]), np.append(w, w[0])


CASES = [
    ("sphere2048", lambda: synth.fibonacci_sphere(2048), 8.0, 32, {}),
    ("sphere8192_k16", lambda: synth.fibonacci_sphere(8192), 16.0, 64, {}),
    ("ellipsoid4096", lambda: synth.ellipsoid(4096), 12.0, 64, {}),
    ("cube3000", lambda: synth.cube_surface(3000, 9), 9.0, 40, {}),
    ("kappa0", lambda: synth.fibonacci_sphere(1500), 0.0, 32, {}),
    ("lowfreq", lambda: synth.fibonacci_sphere(4096), 11.0, 32, dict(lowfreq_zero=True)),
    ("standard", lambda: synth.fibonacci_sphere(4096), 11.0, 32, dict(standard_only=True)),
    ("eta2_1", lambda: synth.fibonacci_sphere(4096), 11.0, 32, dict(eta2=1.0)),
    ("outlier", _sphere_with_outlier, 8.0, 32, {}),
]


@pytest.mark.parametrize("name,gen,kappa,leaf,kw", CASES, ids=[c[0] for c in CASES])
def test_plan_equals_oracle(name, gen, kappa, leaf, kw):
    pts, w = gen()
    eta2 = kw.get("eta2", 5.0)
    ref = P.build_plan(pts, kappa, leaf, 20.0, eta2, lowfreq_zero=kw.get("lowfreq_zero", False),
                       standard_only=kw.get("standard_only", False))
    o = dh2.opts(leaf_size=leaf, eta1=20.0, eta2=eta2,
                 lowfreq_zero_dir=int(kw.get("lowfreq_zero", False)),
                 standard_only=int(kw.get("standard_only", False)))
    t = dh2.tree_build(pts, kappa, o)
    te = dh2.tree_export(t)
    tr = ref.tree
    assert np.array_equal(te["perm"], tr.perm)
    assert np.array_equal(te["off"], tr.off)
    assert np.array_equal(te["size"], tr.size)
    assert np.array_equal(te["level"], tr.level)
    assert np.array_equal(te["son1"], tr.son1)
    assert np.array_equal(te["son2"], tr.son2)
    # floating point bit for bit
    assert np.array_equal(te["lo"].view(np.uint64), tr.lo.view(np.uint64))
    assert np.array_equal(te["hi"].view(np.uint64), tr.hi.view(np.uint64))
    assert np.array_equal(te["diam"].view(np.uint64), tr.diam.view(np.uint64))
    assert np.array_equal(te["delta"].view(np.uint64), tr.delta.view(np.uint64))
    for lv in range(tr.depth + 1):
        dirs, sd = dh2.tree_directions(t, lv)
        assert np.array_equal(dirs.view(np.uint64), ref.dirs.dirs[lv].view(np.uint64))
        if lv < tr.depth:
            assert np.array_equal(sd, ref.dirs.sd[lv])
        else:
            assert np.all(sd == -1)
    b = dh2.blocks_build(t, o)
    be = dh2.blocks_export(b)
    assert np.array_equal(be["adm_t"], ref.blocks.adm_t)
    assert np.array_equal(be["adm_s"], ref.blocks.adm_s)
    assert np.array_equal(be["adm_c"], ref.blocks.adm_c)
    assert np.array_equal(be["near_t"], ref.blocks.near_t)
    assert np.array_equal(be["near_s"], ref.blocks.near_s)
    for side, sets in ((0, ref.rowsets), (1, ref.colsets)):
        cs = dh2.blocks_colsets(b, side)
        items = [(t_, c) for t_ in range(tr.nc) for c in sets.used(t_)]
        assert len(items) == len(cs["item_t"])
        assert [tuple(x) for x in zip(cs["item_t"], cs["item_c"])] == items
        for i, (t_, c) in enumerate(items):
            lo_, hi_ = cs["item_begin"][i], cs["item_begin"][i + 1]
            got = list(zip(cs["ent_b"][lo_:hi_], cs["ent_s"][lo_:hi_], cs["ent_d"][lo_:hi_]))
            assert got == [tuple(e) for e in sets.F[t_][c]]


def test_eta2_reading_statistics():
    """Evidence for the reading of the admissibility parameter: with eta2 = 1
    the 2048-point workload keeps almost the whole matrix as near field, with
    the paper's eta2 = 5 about a third of it."""
    pts, w = synth.fibonacci_sphere(2048)
    o1 = dh2.opts(leaf_size=32, eta2=1.0)
    o5 = dh2.opts(leaf_size=32, eta2=5.0)
    t = dh2.tree_build(pts, 8.0, o1)
    i1 = dh2.blocks_info(dh2.blocks_build(t, o1))
    i5 = dh2.blocks_info(dh2.blocks_build(t, o5))
    assert i1["near_entries"] / 2048 ** 2 > 0.9
    assert i5["near_entries"] / 2048 ** 2 < 0.4
    assert i5["nadm"] > 1000


def test_invalid_arguments():
    """Argument checks return DH2_EINVAL without touching the output."""
    pts, w = synth.fibonacci_sphere(64)
    o = dh2.opts()
    with pytest.raises(dh2.DH2Error) as e:
        dh2.tree_build(pts, -1.0, o)
    assert e.value.code == -1
    bad = pts.copy()
    bad[3, 1] = math.nan
    with pytest.raises(dh2.DH2Error) as e:
        dh2.tree_build(bad, 1.0, o)
    assert e.value.code == -1
    with pytest.raises(dh2.DH2Error) as e:
        dh2.tree_build(pts, 1.0, dh2.opts(leaf_size=0))
    assert e.value.code == -1
    with pytest.raises(dh2.DH2Error) as e:
        dh2.tree_build(pts, 1.0, dh2.opts(zeta=0.8))
    assert e.value.code == -1
    with pytest.raises(dh2.DH2Error) as e:
        dh2.tree_build(pts[:0], 1.0, o)
    assert e.value.code == -1
    dup = np.vstack([pts, pts[17:18]])
    with pytest.raises(dh2.DH2Error) as e:
        dh2.tree_build(dup, 1.0, o)
    assert e.value.code == -1 and "coincident" in str(e.value)


@pytest.mark.parametrize("side", [0, 1])
def test_inherited_columns_form_a_prefix(side):
    """The father's sets F_tc, taken in the father's direction order, are the
    leading columns of the son's set for sd(c), and the son's own blocks come
    last (the R recursion of the paper's transfer step reads only inherited
    columns, so the column sweep forms R over that prefix alone)."""
    pts, _ = synth.fibonacci_sphere(8192)
    o = dh2.opts(leaf_size=64)
    t = dh2.tree_build(pts, 16.0, o)
    te = dh2.tree_export(t)
    b = dh2.blocks_build(t, o)
    cs = dh2.blocks_colsets(b, side)
    beg = cs["item_begin"]
    ent = list(zip(cs["ent_b"], cs["ent_s"], cs["ent_d"]))
    item = {(int(t_), int(c)): i for i, (t_, c) in enumerate(zip(cs["item_t"], cs["item_c"]))}
    father = {}
    for f, (s1, s2) in enumerate(zip(te["son1"], te["son2"])):
        if s1 >= 0:
            father[int(s1)] = f
            father[int(s2)] = f
    checked = 0
    for (t_, c), i in item.items():
        es = ent[beg[i]:beg[i + 1]]
        d = [e[2] for e in es]
        nown = sum(1 for x in d if x == 0)
        assert all(x > 0 for x in d[:len(d) - nown]) and all(x == 0 for x in d[len(d) - nown:])
        if t_ not in father:
            continue
        f = father[t_]
        _, sd = dh2.tree_directions(t, int(te["level"][f]))
        expect = []
        for cf in sorted(c2 for (t2, c2) in item if t2 == f):
            if sd[cf] == c:
                j = item[(f, cf)]
                expect += [(e[0], e[1], e[2] + 1) for e in ent[beg[j]:beg[j + 1]]]
        assert es[:len(es) - nown] == expect
        checked += 1
    assert checked > 0


def test_admissible_blocks_are_separated():
    """A one-point cluster meets (b) and (c) with itself (diam = dist = 0); its
    block holds the singular diagonal entry and must stay in the near field:
    every admissible block has boxes at positive distance, also with a
    one-point leaf, and a single point is one near-field block."""
    pts, _ = _sphere_with_outlier()
    o = dh2.opts(leaf_size=32)
    t = dh2.tree_build(pts, 8.0, o)
    te = dh2.tree_export(t)
    assert 1 in set(int(x) for x in te["size"])
    b = dh2.blocks_build(t, o)
    be = dh2.blocks_export(b)
    lo, hi = te["lo"].reshape(-1, 3), te["hi"].reshape(-1, 3)
    for t_, s_ in zip(be["adm_t"], be["adm_s"]):
        gap = np.maximum(0.0, np.maximum(lo[s_] - hi[t_], lo[t_] - hi[s_]))
        assert np.sqrt(np.sum(gap ** 2)) > 0.0
    one = dh2.blocks_info(dh2.blocks_build(dh2.tree_build(pts[:1], 8.0, o), o))
    assert one["nadm"] == 0 and one["nnear"] == 1
