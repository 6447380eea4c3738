"""Pins for the oracle's cluster tree, directions and block tree.

Each test checks the oracle against what the paper's definitions fix, by an
independent route (brute force, closed forms, the lemma's inequality).
"""
import math

import numpy as np
import pytest

import synth
from oracle import plan as P


def small_sphere(n=384, kappa=6.0, leaf=16):
    p, w = synth.fibonacci_sphere(n)
    return p, P.build_plan(p, kappa, leaf, eta1=20.0, eta2=5.0)


def test_cluster_tree_partition():
    """Definition 'Cluster tree': sons partition the father; contiguous ranges."""
    p, pl = small_sphere()
    tr = pl.tree
    assert tr.off[0] == 0 and tr.size[0] == tr.n
    assert sorted(tr.perm.tolist()) == list(range(tr.n))
    for t in range(tr.nc):
        if tr.son1[t] >= 0:
            a, b = tr.son1[t], tr.son2[t]
            assert tr.off[a] == tr.off[t]
            assert tr.off[b] == tr.off[a] + tr.size[a]
            assert tr.size[a] + tr.size[b] == tr.size[t]
            assert tr.size[a] > 0 and tr.size[b] > 0
            assert tr.level[a] == tr.level[t] + 1 == tr.level[b]
        else:
            assert tr.size[t] <= 16
    # every point lies in the tight box of each cluster containing it
    pts = p[tr.perm]
    for t in range(tr.nc):
        q = pts[tr.off[t]:tr.off[t] + tr.size[t]]
        assert np.array_equal(q.min(axis=0), tr.lo[t])
        assert np.array_equal(q.max(axis=0), tr.hi[t])


def test_cluster_split_rule():
    """Split at the midpoint of the longest box edge (reading of 'regular subdivision')."""
    p, pl = small_sphere()
    tr = pl.tree
    pts = p[tr.perm]
    for t in range(tr.nc):
        if tr.son1[t] < 0:
            continue
        ext = tr.hi[t] - tr.lo[t]
        ax = int(np.argmax(ext))  # numpy returns the first maximum
        mid = 0.5 * (tr.lo[t][ax] + tr.hi[t][ax])
        a, b = tr.son1[t], tr.son2[t]
        assert np.all(pts[tr.off[a]:tr.off[a] + tr.size[a], ax] < mid)
        assert np.all(pts[tr.off[b]:tr.off[b] + tr.size[b], ax] >= mid)


def test_block_leaves_partition_index_square():
    """Definition 'Block tree': the leaves cover I x I exactly once (brute force)."""
    p, pl = small_sphere()
    tr, bt = pl.tree, pl.blocks
    cover = np.zeros((tr.n, tr.n), dtype=np.int32)
    for t, s in list(zip(bt.adm_t, bt.adm_s)) + list(zip(bt.near_t, bt.near_s)):
        cover[tr.off[t]:tr.off[t] + tr.size[t], tr.off[s]:tr.off[s] + tr.size[s]] += 1
        assert tr.level[t] == tr.level[s]
    assert np.all(cover == 1)
    assert len(bt.adm_t) > 0


def test_admissibility_and_minimal_tree():
    """Every admissible leaf satisfies (b) and (c); every inadmissible leaf has
    a leaf cluster; every split block violates them (minimal block tree)."""
    p, pl = small_sphere()
    tr, bt = pl.tree, pl.blocks
    kappa, eta2 = pl.kappa, pl.eta2
    pts = p[tr.perm]

    def point_dist(t, s):
        a = pts[tr.off[t]:tr.off[t] + tr.size[t]]
        b = pts[tr.off[s]:tr.off[s] + tr.size[s]]
        return np.min(np.linalg.norm(a[:, None, :] - b[None, :, :], axis=2))

    for t, s in zip(bt.adm_t, bt.adm_s):
        d = P.box_dist(tr.lo[t], tr.hi[t], tr.lo[s], tr.hi[s])
        dm = max(tr.diam[t], tr.diam[s])
        assert kappa * dm * dm <= eta2 * d * (1 + 1e-15)
        assert dm <= eta2 * d
        # the box distance is a lower bound for the point distance
        assert d <= point_dist(t, s) + 1e-14
    for t, s in zip(bt.near_t, bt.near_s):
        assert tr.son1[t] < 0 or tr.son1[s] < 0
        assert not P.admissible(tr, t, s, kappa, eta2)
    # walk the block tree again and collect inner blocks
    inner = []
    stack = [(0, 0)]
    while stack:
        t, s = stack.pop()
        if P.admissible(tr, t, s, kappa, eta2):
            continue
        if tr.son1[t] >= 0 and tr.son1[s] >= 0:
            inner.append((t, s))
            stack += [(a, b) for a in tr.sons(t) for b in tr.sons(s)]
    for t, s in inner:
        assert not P.admissible(tr, t, s, kappa, eta2)


def test_directions_cover_sphere():
    """Covering condition of Section 3: min_c |z-c| <= eta1/(kappa delta_l)."""
    rng = np.random.default_rng(0)
    z = rng.standard_normal((100000, 3))
    z /= np.linalg.norm(z, axis=1)[:, None]
    for kappa, delta, eta1 in [(64.0, 0.42, 20.0), (32.0, 1.1, 20.0), (8.0, 3.4, 20.0),
                               (100.0, 0.9, 5.0)]:
        m = P.directions_per_edge(kappa, delta, eta1)
        D = P.cube_directions(m)
        assert D.shape == (6 * m * m, 3)
        assert np.allclose(np.linalg.norm(D, axis=1), 1.0)
        dmin = np.sqrt(((z[:, None, :] - D[None, :, :]) ** 2).sum(-1)).min(axis=1)
        assert dmin.max() <= eta1 / (kappa * delta)
        # squares have diameter <= 2 eta1 / (kappa delta)
        assert 2.0 * math.sqrt(2.0) / m <= 2.0 * eta1 / (kappa * delta) + 1e-15


def test_projection_lemma():
    """Lemma 'Projection': |x/|x| - y/|y|| <= |x-y| for |x|,|y| >= 1."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal((20000, 3))
    y = rng.standard_normal((20000, 3))
    x *= (1.0 + rng.random(20000) * 3)[:, None] / np.linalg.norm(x, axis=1)[:, None]
    y *= (1.0 + rng.random(20000) * 3)[:, None] / np.linalg.norm(y, axis=1)[:, None]
    lhs = np.linalg.norm(x / np.linalg.norm(x, axis=1)[:, None]
                         - y / np.linalg.norm(y, axis=1)[:, None], axis=1)
    assert np.all(lhs <= np.linalg.norm(x - y, axis=1) + 1e-15)


def test_son_maps_nearest():
    """Definition 'Hierarchical directions': sd maps to a nearest direction."""
    p, w = synth.fibonacci_sphere(8192)
    pl = P.build_plan(p, 16.0, 32)
    dr = pl.dirs
    for lv, sd in enumerate(dr.sd):
        A, B = dr.dirs[lv], dr.dirs[lv + 1]
        d = np.linalg.norm(A[:, None, :] - B[None, :, :], axis=2)
        chosen = d[np.arange(len(A)), sd]
        assert np.allclose(chosen, d.min(axis=1), rtol=0, atol=1e-15)


def test_block_direction_nearest():
    """Block direction c_b: nearest to (m_t-m_s)/|m_t-m_s| (condition (a))."""
    p, pl = small_sphere(1024, 10.0, 16)
    tr, bt, dr = pl.tree, pl.blocks, pl.dirs
    for t, s, c in zip(bt.adm_t, bt.adm_s, bt.adm_c):
        mt = 0.5 * (tr.lo[t] + tr.hi[t])
        ms = 0.5 * (tr.lo[s] + tr.hi[s])
        z = (mt - ms) / np.linalg.norm(mt - ms)
        D = dr.dirs[tr.level[t]]
        d = np.linalg.norm(D - z, axis=1)
        assert abs(d[c] - d.min()) <= 1e-15
        # condition (a) then holds with the per-level covering bound
        dm = max(tr.diam[t], tr.diam[s])
        assert pl.kappa * d[c] <= pl.eta1 / dm * (1 + 1e-12)


def test_kappa_zero_single_direction():
    """kappa=0: a single zero direction per level; the block tree is the
    standard-admissibility tree (condition (b) always holds)."""
    p, w = synth.fibonacci_sphere(1024)
    pl0 = P.build_plan(p, 0.0, 16)
    assert all(len(d) == 1 and np.all(d == 0) for d in pl0.dirs.dirs)
    pls = P.build_plan(p, 0.0, 16, standard_only=True)
    assert np.array_equal(pl0.blocks.adm_t, pls.blocks.adm_t)
    assert np.array_equal(pl0.blocks.adm_s, pls.blocks.adm_s)


def test_column_sets_definition():
    """F_tc (Section 6) recomputed straight from its definition: s in F_tc iff
    some ancestor-or-self t+ has an admissible block (t+,s) whose direction,
    pushed down by the son maps, equals c."""
    p, pl = small_sphere(1024, 10.0, 16)
    tr, bt, dr = pl.tree, pl.blocks, pl.dirs
    ref = [dict() for _ in range(tr.nc)]
    for b in range(len(bt.adm_t)):
        tp, s, c = int(bt.adm_t[b]), int(bt.adm_s[b]), int(bt.adm_c[b])
        # all descendants of tp with the pushed direction
        stack = [(tp, c, 0)]
        while stack:
            t, cc, d = stack.pop()
            ref[t].setdefault(cc, set()).add((b, s, d))
            for ts in tr.sons(t):
                stack.append((ts, int(dr.sd[tr.level[t]][cc]), d + 1))
    for t in range(tr.nc):
        got = {c: set(v) for c, v in pl.rowsets.F[t].items()}
        assert got == ref[t]
        # directions partition the columns: sets for different c are disjoint
        seen = set()
        for c, v in pl.rowsets.F[t].items():
            cols = set(int(s) for (_, s, _) in v)
            assert not (cols & seen)
            seen |= cols


@pytest.mark.parametrize("n,kappa,leaf", [(2048, 8.0, 32), (1500, 0.0, 20)])
def test_block_tree_symmetric(n, kappa, leaf):
    """Admissibility is symmetric, so (t,s) in L+ iff (s,t) in L+, and the
    block directions are opposite (the cube directions satisfy D = -D)."""
    p, w = synth.fibonacci_sphere(n)
    pl = P.build_plan(p, kappa, leaf)
    bt, dr, tr = pl.blocks, pl.dirs, pl.tree
    idx = {(int(t), int(s)): b for b, (t, s) in enumerate(zip(bt.adm_t, bt.adm_s))}
    for (t, s), b in idx.items():
        assert (s, t) in idx
        D = dr.dirs[tr.level[t]]
        c1, c2 = bt.adm_c[b], bt.adm_c[idx[(s, t)]]
        assert np.allclose(D[c1], -D[c2])
