"""Oracle: cluster tree, hierarchical directions, block tree and column sets.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings of the paper fixed here (the paper leaves them open):

* Cluster tree (Definition "Cluster tree"; Section 7 uses geometrically
  regular subdivision): the tight axis-parallel box of a cluster's points is
  split on its longest edge (ties to the lowest axis) at the midpoint
  0.5*(lo+hi); points with coordinate < mid go to the first son, the rest to the
  second, keeping their order.  Recursion stops at <= leaf_size points or when
  the box has no extent.  Clusters are numbered in depth-first pre-order and
  occupy contiguous ranges of the permuted index order.
* diam(B) is the Euclidean box diagonal, dist(B_t,B_s) the Euclidean gap
  between the boxes (0 if they touch), m_t the box midpoint.
* Directions (Section 3, construction after the covering condition): on each
  level, m = ceil(sqrt(2)*kappa*delta_l/eta1) squares per cube-face edge, face
  order +x,-x,+y,-y,+z,-z, square midpoints (-1+(2i+1)/m, -1+(2j+1)/m),
  normalised.  kappa*delta_l == 0 gives the single direction 0.
* Son maps (Definition "Hierarchical directions"): the nearest direction on
  the next level, ties to the smallest index.
* Block tree (Section 3, conditions (b) parabolic and (c) standard decide
  admissibility; the minimal block tree): admissible -> leaf with block
  direction c_b = nearest direction to (m_t-m_s)/|m_t-m_s|; otherwise split if
  both clusters have sons, else an inadmissible leaf.
* Column sets F_tc (Section 6): inherited from the father through the son map
  first (father directions in increasing order), then the cluster's own
  admissible blocks in block order.

All floating-point predicates are evaluated with the exact expression order
written below, so that an independent implementation can reproduce the
integer results bit for bit.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------
# cluster tree (Definition "Cluster tree", levels and depth)
# --------------------------------------------------------------------------
@dataclass
class ClusterTree:
    n: int
    perm: np.ndarray          # perm[pos] = original index of the point at pos
    off: np.ndarray           # first position of each cluster
    size: np.ndarray          # number of indices
    level: np.ndarray
    father: np.ndarray        # -1 for the root
    son1: np.ndarray          # -1 for leaves
    son2: np.ndarray
    lo: np.ndarray            # (nc,3) tight box
    hi: np.ndarray
    diam: np.ndarray
    depth: int
    delta: np.ndarray         # per level: max diam on that level

    @property
    def nc(self) -> int:
        return len(self.off)

    def is_leaf(self, t: int) -> bool:
        return self.son1[t] < 0

    def sons(self, t: int):
        return () if self.son1[t] < 0 else (int(self.son1[t]), int(self.son2[t]))

    def rows(self, t: int) -> np.ndarray:
        """Positions (permuted order) of the indices of cluster t."""
        return np.arange(self.off[t], self.off[t] + self.size[t])


def box_diam(lo, hi) -> float:
    e0 = hi[0] - lo[0]
    e1 = hi[1] - lo[1]
    e2 = hi[2] - lo[2]
    return math.sqrt(e0 * e0 + e1 * e1 + e2 * e2)


def build_cluster_tree(points: np.ndarray, leaf_size: int) -> ClusterTree:
    pts = np.asarray(points, dtype=np.float64)
    n = pts.shape[0]
    perm = np.arange(n, dtype=np.int64)
    off, size, level, father, son1, son2, lo, hi = [], [], [], [], [], [], [], []

    # explicit stack emulating the depth-first pre-order recursion
    stack = [(0, n, 0, -1, None)]  # (off, size, level, father, slot in father)
    while stack:
        o, sz, lv, fa, slot = stack.pop()
        idx = perm[o:o + sz]
        p = pts[idx]
        blo = p.min(axis=0)
        bhi = p.max(axis=0)
        cid = len(off)
        off.append(o); size.append(sz); level.append(lv); father.append(fa)
        son1.append(-1); son2.append(-1)
        lo.append(blo); hi.append(bhi)
        if fa >= 0:
            if slot == 0:
                son1[fa] = cid
            else:
                son2[fa] = cid
        if sz <= leaf_size:
            continue
        ext = bhi - blo
        axis = 0
        for a in (1, 2):
            if ext[a] > ext[axis]:
                axis = a
        if not ext[axis] > 0.0:
            continue
        mid = 0.5 * (blo[axis] + bhi[axis])
        sel = p[:, axis] < mid
        left = idx[sel]
        right = idx[~sel]
        perm[o:o + sz] = np.concatenate([left, right])
        nl = len(left)
        # push the second son first so the first son is numbered next
        stack.append((o + nl, sz - nl, lv + 1, cid, 1))
        stack.append((o, nl, lv + 1, cid, 0))

    lo = np.array(lo); hi = np.array(hi)
    diam = np.array([box_diam(lo[t], hi[t]) for t in range(len(off))])
    level = np.array(level, dtype=np.int64)
    depth = int(level.max())
    delta = np.zeros(depth + 1)
    for t in range(len(off)):
        if diam[t] > delta[level[t]]:
            delta[level[t]] = diam[t]
    return ClusterTree(
        n=n, perm=perm,
        off=np.array(off, dtype=np.int64), size=np.array(size, dtype=np.int64),
        level=level, father=np.array(father, dtype=np.int64),
        son1=np.array(son1, dtype=np.int64), son2=np.array(son2, dtype=np.int64),
        lo=lo, hi=hi, diam=diam, depth=depth, delta=delta,
    )


# --------------------------------------------------------------------------
# hierarchical directions and son maps (Definition "Hierarchical directions",
# Section 3 cube construction and Lemma "Projection")
# --------------------------------------------------------------------------
def directions_per_edge(kappa: float, delta: float, eta1: float) -> int:
    x = math.sqrt(2.0) * kappa * delta / eta1
    return int(math.ceil(x))


def cube_directions(m: int) -> np.ndarray:
    """Normalised midpoints of an m x m grid of squares on each cube face."""
    if m == 0:
        return np.zeros((1, 3))
    out = []
    for face in range(6):
        axis, sign = face // 2, (1.0 if face % 2 == 0 else -1.0)
        for i in range(m):
            u = -1.0 + (2.0 * i + 1.0) / m
            for j in range(m):
                v = -1.0 + (2.0 * j + 1.0) / m
                if axis == 0:
                    x, y, z = sign, u, v
                elif axis == 1:
                    x, y, z = u, sign, v
                else:
                    x, y, z = u, v, sign
                nrm = math.sqrt(x * x + y * y + z * z)
                out.append((x / nrm, y / nrm, z / nrm))
    return np.array(out)


def nearest_direction(dirs: np.ndarray, z) -> int:
    """Index of the direction closest to z in the Euclidean norm; first wins."""
    best, bd = 0, math.inf
    for i in range(dirs.shape[0]):
        dx = z[0] - dirs[i, 0]
        dy = z[1] - dirs[i, 1]
        dz = z[2] - dirs[i, 2]
        d2 = dx * dx + dy * dy + dz * dz
        if d2 < bd:
            bd, best = d2, i
    return best


@dataclass
class Directions:
    per_edge: list            # m_l per level
    dirs: list                # list of (n_l,3) arrays
    sd: list                  # sd[l][c] -> index on level l+1 (len depth)


def build_directions(tree: ClusterTree, kappa: float, eta1: float,
                     lowfreq_zero: bool = False) -> Directions:
    per_edge, dirs = [], []
    for lv in range(tree.depth + 1):
        kd = kappa * tree.delta[lv]
        if kd == 0.0 or (lowfreq_zero and kd <= eta1):
            m = 0
        else:
            m = directions_per_edge(kappa, tree.delta[lv], eta1)
        per_edge.append(m)
        dirs.append(cube_directions(m))
    sd = []
    for lv in range(tree.depth):
        nxt = dirs[lv + 1]
        sd.append(np.array([nearest_direction(nxt, c) for c in dirs[lv]],
                           dtype=np.int64))
    return Directions(per_edge=per_edge, dirs=dirs, sd=sd)


# --------------------------------------------------------------------------
# block tree (Definition "Block tree", admissibility conditions (b), (c))
# --------------------------------------------------------------------------
def box_dist(lo_t, hi_t, lo_s, hi_s) -> float:
    d2 = 0.0
    for a in range(3):
        g = max(0.0, max(lo_s[a] - hi_t[a], lo_t[a] - hi_s[a]))
        d2 = d2 + g * g
    return math.sqrt(d2)


def admissible(tree: ClusterTree, t: int, s: int, kappa: float, eta2: float,
               standard_only: bool = False) -> bool:
    dmax = max(tree.diam[t], tree.diam[s])
    dist = box_dist(tree.lo[t], tree.hi[t], tree.lo[s], tree.hi[s])
    # the far field needs separated boxes: (b) and (c) hold trivially for a
    # one-point cluster with itself (diam = dist = 0), whose block holds the
    # singular diagonal entry
    if not dist > 0.0:
        return False
    cond_c = dmax <= eta2 * dist
    if standard_only:
        return cond_c
    cond_b = kappa * (dmax * dmax) <= eta2 * dist
    return cond_b and cond_c


def block_direction(tree: ClusterTree, dirs: np.ndarray, t: int, s: int) -> int:
    mt = [0.5 * (tree.lo[t][a] + tree.hi[t][a]) for a in range(3)]
    ms = [0.5 * (tree.lo[s][a] + tree.hi[s][a]) for a in range(3)]
    u = [mt[a] - ms[a] for a in range(3)]
    nrm = math.sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2])
    z = [u[a] / nrm for a in range(3)]
    return nearest_direction(dirs, z)


@dataclass
class BlockTree:
    adm_t: np.ndarray
    adm_s: np.ndarray
    adm_c: np.ndarray
    near_t: np.ndarray
    near_s: np.ndarray


def build_block_tree(tree: ClusterTree, dr: Directions, kappa: float, eta2: float,
                     standard_only: bool = False) -> BlockTree:
    at, as_, ac, nt, ns = [], [], [], [], []
    stack = [(0, 0)]
    while stack:
        t, s = stack.pop()
        if admissible(tree, t, s, kappa, eta2, standard_only):
            at.append(t); as_.append(s)
            ac.append(block_direction(tree, dr.dirs[tree.level[t]], t, s))
        elif tree.son1[t] >= 0 and tree.son1[s] >= 0:
            pairs = [(a, b) for a in tree.sons(t) for b in tree.sons(s)]
            for p in reversed(pairs):
                stack.append(p)
        else:
            nt.append(t); ns.append(s)
    i64 = lambda v: np.array(v, dtype=np.int64)
    return BlockTree(i64(at), i64(as_), i64(ac), i64(nt), i64(ns))


# --------------------------------------------------------------------------
# column sets F_tc (Section 6: desc, dscd, F_tc and the union of their sets)
# --------------------------------------------------------------------------
@dataclass
class ColumnSets:
    """F[t] maps a direction index c on level(t) to a list of entries
    (b, s, d): admissible block b=(t+,s) of an ancestor-or-self t+ of t, whose
    direction chain passes through c, with d = level(t) - level(t+)."""

    F: list = field(default_factory=list)

    def used(self, t: int):
        return sorted(self.F[t].keys())


def build_column_sets(tree: ClusterTree, dr: Directions, own_blocks,
                      block_dir: np.ndarray, partner: np.ndarray) -> ColumnSets:
    """own_blocks[t]: block ids whose 'row' cluster (for this basis) is t, in
    block order; partner[b]: the other cluster of block b."""
    F = [dict() for _ in range(tree.nc)]
    for t in range(tree.nc):  # pre-order: fathers come before sons
        fa = tree.father[t]
        if fa >= 0:
            sdf = dr.sd[tree.level[fa]]
            for cp in sorted(F[fa].keys()):
                c = int(sdf[cp])
                F[t].setdefault(c, []).extend((b, s, d + 1) for (b, s, d) in F[fa][cp])
        for b in own_blocks[t]:
            F[t].setdefault(int(block_dir[b]), []).append((int(b), int(partner[b]), 0))
    return ColumnSets(F=F)


@dataclass
class Plan:
    tree: ClusterTree
    dirs: Directions
    blocks: BlockTree
    rowsets: ColumnSets       # for the row basis (blocks (t,s) -> row cluster t)
    colsets: ColumnSets       # for the column basis (G^*: blocks (s,t))
    kappa: float
    eta1: float
    eta2: float


def build_plan(points: np.ndarray, kappa: float, leaf_size: int, eta1: float = 20.0,
               eta2: float = 5.0, lowfreq_zero: bool = False,
               standard_only: bool = False) -> Plan:
    tree = build_cluster_tree(points, leaf_size)
    dr = build_directions(tree, kappa, eta1, lowfreq_zero)
    bt = build_block_tree(tree, dr, kappa, eta2, standard_only)
    own_row = [[] for _ in range(tree.nc)]
    own_col = [[] for _ in range(tree.nc)]
    for b in range(len(bt.adm_t)):
        own_row[bt.adm_t[b]].append(b)
        own_col[bt.adm_s[b]].append(b)
    rows = build_column_sets(tree, dr, own_row, bt.adm_c, bt.adm_s)
    cols = build_column_sets(tree, dr, own_col, bt.adm_c, bt.adm_t)
    return Plan(tree, dr, bt, rows, cols, kappa, eta1, eta2)
