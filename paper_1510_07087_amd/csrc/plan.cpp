// Host-side plan construction (see plan.hpp).
//
// Cluster tree: tight bounding box, split of the longest edge (lowest axis on
// ties) at 0.5*(lo+hi), stable partition (coordinate < mid first), leaves at
// <= leaf_size indices or zero extent; clusters numbered in depth-first
// pre-order.  (Definition "Cluster tree"; the paper's experiments use
// geometrically regular subdivision.)
//
// Directions: m_l = ceil(sqrt(2) kappa delta_l / eta1) squares per cube-face
// edge, faces +x,-x,+y,-y,+z,-z, midpoints normalised (Section 3 and Lemma
// "Projection"); son maps to the nearest direction of the next level
// (Definition "Hierarchical directions").
//
// Block tree: admissible iff kappa*dmax^2 <= eta2*dist and dmax <= eta2*dist
// (Section 3, conditions (b) and (c)); otherwise split when both clusters
// have sons, else an inadmissible leaf.  c_b is the direction nearest to
// (m_t - m_s)/|m_t - m_s| (condition (a)).
//
// Column sets (Section 6, F_tc): inherited from the father through the son
// map (father directions in increasing order), then own admissible blocks in
// block order.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <map>

namespace dh2 {

static double box_diam(const double* lo, const double* hi) {
  double e0 = hi[0] - lo[0];
  double e1 = hi[1] - lo[1];
  double e2 = hi[2] - lo[2];
  return std::sqrt(e0 * e0 + e1 * e1 + e2 * e2);
}

ClusterTree build_cluster_tree(const double* pts, int64_t n, int32_t leaf_size) {
  ClusterTree tr;
  tr.n = n;
  tr.perm.resize(n);
  for (int64_t i = 0; i < n; ++i) tr.perm[i] = i;
  struct Job {
    int64_t off, size;
    int32_t level, father, slot;
  };
  std::vector<Job> stack;
  stack.push_back({0, n, 0, -1, 0});
  std::vector<int64_t> left, right;
  while (!stack.empty()) {
    Job j = stack.back();
    stack.pop_back();
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = pts[3 * tr.perm[j.off] + a];
      hi[a] = lo[a];
    }
    for (int64_t p = j.off; p < j.off + j.size; ++p) {
      const double* x = pts + 3 * tr.perm[p];
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], x[a]);
        hi[a] = std::max(hi[a], x[a]);
      }
    }
    int32_t cid = (int32_t)tr.off.size();
    tr.off.push_back(j.off);
    tr.size.push_back(j.size);
    tr.level.push_back(j.level);
    tr.father.push_back(j.father);
    tr.son1.push_back(-1);
    tr.son2.push_back(-1);
    for (int a = 0; a < 3; ++a) tr.lo.push_back(lo[a]);
    for (int a = 0; a < 3; ++a) tr.hi.push_back(hi[a]);
    if (j.father >= 0) {
      if (j.slot == 0)
        tr.son1[j.father] = cid;
      else
        tr.son2[j.father] = cid;
    }
    if (j.size <= leaf_size) continue;
    double ext[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    int axis = 0;
    for (int a = 1; a < 3; ++a)
      if (ext[a] > ext[axis]) axis = a;
    if (!(ext[axis] > 0.0)) continue;
    double mid = 0.5 * (lo[axis] + hi[axis]);
    left.clear();
    right.clear();
    for (int64_t p = j.off; p < j.off + j.size; ++p) {
      int64_t i = tr.perm[p];
      if (pts[3 * i + axis] < mid)
        left.push_back(i);
      else
        right.push_back(i);
    }
    int64_t nl = (int64_t)left.size();
    std::copy(left.begin(), left.end(), tr.perm.begin() + j.off);
    std::copy(right.begin(), right.end(), tr.perm.begin() + j.off + nl);
    stack.push_back({j.off + nl, j.size - nl, j.level + 1, cid, 1});
    stack.push_back({j.off, nl, j.level + 1, cid, 0});
  }
  int32_t nc = tr.nc();
  tr.diam.resize(nc);
  tr.depth = 0;
  for (int32_t t = 0; t < nc; ++t) {
    tr.diam[t] = box_diam(&tr.lo[3 * t], &tr.hi[3 * t]);
    tr.depth = std::max(tr.depth, tr.level[t]);
  }
  tr.delta.assign(tr.depth + 1, 0.0);
  for (int32_t t = 0; t < nc; ++t)
    if (tr.diam[t] > tr.delta[tr.level[t]]) tr.delta[tr.level[t]] = tr.diam[t];
  return tr;
}

static int32_t nearest_direction(const std::vector<double>& dirs, const double* z) {
  int32_t best = 0;
  double bd = INFINITY;
  int32_t nd = (int32_t)(dirs.size() / 3);
  for (int32_t i = 0; i < nd; ++i) {
    double dx = z[0] - dirs[3 * i + 0];
    double dy = z[1] - dirs[3 * i + 1];
    double dz = z[2] - dirs[3 * i + 2];
    double d2 = dx * dx + dy * dy + dz * dz;
    if (d2 < bd) {
      bd = d2;
      best = i;
    }
  }
  return best;
}

static std::vector<double> cube_directions(int32_t m) {
  std::vector<double> out;
  if (m == 0) {
    out.assign(3, 0.0);
    return out;
  }
  out.reserve((size_t)18 * m * m);
  for (int face = 0; face < 6; ++face) {
    int axis = face / 2;
    double sign = (face % 2 == 0) ? 1.0 : -1.0;
    for (int32_t i = 0; i < m; ++i) {
      double u = -1.0 + (2.0 * i + 1.0) / (double)m;
      for (int32_t j = 0; j < m; ++j) {
        double v = -1.0 + (2.0 * j + 1.0) / (double)m;
        double x, y, z;
        if (axis == 0) {
          x = sign; y = u; z = v;
        } else if (axis == 1) {
          x = u; y = sign; z = v;
        } else {
          x = u; y = v; z = sign;
        }
        double nrm = std::sqrt(x * x + y * y + z * z);
        out.push_back(x / nrm);
        out.push_back(y / nrm);
        out.push_back(z / nrm);
      }
    }
  }
  return out;
}

Directions build_directions(const ClusterTree& tr, double kappa, double eta1, bool lowfreq_zero) {
  Directions dr;
  for (int32_t l = 0; l <= tr.depth; ++l) {
    double kd = kappa * tr.delta[l];
    int32_t m;
    if (kd == 0.0 || (lowfreq_zero && kd <= eta1)) {
      m = 0;
    } else {
      double x = std::sqrt(2.0) * kappa * tr.delta[l] / eta1;
      m = (int32_t)std::ceil(x);
    }
    dr.per_edge.push_back(m);
    dr.dirs.push_back(cube_directions(m));
  }
  for (int32_t l = 0; l < tr.depth; ++l) {
    const auto& cur = dr.dirs[l];
    const auto& nxt = dr.dirs[l + 1];
    int32_t nd = (int32_t)(cur.size() / 3);
    std::vector<int32_t> sd(nd);
    for (int32_t c = 0; c < nd; ++c) sd[c] = nearest_direction(nxt, &cur[3 * c]);
    dr.sd.push_back(std::move(sd));
  }
  return dr;
}

static double box_dist(const double* lo_t, const double* hi_t, const double* lo_s,
                       const double* hi_s) {
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    double g = std::max(0.0, std::max(lo_s[a] - hi_t[a], lo_t[a] - hi_s[a]));
    d2 = d2 + g * g;
  }
  return std::sqrt(d2);
}

BlockTree build_block_tree(const ClusterTree& tr, const Directions& dr, double kappa, double eta2,
                           bool standard_only) {
  BlockTree bt;
  std::vector<std::pair<int32_t, int32_t>> stack;
  stack.push_back({0, 0});
  while (!stack.empty()) {
    auto [t, s] = stack.back();
    stack.pop_back();
    const double* lt = &tr.lo[3 * t];
    const double* ht = &tr.hi[3 * t];
    const double* ls = &tr.lo[3 * s];
    const double* hs = &tr.hi[3 * s];
    double dmax = std::max(tr.diam[t], tr.diam[s]);
    double dist = box_dist(lt, ht, ls, hs);
    // separated boxes only: (b) and (c) hold trivially for a one-point
    // cluster with itself (diam = dist = 0), a block with the singular
    // diagonal entry
    bool cond_c = dist > 0.0 && dmax <= eta2 * dist;
    bool adm = cond_c;
    if (!standard_only) adm = (kappa * (dmax * dmax) <= eta2 * dist) && cond_c;
    if (adm) {
      double mt[3], ms[3], u[3];
      for (int a = 0; a < 3; ++a) {
        mt[a] = 0.5 * (lt[a] + ht[a]);
        ms[a] = 0.5 * (ls[a] + hs[a]);
        u[a] = mt[a] - ms[a];
      }
      double nrm = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      double z[3] = {u[0] / nrm, u[1] / nrm, u[2] / nrm};
      bt.adm_t.push_back(t);
      bt.adm_s.push_back(s);
      bt.adm_c.push_back(nearest_direction(dr.dirs[tr.level[t]], z));
    } else if (tr.son1[t] >= 0 && tr.son1[s] >= 0) {
      int32_t ts[2] = {tr.son1[t], tr.son2[t]};
      int32_t ss[2] = {tr.son1[s], tr.son2[s]};
      for (int a = 1; a >= 0; --a)
        for (int b = 1; b >= 0; --b) stack.push_back({ts[a], ss[b]});
    } else {
      bt.near_t.push_back(t);
      bt.near_s.push_back(s);
    }
  }
  return bt;
}

int32_t ColumnSets::find(int32_t t, int32_t c) const {
  int32_t f = first[t], e = first[t] + count[t];
  // items of a cluster are sorted by direction
  int32_t lo = f, hi = e;
  while (lo < hi) {
    int32_t mid = (lo + hi) / 2;
    if (item_c[mid] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < e && item_c[lo] == c) ? lo : -1;
}

ColumnSets build_column_sets(const ClusterTree& tr, const Directions& dr, const BlockTree& bt,
                             int side) {
  int32_t nc = tr.nc();
  std::vector<std::vector<int32_t>> own(nc);
  int64_t nadm = (int64_t)bt.adm_t.size();
  for (int64_t b = 0; b < nadm; ++b) own[side == 0 ? bt.adm_t[b] : bt.adm_s[b]].push_back((int32_t)b);
  std::vector<std::map<int32_t, std::vector<ColEntry>>> F(nc);
  ColumnSets cs;
  cs.first.assign(nc, 0);
  cs.count.assign(nc, 0);
  for (int32_t t = 0; t < nc; ++t) {  // pre-order: fathers first
    int32_t fa = tr.father[t];
    auto& Ft = F[t];
    if (fa >= 0) {
      const auto& sdf = dr.sd[tr.level[fa]];
      for (const auto& kv : F[fa]) {  // increasing father direction
        auto& dst = Ft[sdf[kv.first]];
        for (const ColEntry& e : kv.second) dst.push_back({e.b, e.s, e.d + 1});
      }
    }
    for (int32_t b : own[t]) {
      int32_t partner = side == 0 ? bt.adm_s[b] : bt.adm_t[b];
      Ft[bt.adm_c[b]].push_back({b, partner, 0});
    }
    cs.first[t] = (int32_t)cs.item_t.size();
    for (const auto& kv : Ft) {
      cs.item_t.push_back(t);
      cs.item_c.push_back(kv.first);
      cs.begin.push_back((int64_t)cs.ent.size());
      cs.ent.insert(cs.ent.end(), kv.second.begin(), kv.second.end());
    }
    cs.count[t] = (int32_t)cs.item_t.size() - cs.first[t];
    // free the father's sets once both sons are done
    if (fa >= 0 && tr.son2[fa] == t) F[fa].clear();
  }
  cs.begin.push_back((int64_t)cs.ent.size());
  return cs;
}

}  // namespace dh2
