// Host-side plan: cluster tree, hierarchical directions, block tree and the
// column sets F_tc of both bases.  Pure C++17, no device code.
//
// Every floating-point predicate is evaluated with a fixed expression order
// (no contraction) so that the integer results are reproducible bit for bit
// by any implementation that evaluates the same IEEE expressions.
#pragma once

#include <cstdint>
#include <vector>

namespace dh2 {

struct ClusterTree {
  int64_t n = 0;
  std::vector<int64_t> perm;   // perm[pos] = original index
  std::vector<int64_t> off, size;
  std::vector<int32_t> level, father, son1, son2;
  std::vector<double> lo, hi;  // 3 per cluster
  std::vector<double> diam;
  int32_t depth = 0;
  std::vector<double> delta;   // per level
  int32_t nc() const { return (int32_t)off.size(); }
  bool leaf(int32_t t) const { return son1[t] < 0; }
};

struct Directions {
  std::vector<int32_t> per_edge;            // m_l
  std::vector<std::vector<double>> dirs;    // 3 * |D_l| per level
  std::vector<std::vector<int32_t>> sd;     // level l -> index on l+1 (depth levels)
  int32_t count(int32_t l) const { return (int32_t)(dirs[l].size() / 3); }
};

struct BlockTree {
  std::vector<int32_t> adm_t, adm_s, adm_c;
  std::vector<int32_t> near_t, near_s;
};

// One entry (b, s, d) of a column set: admissible block b whose column
// cluster (for this basis) is s, contributing with level difference d.
struct ColEntry {
  int32_t b, s, d;
};

// Column sets of one basis as a flat item list: items ordered by cluster
// (pre-order) then direction; entries of item i in [begin[i], begin[i+1]).
struct ColumnSets {
  std::vector<int32_t> item_t, item_c;
  std::vector<int64_t> begin;
  std::vector<ColEntry> ent;
  // per cluster: first item index and count
  std::vector<int32_t> first, count;
  int32_t nitems() const { return (int32_t)item_t.size(); }
  // item index of (t,c), -1 if unused
  int32_t find(int32_t t, int32_t c) const;
};

ClusterTree build_cluster_tree(const double* pts, int64_t n, int32_t leaf_size);
Directions build_directions(const ClusterTree& tr, double kappa, double eta1, bool lowfreq_zero);
BlockTree build_block_tree(const ClusterTree& tr, const Directions& dr, double kappa, double eta2,
                           bool standard_only);
// side 0: row basis (own blocks by row cluster), side 1: column basis.
ColumnSets build_column_sets(const ClusterTree& tr, const Directions& dr, const BlockTree& bt,
                             int side);

}  // namespace dh2
