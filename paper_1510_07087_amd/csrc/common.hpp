// Structures shared between the host scheduler and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dh2 {

// Source of matrix entries.
// SRC_DLP: the double-layer entries of the Helmholtz kernel generated from
// the points and their normals (FP64 form; row and column data hold
// positions, as for the dense source)
enum EntrySource : int32_t { SRC_HELMHOLTZ = 0, SRC_DENSE = 1, SRC_DLP = 2 };

// Geometry and matrix access, all in the permuted (cluster-tree) order.
struct GeomDev {
  const double* pts;      // n x 4: x, y, z, w
  const float* pts32;     // n x 4 (mixed precision), may be null
  const double* G;        // dense complex128, ORIGINAL order, row-major (interleaved)
  const int64_t* perm;    // position -> original index
  int64_t ldg;            // leading dimension of G in complex elements
  const double* cbox;     // per cluster: lo[3], hi[3], largest weight, 0 (bounds of entries)
  const double* nrm;      // SRC_DLP: n x 4 unit normals (nx, ny, nz, 0), permuted order
  int64_t n;
  double kappa;
};

// One (cluster, direction) block row of a basis.
struct ItemDev {
  int64_t row_off;   // first permuted position of the cluster
  int64_t N;         // number of columns of F_tc
  int64_t ent_begin; // leaf: first column-set entry
  int64_t ent_end;
  int64_t col_off;   // non-leaf: offset of F_tc inside the sons' sets
  int64_t ninh;      // columns of F_tc inherited from the father (the first ninh)
  void* R;           // R^T of the inherited columns (ninh x k, complex FP64 or FP32),
                     // in the arena of its level
  void* Rown;        // row basis: R^T of the own-block columns ((N - ninh) x k), kept
                     // for the projection; null in the column basis (not formed)
  double2* M;        // Gram (r x r, column-major)
  double2* Q;        // factor: r x k row-major (leaf: Q_tc, other: [E_t1c; E_t2c])
  double* sig;       // singular values (r)
  double4* cols;     // leaf: per-column data of F_tc for the current level (x, y, z, factor)
  float* rmax;       // mixed form: largest |component| of every row of R (k values)
  int32_t m;         // rows of the cluster
  int32_t r;         // rows of the factor (m or k1+k2)
  int32_t k;         // rank (filled by the factorisation)
  int32_t leaf;
  int32_t son[2];    // non-leaf: item ids of (t1,c'), (t2,c')
  int32_t level;
  int32_t pad;
};

// Column-set entry for generated block rows.
struct EntDev {
  int64_t col_start;  // first column of this entry inside F_tc
  int64_t pos;        // first permuted position of the column cluster
  int64_t len;        // number of columns
  int32_t b;          // admissible block
  int32_t d;          // level difference
  double scale;       // 1 / (omega_b zeta^d)
  int32_t s;          // column cluster
  int32_t pad;
};

// A contiguous column range of one block row, processed by one workgroup.
struct UnitDev {
  int32_t item;
  // Gram units: row tiles [a0, a0+na) against row tiles [b0, b0+nb) of the
  // 16-row tiles of the factor; a0 == b0 marks a diagonal block (pairs J <= I)
  int8_t a0, na, b0, nb;
  int64_t col_begin;
  int64_t ncols;
  int64_t slot_off;   // partial-Gram slot offset in complex elements (Gram units)
};

// Projection task: S_b = omega_b * (R_tc restricted to the columns of s) * Wexp_sc.
struct ProjDev {
  const void* R;      // R^T rows of the block (|s| x kt), complex FP64 or FP32
  const void* W;      // expanded column basis (|s| x ks row-major), complex FP64 or FP32
  void* S;            // output (kt x ks column-major), complex FP64 (FP64 form) or FP32 (mixed)
  int32_t kt, ks;
  int32_t ns;         // |s|
  int32_t b;
};

// Stacked projection of the mixed form: the blocks of one level that share
// the expanded column basis W_sc are stacked row-wise (their R rows one after
// the other); a tile is up to 64 consecutive stacked rows.
struct PBlkDev {
  const float2* R;  // R^T rows of the block: column j of s at R[j * kt + i]
  float2* S;        // output (kt x ks column-major)
  int32_t kt, b;
};
struct PTileDev {
  const float2* W;  // expanded column basis (|s| x ks row-major), complex FP32
  int32_t blk0;     // block holding the tile's first row (index into the PBlkDev array)
  int32_t i0;       // that row inside blk0
  int32_t rows;     // stacked rows of the tile (1..64)
  int32_t nblk;     // blocks the tile intersects (1..64)
  int32_t ns, ks;   // |s| and the rank of W (1..64)
};

// Conversion task of the mixed form: count complex values FP64 -> FP32.
struct CvtDev {
  const double2* src;
  float2* dst;
  int64_t count;
};

// Expansion task: rows of one son inside Wexp_sc = Wexp_{s_i c'} E_{s_i c}.
struct ExpandDev {
  const double2* src; // Wexp of the son (rows x ks) row-major
  const double2* E;   // E rows inside the father's factor (ks x k row-major)
  double2* dst;       // destination rows inside the father's Wexp
  int32_t rows;       // |s_i|
  int32_t ks;         // son rank
  int32_t k;          // father rank
  int32_t pad;
};

// Task of the matrix-vector product's last step: rows of one leaf cluster,
// its items in the basis being applied (first task of the leaf only), and a
// range of its references into the near field.  slot < 0: the task holds all
// of the leaf's work and writes its rows; otherwise it writes partial sums
// into slot `slot` of the partial buffer (64 rows x nr), added per leaf in
// slot order afterwards.  For that reduction item_first / item_count give
// the leaf's first slot and slot count.
struct LeafDev {
  int64_t row_off;
  int32_t len;
  int32_t item_first;
  int32_t item_count;
  int32_t slot;
  int64_t near_begin;
  int64_t near_end;
};

// Inadmissible block: its dense entries (|t| x |s| column-major) at off.
struct NearDev {
  int64_t off;
  int64_t t_off, t_len;
  int64_t s_off, s_len;
};

// A leaf's reference to a near-field block that contains its rows.
struct NearRefDev {
  int64_t b;
  int64_t row0;   // first row (op N) or column (op C) of the leaf inside the block
};

constexpr int kMaxR = 128;      // largest factor size of the LDS-resident kernels
constexpr int kMaxRBig = 512;   // largest factor size of the kernels that stage in memory

}  // namespace dh2
