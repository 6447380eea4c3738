// Launchers of the gfx950 kernels (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace dh2 {

// spectral norms of the admissible blocks (power method, clusters of at most
// block_norm2_max_size() points)
void launch_block_norm2(int src, const GeomDev& g, const int64_t* t_off, const int64_t* t_len,
                        const int64_t* s_off, const int64_t* s_len, int64_t nblocks,
                        int max_iter, double tol, double* omega, hipStream_t st);
int block_norm2_max_size();
void launch_block_norm(int src, const GeomDev& g, const int64_t* t_off, const int64_t* t_len,
                       const int64_t* s_off, const int64_t* s_len, int64_t nblocks, double* omega,
                       hipStream_t st);
void launch_entry_scale(EntDev* ent, int64_t nent, const double* omega, double zeta,
                        hipStream_t st);
void launch_gram(int src, bool inner, bool mixed, const GeomDev& g, const ItemDev* items,
                 const EntDev* ents, const UnitDev* units, int64_t nunits, double zeta, int side,
                 double2* partial, hipStream_t st);
void launch_gram_reduce(const ItemDev* items, const int32_t* litems, int32_t nl,
                        const int32_t* ubegin, const UnitDev* units, const double2* partial,
                        hipStream_t st);
// ranks k of items [0, n) into out (the host reads them back after a level's
// factorisations)
void launch_ranks(const ItemDev* items, int32_t n, int32_t* out, hipStream_t st);
void launch_factor(ItemDev* items, const int32_t* litems, int32_t nl, int32_t rmax, double eps,
                   int max_sweeps, int32_t* status, hipStream_t st, bool wide = false);
// factors with r up to kMaxRBig, X of the q-th listed item at xptr[q]
// (r (r + 1) complex elements)
void launch_factor_big(ItemDev* items, const int32_t* litems, int32_t nl, double eps,
                       int max_sweeps, int32_t* status, double2* const* xptr, hipStream_t st);
// Column data (x, y, z, factor) of the listed leaf items into their it.cols.
void launch_leaf_cols(int src, const GeomDev& g, const ItemDev* items, const int32_t* litems,
                      int32_t nl, const EntDev* ents, int side, bool mixed, hipStream_t st);
// Mixed form: Gram units of one workgroup each on int8 MFMA (leaf block rows
// generated, non-leaf block rows from the sons' FP32 R).
void launch_gram_i8(bool inner, const GeomDev& g, const ItemDev* items, const EntDev* ents,
                    const UnitDev* units, int64_t nunits, double zeta, int side, double2* partial,
                    hipStream_t st, bool dlp = false);
// LDS bytes of the non-leaf R-product workgroup for an item (r rows, rank k)
size_t rprod_inner_lds(bool mixed, int r, int k);
size_t rprod_inner_lds_max();
// R-products: one workgroup per unit; non-leaf launches hold units of items
// with ceil(k / 16) = kt only
void launch_rprod_leaf(int src, bool mixed, const GeomDev& g, const ItemDev* items,
                       const EntDev* ents, const UnitDev* units, int64_t nunits, int side,
                       hipStream_t st);
void launch_rprod_inner(bool mixed, int kt, const ItemDev* items, const UnitDev* units,
                        int64_t nunits, double zeta, size_t lds, hipStream_t st);
// Large transfer factors: Q_hat of item[q] packed into 64-column chunk
// chunk[q] at dst[q] ((r + 8) x 64, compute precision); R^T units with the
// chunk index in UnitDev::a0 and the chunk's address in qchunk[unit]
void launch_pack_q(const ItemDev* items, const int32_t* item, const int32_t* chunk,
                   void* const* dst, int64_t ntasks, bool mixed, hipStream_t st);
void launch_rprod_inner_big(bool mixed, const ItemDev* items, const UnitDev* units,
                            int64_t nunits, double zeta, const void* const* qchunk,
                            hipStream_t st);
void launch_expand(const ExpandDev* tasks, int64_t ntasks, hipStream_t st);
void launch_cvt(const CvtDev* tasks, int64_t ntasks, hipStream_t st);
// one workgroup per task, 8-byte words
void launch_copy_c(const double2* src, int64_t src_off, double2* dst, int64_t dst_off,
                   int64_t count, hipStream_t st);
void launch_project(bool mixed, const ProjDev* tasks, int64_t ntasks, const double* omega,
                    hipStream_t st);
// mixed form, blocks stacked by shared W (ks <= 64): one launch per column
// group count nc = ceil(ks / 4) in 1..16
void launch_project_stacked(int nc, const PTileDev* tiles, int64_t ntiles, const PBlkDev* blks,
                            const double* omega, hipStream_t st);
// blocks with ks <= 64: every task of one launch has ceil(ks/16) = nj and is
// processed in passes of ni = min(ceil(kt/16), project_rows_per_pass) row tiles
int project_rows_per_pass(bool mixed, int nj);
// split: one workgroup per task with the columns of s divided among its waves
void launch_project_tiled(bool mixed, int ni, int nj, bool split, const ProjDev* tasks,
                          int64_t ntasks, const double* omega, hipStream_t st);
// f32 (below): the coupling matrices and near-field blocks are stored as
// complex FP32 (mixed form), else as complex FP64; products with them are FP64.
void launch_near(int src, const GeomDev& g, const int64_t* t_off, const int64_t* t_len,
                 const int64_t* s_off, const int64_t* s_len, const int64_t* out_off,
                 int64_t nblocks, void* out, int f32, hipStream_t st);
// Device address of this device's scratch array for the allocation-free
// matrix-vector product (looked up once per device), and its size in bytes.
hipError_t noalloc_scratch(void** out);
size_t noalloc_scratch_bytes();
// Matrix-vector product kernels.  Work vectors hold nr <= 8 right-hand
// sides interleaved (entry p of right-hand side q at [p * nr + q]); the
// caller's vectors are column-major (x[q * n + i]).
void launch_gather_perm(const double2* x, const int64_t* perm, int64_t n, double2* xp,
                        hipStream_t st, int nr = 1);
void launch_scatter_perm(const double2* yp, const int64_t* perm, int64_t n, double2* y,
                         hipStream_t st, int nr = 1);
void launch_fwd_leaf(const ItemDev* items, const int32_t* litems, int32_t nl,
                     const int64_t* xh_off, const double2* xp, double2* xh, int nr,
                     hipStream_t st);
void launch_fwd_inner(const ItemDev* items, const int32_t* litems, int32_t nl,
                      const int64_t* xh_off, double2* xh, int nr, hipStream_t st);
void launch_coupling_transpose(const void* const* S, void* const* ST, const int32_t* rows,
                               const int32_t* cols, int64_t nblocks, int f32, hipStream_t st);
void launch_coupling(const ItemDev* items, int32_t nitems, int32_t nheavy,
                     const int32_t* order, const int64_t* cbegin, const int32_t* cblock,
                     const int32_t* cpartner, const void* const* S_ptr,
                     const int32_t* S_rows, const int32_t* S_cols, const int64_t* xh_off,
                     const double2* xh, const int64_t* yh_off, double2* yh, int adjoint, int nr,
                     int f32, hipStream_t st);
void launch_bwd_inner(const ItemDev* items, const int32_t* litems, int32_t nl,
                      const int64_t* fbegin, const int32_t* fitem, const int32_t* fsonidx,
                      const int64_t* yh_off, double2* yh, int nr, hipStream_t st);
void launch_bwd_leaf(const ItemDev* items, const LeafDev* leaves, int32_t nleaves,
                     const NearRefDev* nref, const NearDev* nears, const void* nearv,
                     const void* nearT, const int64_t* yh_off, const double2* yh,
                     const double2* xp, double2* yp, double2* partial, int adjoint, int nr,
                     int near, int accumulate, int f32, hipStream_t st);
void launch_leaf_sum(const LeafDev* leaves, int32_t nleaves, const double2* partial, double2* yp,
                     int nr, hipStream_t st);
void launch_near_transpose(const NearDev* nears, int64_t nblocks, const void* B, void* BT,
                           int f32, hipStream_t st);
void launch_direct(int src, const GeomDev& g, const int64_t* rows, int64_t nrows,
                   const double2* xp, int adjoint, double2* out, hipStream_t st);

}  // namespace dh2
