/*
 * dh2.h -- C ABI of the MI355X directional H2-matrix compression library.
 *
 * The library approximates a dense complex matrix G (given as a device array,
 * or generated on the device from points, weights and a wave number) by a
 * directional H2 (DH2) matrix, following S. Boerm, "Directional H2-matrix
 * compression for high-frequency problems" (2015):
 *
 *   - cluster tree over the points (Definition "Cluster tree", geometric
 *     bisection of the tight bounding box),
 *   - hierarchical directions D_l and son maps sd_l (Definition
 *     "Hierarchical directions"; cube-face construction of Section 3),
 *   - block tree with the parabolic and standard admissibility conditions
 *     (Section 3, conditions (b) and (c)) and block directions c_b,
 *   - compression (Section 6): orthonormal nested row and column bases built
 *     bottom-up from the weighted block rows G^w_tc by truncated singular value
 *     decompositions, transfer matrices E, coupling matrices
 *     S_b = V_{t c_b}^* G|_b W_{s c_b}, and the near field G|_b for the
 *     inadmissible leaves,
 *   - the DH2 matrix-vector product (Section 4) and the relative spectral
 *     error measured by a power iteration (Section 7).
 *
 * Conventions (all entry points):
 *   - Every vector and matrix argument is in the caller's ORIGINAL point order;
 *     the library owns the cluster-tree permutation.
 *   - Complex numbers are interleaved (re, im) doubles: the layout of
 *     torch.complex128 and C99 double _Complex.
 *   - "device" pointers are HIP device addresses on the current device;
 *     "host" pointers are ordinary host memory.  Device work is enqueued on
 *     `stream` (a hipStream_t passed as void*, NULL = the null stream).
 *     Functions that return host results synchronise that stream.
 *   - Inputs are borrowed for the duration of the call only; the library
 *     copies what it keeps.  Handles are owned by the library until the
 *     matching *_free call.
 *   - Every entry point returns a dh2_status and never throws.  On failure the
 *     output handle is left untouched and dh2_last_error() describes the
 *     failure (thread-local string, valid until the next call on the thread).
 */
#ifndef DH2_H
#define DH2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DH2_OK = 0,
  DH2_EINVAL = -1,      /* invalid argument (sizes, NaN/Inf, parameters)     */
  DH2_ENOMEM = -2,      /* device memory exhausted or max_device_bytes hit   */
  DH2_EDEVICE = -3,     /* HIP runtime error, or no GPU / no gfx950 code     */
  DH2_ENOTCONV = -4,    /* a Jacobi SVD exceeded its sweep limit             */
  DH2_EUNSUPPORTED = -5 /* a size the kernels do not handle (e.g. rank cap)  */
} dh2_status;

typedef enum { DH2_FP64 = 0, DH2_MIXED = 1 } dh2_precision;

typedef struct dh2_tree_s* dh2_tree;     /* points, cluster tree, directions */
typedef struct dh2_blocks_s* dh2_blocks; /* block tree, column sets          */
typedef struct dh2_matrix_s* dh2_matrix; /* compressed DH2 representation    */

/* Parameters.  Defaults (dh2_opts_default): leaf_size 32, eta1 20, eta2 5,
 * zeta 2/3, precision DH2_FP64, no memory cap, automatic subtree grouping,
 * block weights DH2_WEIGHTS_BLOCK, 60 Jacobi sweeps at most.
 *   eta1 : direction parameter; D_l covers the unit sphere with
 *          max distance eta1/(kappa*delta_l) (Section 3).
 *   eta2 : admissibility parameter of conditions (b) and (c).
 *   zeta : level factor of the local tolerances (error-control remark);
 *          must satisfy 2*zeta^2 < 1 for binary cluster trees.
 *   lowfreq_zero_dir : use the single direction 0 on levels with
 *          kappa*delta_l <= eta1 (valid since |z - 0| = 1 <= eta1/(kappa delta)).
 *   standard_only : admissibility by condition (c) alone (Section 7, the
 *          comparison with cross approximation).
 *   max_device_bytes : cap on the library's device allocations (0 = none).
 *   groups : number of subtree groups swept one after another to bound the
 *          memory of the coefficient matrices R (0 = automatic).
 *   weights : block weights omega_b of the remark on error control.
 *          DH2_WEIGHTS_BLOCK (0): omega_b = ||G|_b||_F, block-relative error
 *          bounds (the paper's experiments).  DH2_WEIGHTS_GLOBAL (1): every
 *          block gets (sum over admissible b' of ||G|_b'||_F^2)^(1/2), a
 *          global-relative tolerance.  DH2_WEIGHTS_SPECTRAL (2):
 *          omega_b = ||G|_b||_2 (power method on the device, clusters of at
 *          most 1024 points, else DH2_EUNSUPPORTED).
 *   max_sweeps : limit of the one-sided Jacobi sweeps of each small SVD
 *          (0 = 60); a factorisation that still rotates after that many
 *          sweeps makes the compression fail with DH2_ENOTCONV.  */
typedef struct {
  int32_t leaf_size;
  double eta1;
  double eta2;
  double zeta;
  int32_t precision;
  int32_t lowfreq_zero_dir;
  int32_t standard_only;
  int32_t groups;
  int64_t max_device_bytes;
  int32_t weights;
  int32_t max_sweeps;
} dh2_opts;

typedef enum { DH2_WEIGHTS_BLOCK = 0, DH2_WEIGHTS_GLOBAL = 1, DH2_WEIGHTS_SPECTRAL = 2 } dh2_weights;

void dh2_opts_default(dh2_opts* opts);

/* Human-readable description of the last failure on this thread. */
const char* dh2_last_error(void);

/* ---------------------------------------------------------------------------
 * Cluster tree and directions (Definitions "Cluster tree", "Hierarchical
 * directions"; Section 3 construction).
 *   pts   : host, n x 3 row-major float64 point coordinates (copied).
 *   kappa : wave number >= 0.
 * EINVAL: n < 1, non-finite coordinates, kappa < 0 or non-finite,
 *         leaf_size < 1, eta1 <= 0.                                         */
dh2_status dh2_tree_build(const double* pts, int64_t n, double kappa,
                          const dh2_opts* opts, dh2_tree* out);
void dh2_tree_free(dh2_tree tree);

typedef struct {
  int64_t n;
  int32_t nclusters;
  int32_t depth;      /* levels 0..depth                      */
  int32_t ndirs_total;/* sum over levels of |D_l|             */
  double kappa;
} dh2_tree_info;

dh2_status dh2_tree_get_info(dh2_tree tree, dh2_tree_info* info);

/* Copies the tree to host arrays sized from dh2_tree_get_info:
 *   perm[n]      : perm[p] = original index of the point at position p,
 *   off[nc], size[nc] : index range of each cluster in permuted order,
 *   level[nc], son1[nc], son2[nc] (-1 for leaves; clusters in pre-order),
 *   lo[3nc], hi[3nc] : tight bounding boxes, diam[nc] : box diagonals,
 *   delta[depth+1]   : per-level maximal diameter.
 * Any pointer may be NULL to skip that array.                               */
dh2_status dh2_tree_export(dh2_tree tree, int64_t* perm, int64_t* off,
                           int64_t* size, int32_t* level, int32_t* son1,
                           int32_t* son2, double* lo, double* hi, double* diam,
                           double* delta);

/* Directions of one level: ndir (out), dirs[3*ndir] (unit vectors or 0) and
 * sd[ndir] (son map to level+1; -1 on the deepest level).  Call with
 * dirs == sd == NULL first to get ndir.                                     */
dh2_status dh2_tree_directions(dh2_tree tree, int32_t level, int32_t* ndir,
                               double* dirs, int32_t* sd);

/* ---------------------------------------------------------------------------
 * Block tree (Definition "Block tree"; admissibility (b) and (c); minimal
 * tree) and the column sets F_tc of Section 6 for both bases.
 * EINVAL: eta2 <= 0.                                                        */
dh2_status dh2_blocks_build(dh2_tree tree, const dh2_opts* opts, dh2_blocks* out);
void dh2_blocks_free(dh2_blocks blocks);

typedef struct {
  int64_t nadm;        /* admissible leaves L+                      */
  int64_t nnear;       /* inadmissible leaves L-                    */
  int64_t near_entries;/* sum of |t||s| over L-                     */
  int32_t items[2];    /* used (t,c) pairs: [0] row basis, [1] column basis */
  int64_t entries[2];  /* column-set entries (b,s,d) per basis      */
} dh2_blocks_info;

dh2_status dh2_blocks_get_info(dh2_blocks blocks, dh2_blocks_info* info);

/* Block lists in construction (depth-first) order.  adm_c is the index of c_b
 * in D_level(t).  Any pointer may be NULL.                                  */
dh2_status dh2_blocks_export(dh2_blocks blocks, int32_t* adm_t, int32_t* adm_s,
                             int32_t* adm_c, int32_t* near_t, int32_t* near_s);

/* Column sets of one basis (side 0: rows of G, side 1: rows of G^*).
 * Items (t,c) with non-empty F_tc, ordered by cluster then direction; the
 * entries of item i are ent_*[item_begin[i] .. item_begin[i+1]) in set order:
 * block id, column cluster, and d = level(t) - level of the block.          */
dh2_status dh2_blocks_colsets(dh2_blocks blocks, int32_t side, int32_t* item_t,
                              int32_t* item_c, int64_t* item_begin,
                              int32_t* ent_b, int32_t* ent_s, int32_t* ent_d);

/* ---------------------------------------------------------------------------
 * Compression (Section 6, algorithm "basis" for both bases, coupling
 * matrices by projection, near field).  Each admissible block's columns are
 * weighted by 1/(omega_b zeta^(level(t)-level(t_b))) with omega_b = ||G|_b||_F;
 * ranks are the numbers of singular values above eps of the weighted block
 * rows, so that every block is approximated with error about eps*||G|_b||.
 *
 * dh2_compress_dense:
 *   G  : device, n x n complex128, row-major with leading dimension ld >= n,
 *        in ORIGINAL order.  Read only during the call.
 * dh2_compress_helmholtz: entries generated on the device,
 *        G_ij = w_j exp(i kappa r)/(4 pi r) (i != j, r = |x_i - x_j|),
 *        G_ii = sqrt(w_i/pi)/2 + i kappa w_i/(4 pi).
 *   w  : host, n float64 weights (copied); NULL means 4*pi/n for all points.
 * opts->precision selects complex FP64 throughout (DH2_FP64) or the mixed
 * form (DH2_MIXED; generated entries only: dh2_compress_helmholtz,
 * dh2_compress_helmholtz_dlp and dh2_compress_batch):
 * entries with an FP64 phase reduction and FP32 polynomials, Gram matrices
 * of the weighted block rows from exact int8 slices of their rows (int32
 * accumulation on int8 MFMA, converted to FP64), R^T stored in complex FP32
 * with FP32 MFMA R-products and projection, coupling matrices and near
 * field stored as complex FP32; factorisation, truncation and transfer
 * matrices stay FP64.  The slicing keeps about 2^-42 of the squared
 * row maxima in the Gram matrices, which places the mixed form at eps >=
 * 1e-5; smaller eps takes DH2_FP64.
 * EINVAL: eps <= 0 or non-finite, zeta <= 0 or 2 zeta^2 >= 1, ld < n,
 *         NaN/Inf in w, G or non-positive weights.
 * ENOMEM: allocation failure or max_device_bytes exceeded.
 * EUNSUPPORTED: a block row needs more columns in its factor than the
 *         kernels hold (numerical rank above 128).                          */
dh2_status dh2_compress_dense(dh2_blocks blocks, const void* G, int64_t ld,
                              double eps, const dh2_opts* opts, void* stream,
                              dh2_matrix* out);
dh2_status dh2_compress_helmholtz(dh2_blocks blocks, const double* w, double eps,
                                  const dh2_opts* opts, void* stream,
                                  dh2_matrix* out);

/* Double-layer operator of the Helmholtz kernel (Section 7, the DLP matrix
 * G = M/2 + G_dlp), entries generated on the device in collocation form:
 *   G_ij = w_j (1 - i kappa r) exp(i kappa r) <x_i - x_j, n_j> / (4 pi r^3)
 *   (i != j), G_ii = 1/2.
 *   w       : host, n float64 weights (copied); NULL means 4*pi/n.
 *   normals : host, n x 3 row-major float64 unit normals in the ORIGINAL
 *             point order (copied).
 * Both forms; in the mixed form the double-layer entries are computed in
 * FP64 and rounded to FP32 before the int8 slicing and the R-products.
 * Errors as for dh2_compress_helmholtz, EINVAL also for NULL or non-finite
 * normals.                                                                  */
dh2_status dh2_compress_helmholtz_dlp(dh2_blocks blocks, const double* w,
                                      const double* normals, double eps,
                                      const dh2_opts* opts, void* stream,
                                      dh2_matrix* out);
/* Independent Helmholtz instances in one call (same options and eps for
 * all): blocks[i] with weights w[i] (w or w[i] NULL: 4 pi / n_i).  The
 * instances run concurrently on a few internal streams (default priority),
 * ordered after the work already on `stream`; all work is complete when the
 * call returns.  outs[i] receives the matrix of instance i.
 * Errors: as dh2_compress_helmholtz; on error no handle is returned (the
 * matrices already built are freed) and outs is untouched.                 */
dh2_status dh2_compress_batch(int32_t count, const dh2_blocks* blocks,
                              const double* const* w, double eps,
                              const dh2_opts* opts, void* stream,
                              dh2_matrix* outs);
void dh2_matrix_free(dh2_matrix m);

/* Device memory freed by the library (matrices freed, per-level work arrays)
 * is kept in a process-wide cache, up to 80 % of the device memory, and
 * reused by later calls: handing touched memory back to the driver costs
 * about 10-20 ms per gigabyte.  The pinned host buffers that stage uploads
 * (32 MiB each, one per compression running at a time) are pooled the same
 * way.  This call returns both caches to the driver.  Do not call it while
 * another thread is inside a dh2 call.                                      */
void dh2_release_cached_memory(void);

/* ---------------------------------------------------------------------------
 * Matrix-vector product with the compressed matrix (Section 4: forward
 * transformation, coupling, backward transformation, near field).
 *   op   : 'N' for y = G~ x, 'C' for y = G~^* x.
 *   x, y : device, n x nrhs complex128, column-major (ld = n), ORIGINAL order.
 *          y is overwritten.
 * The near-field rows run on a second stream that the matrix owns, forked
 * from and joined back into `stream` with events, so that y is complete
 * when `stream` reaches this point.  The first call on a matrix builds the
 * product's index lists and transposed copies of the near field and of the
 * coupling matrices (for the adjoint; about as much memory again as those
 * parts of the representation).  Products on one matrix share its work
 * vectors: calls from several host threads must be serialised.          */
dh2_status dh2_matvec(dh2_matrix m, char op, int64_t nrhs, const void* x,
                      void* y, void* stream);

/* Allocation-free variant of dh2_matvec, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, layout and result as dh2_matvec;
 * it calls no hipMalloc, hipFree or allocating routine.
 *   - Its work vectors (permuted x and y, n complex each, the basis
 *     coefficients of the larger side, twice, and 64 complex partial sums
 *     per extra task of leaves whose near field is split over several tasks)
 *     live in a static device array of 64 MiB that the library holds on
 *     every device it runs on until the process ends.  A matrix whose work
 *     vectors exceed it is refused with DH2_EUNSUPPORTED (about n = 10^6
 *     points at the benchmark's ranks).
 *   - The product's index lists are built by the first dh2_matvec on the
 *     matrix; before that this call returns DH2_EINVAL.
 *   - The work is only enqueued (no wait), as for dh2_matvec; y is complete when the
 *     stream reaches this point.  Calls that overlap on one device share the
 *     array and race: serialise them on one stream.                        */
dh2_status dh2_matvec_noalloc(dh2_matrix m, char op, int64_t nrhs, const void* x,
                              void* y, void* stream);

/* Relative spectral error ||G - G~||_2 / ||G||_2 by the power method on
 * A^*A (Section 7), started from a seeded complex Gaussian vector; stops after
 * `iters` iterations or when the Rayleigh quotient changes by < 1e-4.
 *   G : device dense matrix as in dh2_compress_dense, or NULL to use the
 *       entries generated from the points (O(n^2) FP64 direct sums).
 *   rel_err : host, receives the estimate (a lower bound).                   */
dh2_status dh2_error_estimate(dh2_matrix m, const void* G, int64_t ld,
                              int32_t iters, uint64_t seed, double* rel_err,
                              void* stream);

/* Direct check of selected rows: computes (G x)_i by an FP64 sum over all j
 * on the device and (G~ x)_i through the DH2 product, for the given rows.
 *   rows : host, nrows original row indices.  x : device complex128 (n).
 *   direct, approx : host, nrows complex128 each (may be NULL).
 *   max_rel : host, max_i |(Gx)_i - (G~x)_i| / max_i |(Gx)_i|.              */
dh2_status dh2_rows_check(dh2_matrix m, const int64_t* rows, int32_t nrows,
                          const void* x, double* direct, double* approx,
                          double* max_rel, void* stream);

/* ---------------------------------------------------------------------------
 * Statistics and export. */
typedef struct {
  int64_t n;
  int64_t nadm, nnear;
  int32_t k_max;
  int32_t items[2];
  double mem_bytes;        /* bases + transfer + coupling + near field      */
  double mem_per_n_kib;    /* KiB per degree of freedom (complex128 words)  */
  /* device seconds per phase; the near field (t_near) is generated beside
   * the sweeps, and t_total is the device span of the whole compression    */
  double t_row, t_col, t_prj, t_near, t_total;
  /* algorithmic real flops (a complex multiply-add counts 8): per (t,c) with
   * r factor rows, N columns and rank k, 8 r^2 N for the reduction of the
   * block row and 8 k r N for R = Q^* A (columns actually formed); per
   * admissible block 8 k_t k_s #s for the projection                        */
  double flops_row, flops_col, flops_prj;
  double flops_gram, flops_rprod;              /* split of the basis flops   */
  double t_gram_kernel;    /* summed device seconds of the Gram kernels      */
  int32_t groups;          /* subtree groups used                            */
  int32_t precision;
  /* the leaf Gram kernel alone (the largest single kernel): algorithmic
   * flops 8 r^2 N summed over its launches, summed device seconds measured
   * with events on the call's stream, and the number of launches          */
  double flops_gram_leaf, t_gram_leaf;
  int32_t n_gram_leaf;
  int32_t pad;
  double flops_rprod_leaf;   /* R-product flops of leaf block rows */
  double ops_gram_leaf_i8;   /* mixed form: int8 MFMA operations of the leaf Gram
                                matrices, 60 r (r + 1) N per leaf block row      */
  double repr_bytes;         /* device bytes of the stored representation: bases
                                and transfer matrices complex FP64, coupling
                                matrices and near field complex FP64 (FP64 form)
                                or complex FP32 (mixed form); one matrix-vector
                                product reads them once                          */
} dh2_stats;

dh2_status dh2_get_stats(dh2_matrix m, dh2_stats* out);

/* Basis of one side (0 = row basis V, 1 = column basis W).
 * Sizes first: call with all arrays NULL to get nitems, nsigma, nmat.
 * Per item i (same order as dh2_blocks_colsets): cluster t, direction c,
 * rank k, r (rows of the factor: #t for leaves, k_son1 + k_son2 otherwise),
 * sigma[sig_off[i] .. + r) all singular values in descending order (values
 * below the factor resolution are reported as 0),
 * mat[2*mat_off[i] ..] the r x k column-major complex128 matrix: Q_tc for
 * leaves, [E_{t1 c}; E_{t2 c}] for other clusters.                          */
dh2_status dh2_basis_export(dh2_matrix m, int32_t side, int32_t* nitems,
                            int64_t* nsigma, int64_t* nmat, int32_t* item_t,
                            int32_t* item_c, int32_t* item_k, int32_t* item_r,
                            int64_t* sig_off, double* sigma, int64_t* mat_off,
                            double* mat);

/* Coupling matrices: S_b (k_t x k_s column-major complex128) at
 * 2*off[b] of `S`, off has nadm+1 entries.  Sizes first with S == NULL.
 * The mixed form stores S_b and the near field as complex FP32; both exports
 * widen the stored values exactly.                                          */
dh2_status dh2_coupling_export(dh2_matrix m, int64_t* off, double* S);

/* Near-field blocks G|_b (|t| x |s| column-major complex128, permuted order
 * within the block), off has nnear+1 entries.  Sizes first with N == NULL. */
dh2_status dh2_near_export(dh2_matrix m, int64_t* off, double* N);

#ifdef __cplusplus
}
#endif

#endif /* DH2_H */
