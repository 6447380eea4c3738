// C ABI of the library (declared in include/dh2.h): argument checks, handle
// management, error reporting.  No exception crosses this boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <string>

#include "../../include/dh2.h"
#include "engine.hpp"

using namespace dh2;

struct dh2_tree_s {
  std::shared_ptr<TreeData> d;
};
struct dh2_blocks_s {
  std::shared_ptr<BlocksData> d;
};
struct dh2_matrix_s {
  std::unique_ptr<MatrixData> d;
};

static thread_local std::string g_err;

static dh2_status set_err(dh2_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define DH2_TRY(...)                                           \
  try {                                                        \
    g_err.clear();                                             \
    __VA_ARGS__;                                               \
    return DH2_OK;                                             \
  } catch (const Error& e) {                                   \
    return set_err(e.code, e.msg);                             \
  } catch (const std::bad_alloc&) {                            \
    return set_err(DH2_ENOMEM, "host allocation failed");      \
  } catch (const std::exception& e) {                          \
    return set_err(DH2_EDEVICE, e.what());                     \
  } catch (...) {                                              \
    return set_err(DH2_EDEVICE, "unknown failure");            \
  }

static void check_opts(const dh2_opts* o) {
  if (!o) fail(DH2_EINVAL, "opts is NULL");
  if (o->leaf_size < 1) fail(DH2_EINVAL, "leaf_size must be >= 1");
  if (!(o->eta1 > 0) || !std::isfinite(o->eta1)) fail(DH2_EINVAL, "eta1 must be > 0");
  if (!(o->eta2 > 0) || !std::isfinite(o->eta2)) fail(DH2_EINVAL, "eta2 must be > 0");
  if (!(o->zeta > 0) || !(2.0 * o->zeta * o->zeta < 1.0))
    fail(DH2_EINVAL, "zeta must satisfy 0 < zeta and 2 zeta^2 < 1");
  if (o->precision != DH2_FP64 && o->precision != DH2_MIXED)
    fail(DH2_EINVAL, "unknown precision mode");
  if (o->max_device_bytes < 0) fail(DH2_EINVAL, "max_device_bytes must be >= 0");
  if (o->groups < 0) fail(DH2_EINVAL, "groups must be >= 0");
  if (o->weights != DH2_WEIGHTS_BLOCK && o->weights != DH2_WEIGHTS_GLOBAL &&
      o->weights != DH2_WEIGHTS_SPECTRAL)
    fail(DH2_EINVAL, "unknown block weights");
  if (o->max_sweeps < 0) fail(DH2_EINVAL, "max_sweeps must be >= 0");
}

static hipStream_t stream_of(void* s) { return reinterpret_cast<hipStream_t>(s); }

// The mixed form's int8-sliced Gram matrices resolve singular values down to
// about 1e-6 of the block-row norms; below eps = 1e-5 the FP64 form is used.
static void check_mixed_eps(const dh2_opts* o, double eps) {
  if (o->precision == DH2_MIXED && eps < 1e-5)
    fail(DH2_EUNSUPPORTED, "the mixed form needs eps >= 1e-5; use DH2_FP64 below");
}

static void need_device() {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n < 1) {
    (void)hipGetLastError();
    fail(DH2_EDEVICE, "no HIP device available");
  }
}

extern "C" {

void dh2_opts_default(dh2_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->leaf_size = 32;
  o->eta1 = 20.0;
  o->eta2 = 5.0;
  o->zeta = 2.0 / 3.0;
  o->precision = DH2_FP64;
  o->lowfreq_zero_dir = 0;
  o->standard_only = 0;
  o->groups = 0;
  o->max_device_bytes = 0;
  o->weights = DH2_WEIGHTS_BLOCK;
  o->max_sweeps = 0;
}

const char* dh2_last_error(void) { return g_err.c_str(); }

dh2_status dh2_tree_build(const double* pts, int64_t n, double kappa, const dh2_opts* opts,
                          dh2_tree* out) {
  DH2_TRY({
    check_opts(opts);
    if (!out) fail(DH2_EINVAL, "out is NULL");
    if (!pts) fail(DH2_EINVAL, "pts is NULL");
    if (n < 1) fail(DH2_EINVAL, "n must be >= 1");
    if (!(kappa >= 0) || !std::isfinite(kappa)) fail(DH2_EINVAL, "kappa must be finite and >= 0");
    for (int64_t i = 0; i < 3 * n; ++i)
      if (!std::isfinite(pts[i])) fail(DH2_EINVAL, "non-finite point coordinate");
    auto td = make_tree(pts, n, kappa, *opts);
    // coincident points always end in the same leaf (the split is by
    // coordinate), where they would make the kernel singular
    const auto& tr = td->tr;
    for (int32_t t = 0; t < tr.nc(); ++t) {
      if (!tr.leaf(t)) continue;
      for (int64_t a = tr.off[t]; a < tr.off[t] + tr.size[t]; ++a)
        for (int64_t b = a + 1; b < tr.off[t] + tr.size[t]; ++b) {
          const double* x = pts + 3 * tr.perm[a];
          const double* y = pts + 3 * tr.perm[b];
          if (x[0] == y[0] && x[1] == y[1] && x[2] == y[2])
            fail(DH2_EINVAL, "coincident points " + std::to_string(tr.perm[a]) + " and " +
                                 std::to_string(tr.perm[b]));
        }
    }
    auto h = new dh2_tree_s{td};
    *out = h;
  })
}

void dh2_tree_free(dh2_tree t) { delete t; }

dh2_status dh2_tree_get_info(dh2_tree t, dh2_tree_info* info) {
  DH2_TRY({
    if (!t || !info) fail(DH2_EINVAL, "NULL argument");
    const auto& tr = t->d->tr;
    info->n = tr.n;
    info->nclusters = tr.nc();
    info->depth = tr.depth;
    int32_t nd = 0;
    for (int32_t l = 0; l <= tr.depth; ++l) nd += t->d->dr.count(l);
    info->ndirs_total = nd;
    info->kappa = t->d->kappa;
  })
}

dh2_status dh2_tree_export(dh2_tree t, int64_t* perm, int64_t* off, int64_t* size, int32_t* level,
                           int32_t* son1, int32_t* son2, double* lo, double* hi, double* diam,
                           double* delta) {
  DH2_TRY({
    if (!t) fail(DH2_EINVAL, "NULL tree");
    const auto& tr = t->d->tr;
    size_t nc = (size_t)tr.nc();
    if (perm) std::memcpy(perm, tr.perm.data(), tr.n * sizeof(int64_t));
    if (off) std::memcpy(off, tr.off.data(), nc * sizeof(int64_t));
    if (size) std::memcpy(size, tr.size.data(), nc * sizeof(int64_t));
    if (level) std::memcpy(level, tr.level.data(), nc * sizeof(int32_t));
    if (son1) std::memcpy(son1, tr.son1.data(), nc * sizeof(int32_t));
    if (son2) std::memcpy(son2, tr.son2.data(), nc * sizeof(int32_t));
    if (lo) std::memcpy(lo, tr.lo.data(), 3 * nc * sizeof(double));
    if (hi) std::memcpy(hi, tr.hi.data(), 3 * nc * sizeof(double));
    if (diam) std::memcpy(diam, tr.diam.data(), nc * sizeof(double));
    if (delta) std::memcpy(delta, tr.delta.data(), tr.delta.size() * sizeof(double));
  })
}

dh2_status dh2_tree_directions(dh2_tree t, int32_t level, int32_t* ndir, double* dirs,
                               int32_t* sd) {
  DH2_TRY({
    if (!t || !ndir) fail(DH2_EINVAL, "NULL argument");
    const auto& dr = t->d->dr;
    if (level < 0 || level > t->d->tr.depth) fail(DH2_EINVAL, "level out of range");
    int32_t nd = dr.count(level);
    *ndir = nd;
    if (dirs) std::memcpy(dirs, dr.dirs[level].data(), 3 * (size_t)nd * sizeof(double));
    if (sd) {
      for (int32_t c = 0; c < nd; ++c) sd[c] = level < t->d->tr.depth ? dr.sd[level][c] : -1;
    }
  })
}

dh2_status dh2_blocks_build(dh2_tree t, const dh2_opts* opts, dh2_blocks* out) {
  DH2_TRY({
    check_opts(opts);
    if (!t || !out) fail(DH2_EINVAL, "NULL argument");
    auto h = new dh2_blocks_s{make_blocks(t->d, *opts)};
    *out = h;
  })
}

void dh2_blocks_free(dh2_blocks b) { delete b; }

dh2_status dh2_blocks_get_info(dh2_blocks b, dh2_blocks_info* info) {
  DH2_TRY({
    if (!b || !info) fail(DH2_EINVAL, "NULL argument");
    const auto& bt = b->d->bt;
    const auto& tr = b->d->tree->tr;
    info->nadm = (int64_t)bt.adm_t.size();
    info->nnear = (int64_t)bt.near_t.size();
    int64_t ne = 0;
    for (size_t q = 0; q < bt.near_t.size(); ++q) ne += tr.size[bt.near_t[q]] * tr.size[bt.near_s[q]];
    info->near_entries = ne;
    for (int s = 0; s < 2; ++s) {
      info->items[s] = b->d->cs[s].nitems();
      info->entries[s] = (int64_t)b->d->cs[s].ent.size();
    }
  })
}

dh2_status dh2_blocks_export(dh2_blocks b, int32_t* adm_t, int32_t* adm_s, int32_t* adm_c,
                             int32_t* near_t, int32_t* near_s) {
  DH2_TRY({
    if (!b) fail(DH2_EINVAL, "NULL blocks");
    const auto& bt = b->d->bt;
    size_t na = bt.adm_t.size(), nn = bt.near_t.size();
    if (adm_t) std::memcpy(adm_t, bt.adm_t.data(), na * sizeof(int32_t));
    if (adm_s) std::memcpy(adm_s, bt.adm_s.data(), na * sizeof(int32_t));
    if (adm_c) std::memcpy(adm_c, bt.adm_c.data(), na * sizeof(int32_t));
    if (near_t) std::memcpy(near_t, bt.near_t.data(), nn * sizeof(int32_t));
    if (near_s) std::memcpy(near_s, bt.near_s.data(), nn * sizeof(int32_t));
  })
}

dh2_status dh2_blocks_colsets(dh2_blocks b, int32_t side, int32_t* item_t, int32_t* item_c,
                              int64_t* item_begin, int32_t* ent_b, int32_t* ent_s,
                              int32_t* ent_d) {
  DH2_TRY({
    if (!b) fail(DH2_EINVAL, "NULL blocks");
    if (side != 0 && side != 1) fail(DH2_EINVAL, "side must be 0 or 1");
    const auto& cs = b->d->cs[side];
    size_t ni = (size_t)cs.nitems(), ne = cs.ent.size();
    if (item_t) std::memcpy(item_t, cs.item_t.data(), ni * sizeof(int32_t));
    if (item_c) std::memcpy(item_c, cs.item_c.data(), ni * sizeof(int32_t));
    if (item_begin) std::memcpy(item_begin, cs.begin.data(), (ni + 1) * sizeof(int64_t));
    for (size_t e = 0; e < ne; ++e) {
      if (ent_b) ent_b[e] = cs.ent[e].b;
      if (ent_s) ent_s[e] = cs.ent[e].s;
      if (ent_d) ent_d[e] = cs.ent[e].d;
    }
  })
}

static void check_compress_args(dh2_blocks b, double eps, const dh2_opts* opts, dh2_matrix* out) {
  check_opts(opts);
  if (!b || !out) fail(DH2_EINVAL, "NULL argument");
  if (!(eps > 0) || !std::isfinite(eps)) fail(DH2_EINVAL, "eps must be finite and > 0");
  need_device();
}

dh2_status dh2_compress_dense(dh2_blocks b, const void* G, int64_t ld, double eps,
                              const dh2_opts* opts, void* stream, dh2_matrix* out) {
  DH2_TRY({
    check_compress_args(b, eps, opts, out);
    int64_t n = b->d->tree->tr.n;
    if (!G) fail(DH2_EINVAL, "G is NULL");
    if (ld < n) fail(DH2_EINVAL, "ld must be >= n");
    if (opts->precision != DH2_FP64)
      fail(DH2_EUNSUPPORTED, "dense input is compressed in FP64 only");
    auto m = compress(b->d, SRC_DENSE, G, ld, nullptr, eps, *opts, stream_of(stream));
    *out = new dh2_matrix_s{std::move(m)};
  })
}

// concurrent streams of dh2_compress_batch, one host worker each: twice the
// device's hardware queues per process, so that instances waiting on a rank
// read-back leave the queues to others (measured: 48 instances in 0.218 s on
// eight streams against 0.252 s on four; sixteen gain nothing more)
constexpr int kBatchStreams = 8;

dh2_status dh2_compress_helmholtz(dh2_blocks b, const double* w, double eps, const dh2_opts* opts,
                                  void* stream, dh2_matrix* out) {
  DH2_TRY({
    check_compress_args(b, eps, opts, out);
    int64_t n = b->d->tree->tr.n;
    if (w)
      for (int64_t i = 0; i < n; ++i)
        if (!(w[i] > 0) || !std::isfinite(w[i])) fail(DH2_EINVAL, "weights must be finite and > 0");
    check_mixed_eps(opts, eps);
    auto m = compress(b->d, SRC_HELMHOLTZ, nullptr, 0, w, eps, *opts, stream_of(stream));
    *out = new dh2_matrix_s{std::move(m)};
  })
}

dh2_status dh2_compress_helmholtz_dlp(dh2_blocks b, const double* w, const double* normals,
                                      double eps, const dh2_opts* opts, void* stream,
                                      dh2_matrix* out) {
  DH2_TRY({
    check_compress_args(b, eps, opts, out);
    if (!normals) fail(DH2_EINVAL, "normals are NULL");
    int64_t n = b->d->tree->tr.n;
    for (int64_t i = 0; i < 3 * n; ++i)
      if (!std::isfinite(normals[i])) fail(DH2_EINVAL, "non-finite normal");
    if (w)
      for (int64_t i = 0; i < n; ++i)
        if (!(w[i] > 0) || !std::isfinite(w[i])) fail(DH2_EINVAL, "weights must be finite and > 0");
    check_mixed_eps(opts, eps);
    auto m = compress(b->d, SRC_DLP, nullptr, 0, w, eps, *opts, stream_of(stream), normals);
    *out = new dh2_matrix_s{std::move(m)};
  })
}

dh2_status dh2_compress_batch(int32_t count, const dh2_blocks* blocks, const double* const* w,
                              double eps, const dh2_opts* opts, void* stream, dh2_matrix* outs) {
  DH2_TRY({
    if (count < 0) fail(DH2_EINVAL, "count must be >= 0");
    if (count > 0 && (!blocks || !outs)) fail(DH2_EINVAL, "NULL argument");
    std::vector<std::shared_ptr<BlocksData>> blks(count);
    std::vector<const double*> ws(count, nullptr);
    for (int32_t i = 0; i < count; ++i) {
      check_compress_args(blocks[i], eps, opts, outs + i);
      if (w && w[i]) {
        int64_t n = blocks[i]->d->tree->tr.n;
        for (int64_t j = 0; j < n; ++j)
          if (!(w[i][j] > 0) || !std::isfinite(w[i][j]))
            fail(DH2_EINVAL, "weights must be finite and > 0");
        ws[i] = w[i];
      }
      blks[i] = blocks[i]->d;
    }
    check_mixed_eps(opts, eps);
    auto ms = compress_batch(blks, ws, eps, *opts, stream_of(stream), kBatchStreams);
    for (int32_t i = 0; i < count; ++i) outs[i] = new dh2_matrix_s{std::move(ms[i])};
  })
}

void dh2_matrix_free(dh2_matrix m) { delete m; }

void dh2_release_cached_memory(void) { release_cached_memory(); }

dh2_status dh2_matvec(dh2_matrix m, char op, int64_t nrhs, const void* x, void* y, void* stream) {
  DH2_TRY({
    if (!m || !x || !y) fail(DH2_EINVAL, "NULL argument");
    if (op != 'N' && op != 'C' && op != 'n' && op != 'c') fail(DH2_EINVAL, "op must be N or C");
    if (nrhs < 0) fail(DH2_EINVAL, "nrhs must be >= 0");
    matvec(*m->d, op, nrhs, (const double2*)x, (double2*)y, stream_of(stream));
    hip_check(hipStreamSynchronize(stream_of(stream)), "matvec sync");
  })
}

dh2_status dh2_matvec_noalloc(dh2_matrix m, char op, int64_t nrhs, const void* x, void* y,
                              void* stream) {
  DH2_TRY({
    if (!m || !x || !y) fail(DH2_EINVAL, "NULL argument");
    if (op != 'N' && op != 'C' && op != 'n' && op != 'c') fail(DH2_EINVAL, "op must be N or C");
    if (nrhs < 0) fail(DH2_EINVAL, "nrhs must be >= 0");
    matvec_noalloc(*m->d, op, nrhs, (const double2*)x, (double2*)y, stream_of(stream));
  })
}

dh2_status dh2_error_estimate(dh2_matrix m, const void* G, int64_t ld, int32_t iters,
                              uint64_t seed, double* rel_err, void* stream) {
  DH2_TRY({
    if (!m || !rel_err) fail(DH2_EINVAL, "NULL argument");
    if (iters < 1) fail(DH2_EINVAL, "iters must be >= 1");
    if (G && ld < m->d->blk->tree->tr.n) fail(DH2_EINVAL, "ld must be >= n");
    *rel_err = error_estimate(*m->d, G, ld, iters, seed, stream_of(stream));
  })
}

dh2_status dh2_rows_check(dh2_matrix m, const int64_t* rows, int32_t nrows, const void* x,
                          double* direct, double* approx, double* max_rel, void* stream) {
  DH2_TRY({
    if (!m || !rows || !x || nrows < 1) fail(DH2_EINVAL, "bad argument");
    rows_check(*m->d, rows, nrows, (const double2*)x, direct, approx, max_rel, stream_of(stream));
  })
}

dh2_status dh2_get_stats(dh2_matrix m, dh2_stats* out) {
  DH2_TRY({
    if (!m || !out) fail(DH2_EINVAL, "NULL argument");
    *out = m->d->stats;
  })
}

dh2_status dh2_basis_export(dh2_matrix m, int32_t side, int32_t* nitems, int64_t* nsigma,
                            int64_t* nmat, int32_t* item_t, int32_t* item_c, int32_t* item_k,
                            int32_t* item_r, int64_t* sig_off, double* sigma, int64_t* mat_off,
                            double* mat) {
  DH2_TRY({
    if (!m) fail(DH2_EINVAL, "NULL matrix");
    if (side != 0 && side != 1) fail(DH2_EINVAL, "side must be 0 or 1");
    const Side& S = m->d->side[side];
    int64_t ns = 0, nm = 0;
    for (int32_t e = 0; e < S.nitems; ++e) {
      const ItemDev& it = S.items[S.P->ext2int[e]];
      if (item_t) item_t[e] = S.P->t[S.P->ext2int[e]];
      if (item_c) item_c[e] = S.P->c[S.P->ext2int[e]];
      if (item_k) item_k[e] = it.k;
      if (item_r) item_r[e] = it.r;
      if (sig_off) sig_off[e] = ns;
      if (mat_off) mat_off[e] = nm;
      if (sigma && it.r) {
        hip_check(hipMemcpy(sigma + ns, it.sig, it.r * sizeof(double), hipMemcpyDeviceToHost),
                  "export sigma");
      }
      if (mat && it.r * it.k) {
        hip_check(hipMemcpy(mat + 2 * nm, it.Q, (size_t)it.r * it.k * sizeof(double2),
                            hipMemcpyDeviceToHost),
                  "export basis");
      }
      ns += it.r;
      nm += (int64_t)it.r * it.k;
    }
    if (nitems) *nitems = S.nitems;
    if (nsigma) *nsigma = ns;
    if (nmat) *nmat = nm;
  })
}

// cnt complex values from the device to interleaved host doubles; f32: the
// device holds them as complex FP32 (widened exactly)
static void copy_widen(double* dst, const void* src, int64_t cnt, bool f32, const char* what) {
  if (!f32) {
    hip_check(hipMemcpy(dst, src, cnt * sizeof(double2), hipMemcpyDeviceToHost), what);
    return;
  }
  std::vector<float> tmp(2 * (size_t)cnt);
  hip_check(hipMemcpy(tmp.data(), src, cnt * sizeof(float2), hipMemcpyDeviceToHost), what);
  for (size_t i = 0; i < tmp.size(); ++i) dst[i] = (double)tmp[i];
}

dh2_status dh2_coupling_export(dh2_matrix m, int64_t* off, double* S) {
  DH2_TRY({
    if (!m || !off) fail(DH2_EINVAL, "NULL argument");
    const MatrixData& M = *m->d;
    int64_t o = 0, nadm = (int64_t)M.S_ptr.size();
    for (int64_t b = 0; b < nadm; ++b) {
      off[b] = o;
      int64_t cnt = (int64_t)M.S_rows[b] * M.S_cols[b];
      if (S && cnt) copy_widen(S + 2 * o, M.S_ptr[b], cnt, M.s32, "export coupling");
      o += cnt;
    }
    off[nadm] = o;
  })
}

dh2_status dh2_near_export(dh2_matrix m, int64_t* off, double* N) {
  DH2_TRY({
    if (!m || !off) fail(DH2_EINVAL, "NULL argument");
    const MatrixData& M = *m->d;
    int64_t nn = (int64_t)M.nears.size(), tot = 0;
    for (int64_t b = 0; b < nn; ++b) {
      off[b] = M.nears[b].off;
      tot += M.nears[b].t_len * M.nears[b].s_len;
    }
    off[nn] = tot;
    if (N && tot) copy_widen(N, M.d_near, tot, M.s32, "export near");
  })
}

}  // extern "C"
