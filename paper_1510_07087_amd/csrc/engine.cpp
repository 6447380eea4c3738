// Host engine of the directional H2 compression (see engine.hpp).
//
// Compression (Section 6 of the paper): for each basis, the (cluster,
// direction) block rows are processed level by level from the leaves up.
// Per level: Gram matrices of the weighted block rows (leaf clusters:
// entries generated from the points; other clusters: zeta [R_t1c'; R_t2c']
// read from the sons' coefficient matrices), factorisation into singular
// values and left singular vectors, rank read-back, then R_tc = Q^* A.  The
// column basis (rows of G^*) and the row basis are independent and are built
// at the same time on two streams; the column basis is expanded level by
// level, the row sweep keeps the own-block columns of every R_tc, and after
// both every admissible block is projected: S_b = omega_b R_tc|s W_sc =
// V^* G|_b W.  Subtrees rooted above the first level with admissible blocks
// are independent and are swept in batches to bound the memory of the R
// matrices (the paper parallelises over independent subtrees in the same
// way).
#include "engine.hpp"

#include <algorithm>
#include <atomic>
#include <thread>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <condition_variable>
#include <mutex>
#include <numeric>
#include <random>
#include <unordered_map>

#include "kernels.hpp"

namespace dh2 {

void fail(dh2_status code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(e == hipErrorOutOfMemory ? DH2_ENOMEM : DH2_EDEVICE,
         std::string(what) + ": " + hipGetErrorString(e));
  }
}

static void launch_check(const char* what) { hip_check(hipGetLastError(), what); }

// Optional host-side phase tracing (environment DH2_TRACE=1), to stderr.
static bool trace_on() {
  static int on = -1;
  if (on < 0) {
    const char* e = std::getenv("DH2_TRACE");
    on = (e && e[0] == '1') ? 1 : 0;
  }
  return on == 1;
}
struct Trace {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  std::chrono::steady_clock::time_point last = t0;
  void mark(const char* what, int side, int b, int lv) {
    if (!trace_on()) return;
    auto now = std::chrono::steady_clock::now();
    double d = std::chrono::duration<double, std::milli>(now - last).count();
    double tot = std::chrono::duration<double, std::milli>(now - t0).count();
    std::fprintf(stderr, "[dh2 trace] side %d batch %d level %d %-14s %9.2f ms (t=%9.1f)\n", side, b,
                 lv, what, d, tot);
    last = now;
  }
};

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------
// Freed device blocks are kept in a process-wide cache and handed out again
// for requests of a similar size: returning touched memory to the driver is
// expensive (hundreds of milliseconds for tens of gigabytes), and the sweep
// allocates and frees one arena of coefficient matrices per level.
namespace {
struct CachedBlock {
  void* p;
  size_t bytes;
};
std::mutex g_cache_mu;
std::vector<CachedBlock> g_cache;
size_t g_cached = 0;
// serialises the check of the driver's free memory with the allocation that
// follows it, so that two sweeps allocating at once cannot both pass it
std::mutex g_alloc_mu;

size_t size_class(size_t b) {
  if (b < 4096) return (b + 255) & ~size_t(255);
  size_t top = size_t(1) << (63 - __builtin_clzll((unsigned long long)b));
  size_t gran = top / 16;  // at most 6.25 % rounding
  return (b + gran - 1) / gran * gran;
}

size_t cache_limit() {
  static size_t lim = 0;
  if (lim == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      tot = size_t(64) << 30;
    }
    lim = tot / 10 * 8;
  }
  return lim;
}

size_t g_cache_largest_locked() {
  size_t big = 0;
  for (const auto& c : g_cache) big = std::max(big, c.bytes);
  return big;
}

void trim_cache_locked(size_t keep) {
  while (g_cached > keep && !g_cache.empty()) {
    size_t big = 0;
    for (size_t i = 1; i < g_cache.size(); ++i)
      if (g_cache[i].bytes > g_cache[big].bytes) big = i;
    (void)hipFree(g_cache[big].p);
    g_cached -= g_cache[big].bytes;
    g_cache[big] = g_cache.back();
    g_cache.pop_back();
  }
}
}  // namespace

// pinned staging buffers, reused across compressions (a buffer in the pool
// has no transfer in flight)
constexpr size_t kPinBytes = size_t(32) << 20;
static std::mutex g_pin_mu;
static std::vector<char*> g_pin_pool;

void release_cached_memory() {
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    trim_cache_locked(0);
  }
  std::lock_guard<std::mutex> lk(g_pin_mu);
  for (char* p : g_pin_pool) (void)hipHostFree(p);
  g_pin_pool.clear();
}

DevMem::~DevMem() {
  // an error may have left work queued that still uses released blocks or
  // the staging buffer
  if (pin_ || !released_.empty()) (void)hipDeviceSynchronize();
  if (pin_) {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    g_pin_pool.push_back(pin_);
    pin_ = nullptr;
  }
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto& pr : live_) {
    g_cache.push_back({pr.first, pr.second});
    g_cached += pr.second;
  }
  live_.clear();
  for (auto& pr : released_) {
    g_cache.push_back({pr.first, pr.second});
    g_cached += pr.second;
  }
  released_.clear();
  trim_cache_locked(cache_limit());
}

void DevMem::flush_released() {
  if (released_.empty()) return;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto& pr : released_) {
    g_cache.push_back({pr.first, pr.second});
    g_cached += pr.second;
  }
  released_.clear();
  trim_cache_locked(cache_limit());
}

void DevMem::sync(hipStream_t st, const char* what) {
  hip_check(hipStreamSynchronize(st), what);
  pin_off_ = 0;
  flush_released();
}

void DevMem::upload(void* d, const void* h, size_t bytes, hipStream_t st) {
  if (bytes == 0) return;
  const size_t need = (bytes + 255) & ~size_t(255);
  if (!pin_ || need > kPinBytes) {
    hip_check(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st), "upload");
    sync(st, "upload sync");
    return;
  }
  if (pin_off_ + need > kPinBytes) sync(st, "staging sync");  // earlier transfers done
  std::memcpy(pin_ + pin_off_, h, bytes);
  hip_check(hipMemcpyAsync(d, pin_ + pin_off_, bytes, hipMemcpyHostToDevice, st), "upload");
  pin_off_ += need;
}

void DevMem::begin_staging() {
  if (pin_) return;
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    if (!g_pin_pool.empty()) {
      pin_ = g_pin_pool.back();
      g_pin_pool.pop_back();
    }
  }
  if (!pin_) hip_check(hipHostMalloc((void**)&pin_, kPinBytes, hipHostMallocDefault), "hipHostMalloc");
  pin_off_ = 0;
}

void DevMem::end_staging(hipStream_t st) {
  sync(st, "staging end");
  if (!pin_) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_pool.push_back(pin_);
  pin_ = nullptr;
}

void* DevMem::alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = size_class(bytes);
  if (cap_ > 0 && used_ + (int64_t)bytes > cap_)
    fail(DH2_ENOMEM, "device memory cap exceeded (" + std::to_string(used_ + bytes) + " > " +
                         std::to_string(cap_) + " bytes)");
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    size_t best = g_cache.size();
    for (size_t i = 0; i < g_cache.size(); ++i) {
      size_t cb = g_cache[i].bytes;
      if (cb >= bytes && cb <= bytes + bytes / 4 &&
          (best == g_cache.size() || cb < g_cache[best].bytes))
        best = i;
    }
    if (best < g_cache.size()) {
      p = g_cache[best].p;
      bytes = g_cache[best].bytes;
      g_cached -= bytes;
      g_cache[best] = g_cache.back();
      g_cache.pop_back();
    }
  }
  if (!p) {
    // keep cached blocks from pushing the device past its memory: the driver
    // would evict allocations to host memory instead of failing
    const size_t margin = size_t(2) << 30;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      fr = ~size_t(0) >> 1;
    }
    if (fr < bytes + margin && !released_.empty()) {
      hip_check(hipDeviceSynchronize(), "release sync");
      pin_off_ = 0;
      flush_released();
    }
    hipError_t e;
    {
      // the free-memory check and the allocation that relies on it, under
      // one lock, so that two sweeps allocating at once cannot both pass it
      std::lock_guard<std::mutex> alk(g_alloc_mu);
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        fr = ~size_t(0) >> 1;
      }
      {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        while (fr < bytes + margin && !g_cache.empty()) {
          size_t big = g_cache_largest_locked();
          trim_cache_locked(g_cached - std::min(g_cached, big));
          fr += big;
        }
      }
      e = hipMalloc(&p, bytes);
    }
    while (e != hipSuccess) {
      (void)hipGetLastError();
      // blocks released since the last sync: wait for the device, then they
      // are free for anyone
      if (!released_.empty()) {
        hip_check(hipDeviceSynchronize(), "release sync");
        pin_off_ = 0;
        flush_released();
      }
      // no room: take the smallest cached block that is large enough, however
      // large, else return the largest cached block to the driver and retry
      // (freeing the whole cache would make every later level allocate from
      // scratch)
      bool freed = false;
      {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        size_t best = g_cache.size();
        for (size_t i = 0; i < g_cache.size(); ++i)
          if (g_cache[i].bytes >= bytes && (cap_ <= 0 || used_ + (int64_t)g_cache[i].bytes <= cap_) &&
              (best == g_cache.size() || g_cache[i].bytes < g_cache[best].bytes))
            best = i;
        if (best < g_cache.size()) {
          p = g_cache[best].p;
          bytes = g_cache[best].bytes;
          g_cached -= bytes;
          g_cache[best] = g_cache.back();
          g_cache.pop_back();
          break;
        }
        if (!g_cache.empty()) {
          trim_cache_locked(g_cached - std::min(g_cached, g_cache_largest_locked()));
          freed = true;
        }
      }
      if (!freed) fail(DH2_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
      e = hipMalloc(&p, bytes);
    }
  }
  live_.push_back({p, bytes});
  used_ += (int64_t)bytes;
  peak_ = std::max(peak_, used_);
  return p;
}

void DevMem::release(void* p) {
  if (!p) return;
  for (size_t i = live_.size(); i-- > 0;) {
    if (live_[i].first == p) {
      released_.push_back(live_[i]);
      used_ -= (int64_t)live_[i].second;
      live_[i] = live_.back();
      live_.pop_back();
      return;
    }
  }
}

template <class T>
static T* upload(DevMem& mem, const std::vector<T>& v, hipStream_t st) {
  T* d = (T*)mem.alloc(v.size() * sizeof(T));
  mem.upload(d, v.data(), v.size() * sizeof(T), st);
  return d;
}

template <class T>
static void copy_to(DevMem& mem, T* d, const T* h, size_t n, hipStream_t st) {
  mem.upload(d, h, n * sizeof(T), st);
}

template <class T>
static void copy_from(T* h, const T* d, size_t n, hipStream_t st) {
  if (n == 0) return;
  hip_check(hipMemcpyAsync(h, d, n * sizeof(T), hipMemcpyDeviceToHost, st), "copy_from");
  hip_check(hipStreamSynchronize(st), "copy_from sync");
}

// ---------------------------------------------------------------------------
// plan handles
// ---------------------------------------------------------------------------
std::shared_ptr<TreeData> make_tree(const double* pts, int64_t n, double kappa, const dh2_opts& o) {
  auto t = std::make_shared<TreeData>();
  t->pts.assign(pts, pts + 3 * n);
  t->kappa = kappa;
  t->opts = o;
  t->tr = build_cluster_tree(pts, n, o.leaf_size);
  t->dr = build_directions(t->tr, kappa, o.eta1, o.lowfreq_zero_dir != 0);
  return t;
}

std::shared_ptr<BlocksData> make_blocks(std::shared_ptr<TreeData> t, const dh2_opts& o) {
  auto b = std::make_shared<BlocksData>();
  b->tree = t;
  b->opts = o;
  b->bt = build_block_tree(t->tr, t->dr, t->kappa, o.eta2, o.standard_only != 0);
  b->cs[0] = build_column_sets(t->tr, t->dr, b->bt, 0);
  b->cs[1] = build_column_sets(t->tr, t->dr, b->bt, 1);
  return b;
}

// ---------------------------------------------------------------------------
// matvec plan (built on first use)
// ---------------------------------------------------------------------------
struct SideMV {
  int64_t* d_hoff = nullptr;       // coefficient offsets per item
  int64_t total = 0;
  // coupling: for op N on side 0 / op C on side 1 (this side receives)
  int64_t* d_cbegin = nullptr;
  int32_t* d_cblock = nullptr;
  int32_t* d_cpartner = nullptr;
  int32_t* d_corder = nullptr;  // items by descending coupling work (launch order)
  int32_t nheavy = 0;           // the first nheavy of them: one workgroup each
  // backward: per level, items with fathers
  std::vector<int32_t*> d_bl_items;
  std::vector<int32_t> bl_count;
  std::vector<int64_t*> d_bl_fbegin;
  std::vector<int32_t*> d_bl_fitem;
  std::vector<int32_t*> d_bl_fson;
  // forward: leaf items, then non-leaf items per level (deepest first)
  int32_t* d_fwd_leaf = nullptr;
  int32_t n_fwd_leaf = 0;
  std::vector<int32_t*> d_fwd_lvl;
  std::vector<int32_t> fwd_count;
  // tasks of the last step (leaves, or parts of a leaf's near field)
  LeafDev* d_leaves = nullptr;
  NearRefDev* d_nref = nullptr;
  int32_t nleaves = 0;
  // leaves whose work is split over several tasks, and the partial slots
  LeafDev* d_split = nullptr;
  int32_t nsplit = 0;
  int32_t nslots = 0;
  // basis terms of every leaf (added to the near-field rows afterwards)
  LeafDev* d_basis = nullptr;
  int32_t nbasis = 0;
};

struct MatvecPlan {
  SideMV s[2];
  NearDev* d_nears = nullptr;
  void* const* d_Sptr = nullptr;
  int32_t* d_Srows = nullptr;
  int32_t* d_Scols = nullptr;
  void* const* d_STptr = nullptr;  // transposed copies S_b^T for the adjoint
  double2* xp = nullptr;
  double2* yp = nullptr;
  double2* xh = nullptr;  // sized for the larger side
  double2* yh = nullptr;
  double2* part = nullptr;  // partial sums of split leaves (64 rows x kMvRhs per slot)
  int64_t maxh = 0;       // coefficients of the larger side
  int32_t maxslots = 0;   // partial slots of the larger side
  void* d_nearT = nullptr;  // near-field blocks transposed (#s x #t column-major)
  // the near-field rows run on a second stream beside the basis chain
  hipStream_t side = nullptr;
  hipEvent_t ev_x = nullptr, ev_near = nullptr;
  ~MatvecPlan() {
    if (side) {
      (void)hipStreamSynchronize(side);
      (void)hipStreamDestroy(side);
    }
    if (ev_x) (void)hipEventDestroy(ev_x);
    if (ev_near) (void)hipEventDestroy(ev_near);
  }
};

// right-hand sides per pass of the matrix-vector product kernels
constexpr int kMvRhs = 8;

// work vectors of one pass: permuted x and y (n each), coefficients of the
// source and destination bases (maxh each), times the right-hand sides of
// the pass (interleaved)
struct MatvecBufs {
  double2 *xp, *yp, *xh, *yh, *part;
};

MatrixData::~MatrixData() {
  mv.reset();
  mem_col.reset();
  mem.reset();
}

// ---------------------------------------------------------------------------
// side construction
// ---------------------------------------------------------------------------
static int32_t first_adm_level(const BlocksData& B) {
  int32_t l = 1 << 30;
  for (int32_t t : B.bt.adm_t) l = std::min(l, B.tree->tr.level[t]);
  return l;
}

static std::shared_ptr<SidePlan> build_side_plan(const BlocksData& B, int s, int32_t nb,
                                                 const std::vector<int32_t>& batch_of_cluster) {
  auto SP = std::make_shared<SidePlan>();
  SidePlan& S = *SP;
  const ClusterTree& tr = B.tree->tr;
  const Directions& dr = B.tree->dr;
  const ColumnSets& cs = B.cs[s];
  int32_t ni = cs.nitems();
  S.nitems = ni;
  // internal order: (batch, level descending, external index)
  std::vector<int32_t> order(ni);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    int32_t ta = cs.item_t[a], tb = cs.item_t[b];
    int32_t ba = batch_of_cluster[ta], bb = batch_of_cluster[tb];
    if (ba != bb) return ba < bb;
    if (tr.level[ta] != tr.level[tb]) return tr.level[ta] > tr.level[tb];
    return a < b;
  });
  S.int2ext = order;
  S.ext2int.assign(ni, -1);
  for (int32_t i = 0; i < ni; ++i) S.ext2int[order[i]] = i;
  S.items0.assign(ni, ItemDev{});
  S.t.resize(ni);
  S.c.resize(ni);
  S.ninh.resize(ni);
  S.ent_col.assign(cs.ent.size(), 0);
  // per external item: N and entry column starts
  std::vector<int64_t> Next(ni, 0), Ninh(ni, 0);
  for (int32_t e = 0; e < ni; ++e) {
    int64_t col = 0;
    bool own = false;
    for (int64_t q = cs.begin[e]; q < cs.begin[e + 1]; ++q) {
      S.ent_col[q] = col;
      col += tr.size[cs.ent[q].s];
      // inherited entries come first, the item's own blocks last
      if (cs.ent[q].d == 0) own = true;
      else if (own) fail(DH2_EDEVICE, "internal: column set out of order");
      else Ninh[e] = col;
    }
    Next[e] = col;
  }
  // column offsets of F_tc inside the sons' sets
  std::vector<int64_t> coloff(ni, 0);
  for (int32_t t = 0; t < tr.nc(); ++t) {
    if (tr.leaf(t) || cs.count[t] == 0) continue;
    std::map<int32_t, int64_t> run;
    const auto& sdl = dr.sd[tr.level[t]];
    for (int32_t e = cs.first[t]; e < cs.first[t] + cs.count[t]; ++e) {
      int32_t cp = sdl[cs.item_c[e]];
      coloff[e] = run[cp];
      run[cp] += Next[e];
    }
  }
  S.ents.clear();
  {
    size_t nent = 0;
    for (int32_t e = 0; e < ni; ++e)
      if (tr.leaf(cs.item_t[e])) nent += (size_t)(cs.begin[e + 1] - cs.begin[e]);
    S.ents.reserve(nent);
  }
  std::vector<int32_t> son_ext(2 * (size_t)ni, -1);
  S.range.assign(nb, std::vector<std::pair<int32_t, int32_t>>(tr.depth + 1, {0, 0}));
  for (int32_t i = 0; i < ni; ++i) {
    int32_t e = order[i];
    int32_t t = cs.item_t[e], c = cs.item_c[e];
    ItemDev& it = S.items0[i];
    S.t[i] = t;
    S.c[i] = c;
    S.ninh[i] = Ninh[e];
    it.ninh = Ninh[e];
    it.Rown = nullptr;
    it.row_off = tr.off[t];
    it.N = Next[e];
    it.m = (int32_t)tr.size[t];
    it.leaf = tr.leaf(t) ? 1 : 0;
    it.level = tr.level[t];
    it.k = 0;
    it.son[0] = it.son[1] = -1;
    it.col_off = coloff[e];
    if (it.leaf) {
      it.r = it.m;
      it.ent_begin = (int64_t)S.ents.size();
      for (int64_t q = cs.begin[e]; q < cs.begin[e + 1]; ++q) {
        const ColEntry& ce = cs.ent[q];
        EntDev ed{};
        ed.col_start = S.ent_col[q];
        ed.pos = tr.off[ce.s];
        ed.len = tr.size[ce.s];
        ed.b = ce.b;
        ed.d = ce.d;
        ed.scale = 0.0;
        ed.s = ce.s;
        S.ents.push_back(ed);
      }
      it.ent_end = (int64_t)S.ents.size();
    } else {
      int32_t cp = dr.sd[tr.level[t]][c];
      for (int q = 0; q < 2; ++q) {
        int32_t son = q == 0 ? tr.son1[t] : tr.son2[t];
        int32_t se = cs.find(son, cp);
        if (se < 0) fail(DH2_EDEVICE, "internal: son item missing");
        son_ext[2 * (size_t)i + q] = se;
      }
      it.r = 0;
    }
    int32_t b = batch_of_cluster[t];
    auto& rg = S.range[b][it.level];
    if (rg.first == rg.second) rg = {i, i + 1};
    else rg.second = i + 1;
  }
  for (int32_t i = 0; i < ni; ++i)
    if (!S.items0[i].leaf)
      for (int q = 0; q < 2; ++q) {
        int32_t so = S.ext2int[son_ext[2 * (size_t)i + q]];
        S.items0[i].son[q] = so;
        // the kernels read columns col_off .. col_off+N of the son's R, all
        // of them inherited ones
        if (S.items0[i].col_off + S.items0[i].N > S.ninh[so] ||
            S.items0[so].level != S.items0[i].level + 1)
          fail(DH2_EDEVICE, "internal: inconsistent column sets");
      }
  return SP;
}

// Projection tasks of the row sweep per (batch, level), sorted by column item.
static std::vector<std::vector<ProjPlan>> build_proj_plan(const BlocksData& B, const SidePlan& R,
                                                          const SidePlan& C, int32_t nb) {
  const ClusterTree& tr = B.tree->tr;
  const ColumnSets& cs = B.cs[0];
  std::vector<std::vector<ProjPlan>> out((size_t)nb * (tr.depth + 1));
  for (int32_t b = 0; b < nb; ++b)
    for (int32_t lv = 0; lv <= tr.depth; ++lv) {
      auto [lo, hi] = R.range[b][lv];
      auto& v = out[(size_t)b * (tr.depth + 1) + lv];
      for (int32_t i = lo; i < hi; ++i) {
        int32_t e = R.int2ext[i];
        for (int64_t q = cs.begin[e]; q < cs.begin[e + 1]; ++q) {
          const ColEntry& ce = cs.ent[q];
          if (ce.d != 0) continue;
          int32_t we = B.cs[1].find(ce.s, R.c[i]);
          if (we < 0) fail(DH2_EDEVICE, "internal: column item missing");
          v.push_back(ProjPlan{i, C.ext2int[we], ce.b, (int32_t)tr.size[ce.s], R.ent_col[q]});
        }
      }
      std::stable_sort(v.begin(), v.end(),
                       [](const ProjPlan& x, const ProjPlan& y) { return x.witem < y.witem; });
    }
  return out;
}

PlanCache::~PlanCache() {
  for (int s = 0; s < 2; ++s)
    if (d_ents[s]) (void)hipFree(d_ents[s]);
  if (d_adm) (void)hipFree(d_adm);
}

// The plan cache of a block tree for nb batches (built on first use).
static std::shared_ptr<PlanCache> plan_cache(const BlocksData& B, int32_t nb,
                                             const std::vector<int32_t>& batch_of) {
  std::lock_guard<std::mutex> lk(B.cache_mu);
  if (B.cache && B.cache->nbatch == nb) return B.cache;
  auto C = std::make_shared<PlanCache>();
  C->nbatch = nb;
  auto s0 = build_side_plan(B, 0, nb, batch_of);
  auto s1 = build_side_plan(B, 1, nb, batch_of);
  C->proj = build_proj_plan(B, *s0, *s1, nb);
  C->side[0] = s0;
  C->side[1] = s1;
  for (int s = 0; s < 2; ++s) {
    const auto& ents = C->side[s]->ents;
    if (ents.empty()) continue;
    hip_check(hipMalloc(&C->d_ents[s], ents.size() * sizeof(EntDev)), "hipMalloc (plan)");
    hip_check(hipMemcpy(C->d_ents[s], ents.data(), ents.size() * sizeof(EntDev),
                        hipMemcpyHostToDevice),
              "upload (plan)");
  }
  {
    const ClusterTree& tr = B.tree->tr;
    int64_t nadm = (int64_t)B.bt.adm_t.size();
    std::vector<int64_t> adm(4 * (size_t)std::max<int64_t>(1, nadm), 0);
    for (int64_t b = 0; b < nadm; ++b) {
      adm[b] = tr.off[B.bt.adm_t[b]];
      adm[nadm + b] = tr.size[B.bt.adm_t[b]];
      adm[2 * nadm + b] = tr.off[B.bt.adm_s[b]];
      adm[3 * nadm + b] = tr.size[B.bt.adm_s[b]];
    }
    hip_check(hipMalloc(&C->d_adm, adm.size() * sizeof(int64_t)), "hipMalloc (plan)");
    hip_check(hipMemcpy(C->d_adm, adm.data(), adm.size() * sizeof(int64_t), hipMemcpyHostToDevice),
              "upload (plan)");
  }
  B.cache = C;
  return C;
}


// ---------------------------------------------------------------------------
// compression
// ---------------------------------------------------------------------------
// Event-timed phases: each start/stop records an event on the stream; the
// times are read once, after the last stop has completed, so that timing
// adds no wait to the sweep.
struct PhaseTimer {
  hipStream_t st;
  std::vector<hipEvent_t> ev;  // start, stop, start, stop, ...
  explicit PhaseTimer(hipStream_t s) : st(s) {}
  ~PhaseTimer() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  void record() {
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "event");
    ev.push_back(e);
    hip_check(hipEventRecord(e, st), "event record");
  }
  void start() { record(); }
  void stop() { record(); }
  double total() {
    double acc = 0;
    if (ev.empty()) return acc;
    hip_check(hipEventSynchronize(ev.back()), "event sync");
    for (size_t i = 0; i + 1 < ev.size(); i += 2) {
      float ms = 0;
      hip_check(hipEventElapsedTime(&ms, ev[i], ev[i + 1]), "event time");
      acc += ms * 1e-3;
    }
    return acc;
  }
};

struct SweepStats {
  double flops_gram = 0, flops_rprod = 0, flops_prj = 0;
  double t_gram = 0, t_prj = 0;
  double flops_gram_leaf = 0, t_gram_leaf = 0, flops_rprod_leaf = 0, ops_gram_leaf_i8 = 0;
  int32_t n_gram_leaf = 0;
  int64_t n_fac[5] = {0, 0, 0, 0, 0};  // factorisations by size class (last: X in memory)
  int64_t n_redo = 0;                  // factored again (wide LDS pass)
  int64_t n_redo_mem = 0;              // factored a third time with X in memory
};

static void expand_level(MatrixData& M, int s, int32_t lv, hipStream_t st, DevMem& mem);

static void sweep(MatrixData& M, int s, const GeomDev& g, hipStream_t st, SweepStats& ss,
                  int32_t* d_status, DevMem& mem) {
  const BlocksData& B = *M.blk;
  const ClusterTree& tr = B.tree->tr;
  Side& S = M.side[s];
  PhaseTimer tg(st), tgl(st);
  double2* partial = nullptr;
  size_t partial_cap = 0;
  const bool mixed = M.precision == DH2_MIXED;

  Trace tr_;
  for (int32_t b = 0; b < M.nbatch; ++b) {
    void* R_prev = nullptr;
    for (int32_t lv = tr.depth; lv >= 0; --lv) {
      auto [lo, hi] = S.P->range[b][lv];
      if (lo == hi) continue;
      int32_t n = hi - lo;
      tr_.mark("level start", s, b, lv);
      // factor sizes of non-leaf items from the sons' ranks
      int64_t sum_r2 = 0, sum_r = 0;
      for (int32_t i = lo; i < hi; ++i) {
        ItemDev& it = S.items[i];
        if (!it.leaf) it.r = S.items[it.son[0]].k + S.items[it.son[1]].k;
        if (it.r > kMaxRBig)
          fail(DH2_EUNSUPPORTED, "block row with " + std::to_string(it.r) +
                                     " factor rows exceeds the kernel limit " +
                                     std::to_string(kMaxRBig));
        sum_r2 += (int64_t)it.r * it.r;
        sum_r += it.r;
      }
      // column data of the leaf block rows of this level (read by the Gram and
      // R-product kernels)
      std::vector<int32_t> leaf_ids;
      int64_t sum_leafN = 0;
      for (int32_t i = lo; i < hi; ++i)
        if (S.items[i].leaf && S.items[i].N > 0) {
          leaf_ids.push_back(i);
          sum_leafN += S.items[i].N;
        }
      // mixed double layer: positions and factors, then the N column normals
      const int64_t cmul = mixed && M.src == SRC_DLP ? 2 : 1;
      double4* colbuf =
          sum_leafN ? (double4*)mem.alloc(cmul * sum_leafN * sizeof(double4)) : nullptr;
      {
        int64_t o = 0;
        for (int32_t i = lo; i < hi; ++i) {
          S.items[i].cols = nullptr;
          if (S.items[i].leaf && S.items[i].N > 0) {
            S.items[i].cols = colbuf + o;
            o += cmul * S.items[i].N;
          }
        }
      }
      double2* Marena = (double2*)mem.alloc(sum_r2 * sizeof(double2));
      double2* Qarena = (double2*)mem.alloc(sum_r2 * sizeof(double2));
      double* sarena = (double*)mem.alloc(sum_r * sizeof(double));
      S.keep.push_back(Qarena);
      S.keep.push_back(sarena);
      {
        int64_t o2 = 0, o1 = 0;
        for (int32_t i = lo; i < hi; ++i) {
          ItemDev& it = S.items[i];
          it.M = Marena + o2;
          it.Q = Qarena + o2;
          it.sig = sarena + o1;
          o2 += (int64_t)it.r * it.r;
          o1 += it.r;
        }
      }
      copy_to(mem, S.d_items + lo, S.items.data() + lo, n, st);
      int32_t* d_leaf_ids = upload(mem, leaf_ids, st);
      launch_leaf_cols(M.src, g, S.d_items, d_leaf_ids, (int32_t)leaf_ids.size(), S.d_ents, s,
                       mixed, st);
      launch_check("leaf columns");
      tr_.mark("arenas", s, b, lv);
      // Gram units: leaf items first, then non-leaf items
      int64_t totalN = 0;
      for (int32_t i = lo; i < hi; ++i) totalN += S.items[i].N;
      // FP64: one Gram unit per wave, about 8 waves of work per SIMD; mixed:
      // one unit per workgroup of 16 waves (int8 slicing, 64-column chunks)
      int64_t width = mixed ? std::max<int64_t>(512, std::min<int64_t>(8192, totalN / 1024))
                            : std::max<int64_t>(256, std::min<int64_t>(2048, totalN / 8192));
      width = (width + 63) / 64 * 64;
      std::vector<UnitDev> units;
      std::vector<int32_t> litems, ubegin;
      int64_t slot = 0, nleafu = 0;
      for (int pass = 0; pass < 2; ++pass) {
        for (int32_t i = lo; i < hi; ++i) {
          const ItemDev& it = S.items[i];
          if ((pass == 0) != (it.leaf != 0)) continue;
          litems.push_back(i);
          ubegin.push_back((int32_t)units.size());
          if (it.r == 0) continue;
          if (it.leaf && it.m > 64)
            fail(DH2_EUNSUPPORTED, "leaf clusters with more than 64 points are not supported");
          // tile blocks per unit (register budget: at most 10 tile pairs per
          // wave): the 16-row tiles in groups of four; a diagonal block per
          // group and every pair of groups in bands of two row tiles against
          // the column group's (up to) four tiles
          int nt = (it.r + 15) / 16;
          std::vector<std::array<int, 4>> blocksets;
          for (int g0 = 0; g0 < nt; g0 += 4) {
            int gn = std::min(4, nt - g0);
            blocksets.push_back({g0, gn, g0, gn});
            for (int h0 = 0; h0 < g0; h0 += 4)
              for (int a0 = g0; a0 < g0 + gn; a0 += 2)
                blocksets.push_back({a0, std::min(2, g0 + gn - a0), h0, 4});
          }
          for (int64_t c0 = 0; c0 < it.N; c0 += width) {
            for (const auto& bs : blocksets) {
              UnitDev u{};
              u.item = i;
              u.col_begin = c0;
              u.ncols = std::min(width, it.N - c0);
              u.a0 = (int8_t)bs[0];
              u.na = (int8_t)bs[1];
              u.b0 = (int8_t)bs[2];
              u.nb = (int8_t)bs[3];
              int npair = bs[0] == bs[2] ? bs[1] * (bs[1] + 1) / 2 : bs[1] * bs[3];
              u.slot_off = slot;
              slot += (int64_t)npair * 256;
              units.push_back(u);
            }
            // the reduction's algorithmic work, 8 r^2 N real flops per block row
            // (a Householder reduction of the N x r block row; the Gram matrix
            // computes its Hermitian half, 4 r^2 N)
            double rr = it.r;
            double fl = 8.0 * rr * rr * (double)std::min(width, it.N - c0);
            ss.flops_gram += fl;
            if (it.leaf) ss.flops_gram_leaf += fl;
            // int8 slicing: 4 real products x 15 slice pairs x 2 ops on the lower triangle
            if (it.leaf && mixed) ss.ops_gram_leaf_i8 += 60.0 * rr * (rr + 1.0) * (double)std::min(width, it.N - c0);
          }
        }
        if (pass == 0) nleafu = (int64_t)units.size();
      }
      ubegin.push_back((int32_t)units.size());
      if ((size_t)slot * sizeof(double2) > partial_cap) {
        mem.release(partial);
        partial_cap = std::max<size_t>((size_t)slot * sizeof(double2), partial_cap * 3 / 2);
        partial = (double2*)mem.alloc(partial_cap);
      }
      UnitDev* d_units = upload(mem, units, st);
      int32_t* d_litems = upload(mem, litems, st);
      int32_t* d_ubegin = upload(mem, ubegin, st);
      tr_.mark("gram units", s, b, lv);
      tg.start();
      const bool i8 = mixed && (M.src == SRC_HELMHOLTZ || M.src == SRC_DLP);
      if (nleafu > 0) {
        tgl.start();
        if (i8)
          launch_gram_i8(false, g, S.d_items, S.d_ents, d_units, nleafu, M.zeta, s, partial, st,
                         M.src == SRC_DLP);
        else
          launch_gram(M.src, false, mixed, g, S.d_items, S.d_ents, d_units, nleafu, M.zeta, s,
                      partial, st);
        launch_check("gram (leaf)");
        tgl.stop();
        ss.n_gram_leaf += 1;
      }
      if (i8)
        launch_gram_i8(true, g, S.d_items, S.d_ents, d_units + nleafu,
                       (int64_t)units.size() - nleafu, M.zeta, s, partial, st);
      else
        launch_gram(M.src, true, mixed, g, S.d_items, S.d_ents, d_units + nleafu,
                    (int64_t)units.size() - nleafu, M.zeta, s, partial, st);
      launch_check("gram (non-leaf)");
      tg.stop();
      tr_.mark("gram", s, b, lv);
      launch_gram_reduce(S.d_items, d_litems, n, d_ubegin, d_units, partial, st);
      launch_check("gram reduce");
      // factor launches by size class: the LDS of a workgroup follows the
      // largest r of its class, so small factors run more workgroups per CU.
      // A launch lasts at least as long as its slowest item, so a class too
      // small to fill the device joins the next larger one.
      {
        constexpr int kFacClasses = 4;
        constexpr int32_t kFacLimit[kFacClasses - 1] = {32, 48, 64};
        std::vector<int32_t> fl[kFacClasses], big;
        int32_t rm[kFacClasses] = {0, 0, 0, 0};
        for (int32_t i = lo; i < hi; ++i) {
          // factors beyond the LDS-resident kernel stage X in device memory
          if (S.items[i].r > kMaxR) {
            big.push_back(i);
            continue;
          }
          int c = 0;
          while (c < kFacClasses - 1 && S.items[i].r > kFacLimit[c]) ++c;
          fl[c].push_back(i);
          rm[c] = std::max(rm[c], S.items[i].r);
        }
        for (int c = 0; c + 1 < kFacClasses; ++c)
          if (!fl[c].empty() && fl[c].size() < 2048) {
            fl[c + 1].insert(fl[c + 1].end(), fl[c].begin(), fl[c].end());
            rm[c + 1] = std::max(rm[c + 1], rm[c]);
            fl[c].clear();
          }
        std::vector<int32_t> all;
        for (int c = 0; c < kFacClasses; ++c) all.insert(all.end(), fl[c].begin(), fl[c].end());
        for (int c = 0; c < kFacClasses; ++c) ss.n_fac[c] += (int64_t)fl[c].size();
        ss.n_fac[kFacClasses] += (int64_t)big.size();
        int32_t* d_fl = upload(mem, all, st);
        int64_t off = 0;
        for (int c = 0; c < kFacClasses; ++c) {
          launch_factor(S.d_items, d_fl + off, (int32_t)fl[c].size(), rm[c], M.eps,
                        M.max_sweeps, d_status, st);
          off += (int64_t)fl[c].size();
        }
        double2* xws = nullptr;
        int32_t* d_big = nullptr;
        double2** d_xptr = nullptr;
        if (!big.empty()) {
          int64_t tot = 0;
          for (int32_t i : big) tot += (int64_t)S.items[i].r * (S.items[i].r + 1);
          xws = (double2*)mem.alloc((size_t)tot * sizeof(double2));
          std::vector<double2*> xp;
          int64_t o = 0;
          for (int32_t i : big) {
            xp.push_back(xws + o);
            o += (int64_t)S.items[i].r * (S.items[i].r + 1);
          }
          d_big = upload(mem, big, st);
          d_xptr = upload(mem, xp, st);
          launch_factor_big(S.d_items, d_big, (int32_t)big.size(), M.eps, M.max_sweeps, d_status,
                            d_xptr, st);
        }
        launch_check("factor");
        // only the ranks come back to the host (4 bytes per item)
        int32_t* d_k = (int32_t*)mem.alloc((size_t)n * sizeof(int32_t));
        launch_ranks(S.d_items + lo, n, d_k, st);
        launch_check("ranks");
        mem.sync(st, "factor sync");
        std::vector<int32_t> hk(n);
        copy_from(hk.data(), d_k, n, st);
        // factors whose numerical rank outgrew the LDS-resident kernel's columns
        // (rank -1) are factored again with X in device memory
        std::vector<int32_t> redo;
        for (int32_t i = 0; i < n; ++i)
          if (hk[i] < 0) redo.push_back(lo + i);
        ss.n_redo += (int64_t)redo.size();
        if (!redo.empty()) {
          // again in LDS with room for every column (one workgroup per CU)
          int32_t rmx = 0;
          for (int32_t i : redo) rmx = std::max(rmx, S.items[i].r);
          int32_t* d_redo = upload(mem, redo, st);
          launch_factor(S.d_items, d_redo, (int32_t)redo.size(), rmx, M.eps, M.max_sweeps,
                        d_status, st, true);
          launch_check("factor (wide)");
          launch_ranks(S.d_items + lo, n, d_k, st);
          launch_check("ranks");
          copy_from(hk.data(), d_k, n, st);
          mem.release(d_redo);
          redo.clear();
          for (int32_t i = 0; i < n; ++i)
            if (hk[i] < 0) redo.push_back(lo + i);
          ss.n_redo_mem += (int64_t)redo.size();
        }
        if (!redo.empty()) {
          // the rest (more columns than the LDS holds) with X in memory
          int64_t tot = 0;
          for (int32_t i : redo) tot += (int64_t)S.items[i].r * (S.items[i].r + 1);
          double2* xw2 = (double2*)mem.alloc((size_t)tot * sizeof(double2));
          std::vector<double2*> xp;
          int64_t o = 0;
          for (int32_t i : redo) {
            xp.push_back(xw2 + o);
            o += (int64_t)S.items[i].r * (S.items[i].r + 1);
          }
          int32_t* d_redo = upload(mem, redo, st);
          double2** d_xp2 = upload(mem, xp, st);
          launch_factor_big(S.d_items, d_redo, (int32_t)redo.size(), M.eps, M.max_sweeps,
                            d_status, d_xp2, st);
          launch_check("factor (memory-staged)");
          launch_ranks(S.d_items + lo, n, d_k, st);
          launch_check("ranks");
          copy_from(hk.data(), d_k, n, st);
          mem.release(xw2);
          mem.release(d_redo);
          mem.release(d_xp2);
        }
        for (int32_t i = 0; i < n; ++i) S.items[lo + i].k = hk[i];
        mem.release(d_fl);
        mem.release(d_k);
        mem.release(xws);
        mem.release(d_big);
        mem.release(d_xptr);
      }
      int32_t status = 0;
      copy_from(&status, d_status, 1, st);
      if (status & 1)
        fail(DH2_EUNSUPPORTED, "numerical rank of a block row exceeds the factor capacity");
      if (status & 2) fail(DH2_ENOTCONV, "one-sided Jacobi did not converge");
      tr_.mark("factor", s, b, lv);
      mem.release(Marena);
      for (int32_t i = lo; i < hi; ++i) S.items[i].M = nullptr;
      // coefficient matrices R of this level: the inherited columns (read by
      // the fathers) in the level's arena; in the row sweep the own-block
      // columns go straight into an arena kept for the projection
      int64_t sumNk = 0, sumOwn = 0;
      for (int32_t i = lo; i < hi; ++i) {
        sumNk += S.P->ninh[i] * S.items[i].k;
        if (s == 0) sumOwn += (S.items[i].N - S.P->ninh[i]) * S.items[i].k;
      }
      // R^T in complex FP64, or complex FP32 in the mixed form followed by the
      // row maxima of every R (k floats per item, for the parents' int8 Gram)
      size_t esz = mixed ? 2 * sizeof(float) : sizeof(double2);
      int64_t sumk = 0;
      for (int32_t i = lo; i < hi; ++i) sumk += S.items[i].k;
      size_t rbytes = ((size_t)sumNk * esz + 255) / 256 * 256;
      size_t mbytes = mixed ? (size_t)sumk * sizeof(float) : 0;
      char* Rarena = (char*)mem.alloc(rbytes + mbytes);
      char* Oarena = sumOwn > 0 ? (char*)mem.alloc((size_t)sumOwn * esz) : nullptr;
      if (Oarena) S.own_keep.push_back(Oarena);
      {
        int64_t o = 0, ok = 0, oo = 0;
        for (int32_t i = lo; i < hi; ++i) {
          ItemDev& it = S.items[i];
          it.R = Rarena + o * esz;
          it.rmax = mixed ? (float*)(Rarena + rbytes) + ok : nullptr;
          it.Rown = nullptr;
          if (s == 0) {
            it.Rown = Oarena ? Oarena + oo * esz : nullptr;
            S.own[i] = it.Rown;
            oo += (it.N - S.P->ninh[i]) * it.k;
          }
          o += S.P->ninh[i] * it.k;
          ok += it.k;
        }
      }
      if (mbytes) hip_check(hipMemsetAsync(Rarena + rbytes, 0, mbytes, st), "row maxima clear");
      copy_to(mem, S.d_items + lo, S.items.data() + lo, n, st);
      // R-product units: one workgroup per 1024 columns; leaf units first,
      // then non-leaf units grouped by ceil(k / 16).  The father reads only
      // the inherited columns of R; the own-block columns are kept for the
      // projection of the row sweep and not formed in the column sweep.
      std::vector<UnitDev> ru;
      int64_t nleafr = 0, nbigr = 0;
      std::vector<std::array<int64_t, 3>> rlaunch;  // kt, count, lds bytes
      // large transfer factors: Q_hat packed in 64-column chunks
      std::vector<int32_t> pk_item, pk_chunk;
      std::vector<void*> pk_dst, big_q;
      void* pkbuf = nullptr;
      {
        const int64_t rwidth = 1024;
        std::vector<UnitDev> inner_by_kt[9], big_units;
        size_t lds_kt[9] = {0};
        int64_t pk_bytes = 0;
        std::vector<int64_t> pk_off;
        for (int32_t i = lo; i < hi; ++i) {
          const ItemDev& it = S.items[i];
          if (it.k == 0) continue;
          int kt = (it.k + 15) / 16;
          const bool bigq = !it.leaf && (it.k > kMaxR || rprod_inner_lds(mixed, it.r, it.k) >
                                                             rprod_inner_lds_max());
          if (!it.leaf && !bigq)
            lds_kt[kt] = std::max(lds_kt[kt], rprod_inner_lds(mixed, it.r, it.k));
          const int64_t nr = s == 0 ? it.N : S.P->ninh[i];
          if (bigq) {
            const int nch = (it.k + 63) / 64;
            for (int c = 0; c < nch; ++c) {
              pk_item.push_back(i);
              pk_chunk.push_back(c);
              pk_off.push_back(pk_bytes);
              pk_bytes += (int64_t)(it.r + 8) * 64 * (mixed ? sizeof(float2) : sizeof(double2));
              for (int64_t c0 = 0; c0 < nr; c0 += rwidth) {
                UnitDev u{};
                u.item = i;
                u.a0 = (int8_t)c;
                u.col_begin = c0;
                u.ncols = std::min(rwidth, nr - c0);
                big_units.push_back(u);
                big_q.push_back((void*)(intptr_t)(pk_off.size() - 1));
              }
            }
          } else {
            for (int64_t c0 = 0; c0 < nr; c0 += rwidth) {
              UnitDev u{};
              u.item = i;
              u.col_begin = c0;
              u.ncols = std::min(rwidth, nr - c0);
              (it.leaf ? ru : inner_by_kt[kt]).push_back(u);
            }
          }
          ss.flops_rprod += 8.0 * it.k * (double)it.r * (double)nr;
          if (it.leaf) ss.flops_rprod_leaf += 8.0 * it.k * (double)it.r * (double)nr;
        }
        nleafr = (int64_t)ru.size();
        for (int kt = 1; kt <= 8; ++kt) {
          if (inner_by_kt[kt].empty()) continue;
          rlaunch.push_back({kt, (int64_t)inner_by_kt[kt].size(), (int64_t)lds_kt[kt]});
          ru.insert(ru.end(), inner_by_kt[kt].begin(), inner_by_kt[kt].end());
        }
        nbigr = (int64_t)big_units.size();
        ru.insert(ru.end(), big_units.begin(), big_units.end());
        if (pk_bytes > 0) {
          pkbuf = mem.alloc((size_t)pk_bytes);
          for (int64_t off : pk_off) pk_dst.push_back((char*)pkbuf + off);
          for (auto& q : big_q) q = pk_dst[(size_t)(intptr_t)q];
        }
      }
      UnitDev* d_ru = upload(mem, ru, st);
      tr_.mark("rprod units", s, b, lv);
      launch_rprod_leaf(M.src, mixed, g, S.d_items, S.d_ents, d_ru, nleafr, s, st);
      launch_check("rprod (leaf)");
      {
        int64_t off = nleafr;
        for (const auto& L : rlaunch) {
          launch_rprod_inner(mixed, (int)L[0], S.d_items, d_ru + off, L[1], M.zeta, (size_t)L[2],
                             st);
          off += L[1];
        }
      }
      if (nbigr > 0) {
        int32_t* d_pki = upload(mem, pk_item, st);
        int32_t* d_pkc = upload(mem, pk_chunk, st);
        void** d_pkd = upload(mem, pk_dst, st);
        void** d_bq = upload(mem, big_q, st);
        launch_pack_q(S.d_items, d_pki, d_pkc, d_pkd, (int64_t)pk_item.size(), mixed, st);
        launch_rprod_inner_big(mixed, S.d_items, d_ru + (ru.size() - nbigr), nbigr, M.zeta, d_bq,
                               st);
        mem.release(d_pki);
        mem.release(d_pkc);
        mem.release(d_pkd);
        mem.release(d_bq);
        mem.release(pkbuf);
      }
      launch_check("rprod (non-leaf)");
      if (trace_on()) hip_check(hipStreamSynchronize(st), "trace sync");
      tr_.mark("rprod", s, b, lv);
      // no wait here: the next level's host work overlaps this level's
      // kernels, and the released blocks are reused only after a sync
      mem.release(d_units);
      mem.release(d_litems);
      mem.release(d_ubegin);
      mem.release(d_ru);
      mem.release(d_leaf_ids);
      mem.release(colbuf);
      for (int32_t i = lo; i < hi; ++i) S.items[i].cols = nullptr;
      mem.release(R_prev);
      R_prev = Rarena;
      tr_.mark("level end", s, b, lv);
      if (trace_on()) {
        size_t fr = 0, tot = 0;
        (void)hipMemGetInfo(&fr, &tot);
        size_t cached = 0;
        {
          std::lock_guard<std::mutex> lk(g_cache_mu);
          cached = g_cached;
        }
        std::fprintf(stderr,
                     "[dh2 mem] side %d batch %d level %d: owner %.1f GB (peak %.1f), cache %.1f "
                     "GB, driver free %.1f GB\n",
                     s, b, lv, mem.used() * 1e-9, mem.peak() * 1e-9, cached * 1e-9, fr * 1e-9);
      }
    }
    mem.release(R_prev);
    for (int32_t i = 0; i < S.nitems; ++i) {
      S.items[i].R = nullptr;
      S.items[i].Rown = nullptr;
    }
  }
  mem.release(partial);
  ss.t_gram += tg.total();
  ss.t_gram_leaf += tgl.total();
}

// Expanded column basis of one level (W_sc as an explicit #s x k matrix,
// from the sons' expanded bases and the transfer matrices; leaves: Q), and in
// the mixed form its complex FP32 copy for the projection.
static void expand_level(MatrixData& M, int s, int32_t lv, hipStream_t st, DevMem& mem) {
  Side& S = M.side[s];
  std::vector<int32_t> idx;
  int64_t total = 0, total32 = 0;
  for (int32_t b = 0; b < M.nbatch; ++b)
    for (int32_t i = S.P->range[b][lv].first; i < S.P->range[b][lv].second; ++i) {
      idx.push_back(i);
      if (!S.items[i].leaf) total += (int64_t)S.items[i].m * S.items[i].k;
      total32 += (int64_t)S.items[i].m * S.items[i].k;
    }
  if (idx.empty()) return;
  if (S.wexp32.size() != (size_t)S.nitems) S.wexp32.assign(S.nitems, nullptr);
  double2* arena = total ? (double2*)mem.alloc(total * sizeof(double2)) : nullptr;
  if (arena) S.keep.push_back(arena);
  std::vector<ExpandDev> tasks;
  int64_t o = 0;
  for (int32_t i : idx) {
    ItemDev& it = S.items[i];
    if (it.leaf) {
      S.wexp[i] = it.Q;
      continue;
    }
    S.wexp[i] = arena + o;
    int64_t rowo = 0;
    int32_t koff = 0;
    for (int q = 0; q < 2; ++q) {
      const ItemDev& so = S.items[it.son[q]];
      ExpandDev ed{};
      ed.src = S.wexp[it.son[q]];
      ed.E = it.Q + (int64_t)koff * it.k;
      ed.dst = arena + o + rowo * it.k;
      ed.rows = so.m;
      ed.ks = so.k;
      ed.k = it.k;
      if (it.k > 0) tasks.push_back(ed);
      rowo += so.m;
      koff += so.k;
    }
    o += (int64_t)it.m * it.k;
  }
  ExpandDev* d_tasks = upload(mem, tasks, st);
  launch_expand(d_tasks, (int64_t)tasks.size(), st);
  launch_check("expand");
  mem.release(d_tasks);
  if (M.precision == DH2_MIXED) {
    float2* a32 = (float2*)mem.alloc(std::max<int64_t>(1, total32) * sizeof(float2));
    S.keep.push_back(a32);
    std::vector<CvtDev> ct;
    int64_t o32 = 0;
    for (int32_t i : idx) {
      int64_t cnt = (int64_t)S.items[i].m * S.items[i].k;
      S.wexp32[i] = a32 + o32;
      if (cnt > 0) ct.push_back(CvtDev{S.wexp[i], a32 + o32, cnt});
      o32 += cnt;
    }
    CvtDev* d_ct = upload(mem, ct, st);
    launch_cvt(d_ct, (int64_t)ct.size(), st);
    launch_check("basis conversion");
    mem.release(d_ct);
  }
}

// expanded column bases, level by level from the leaves
static void expand_side(MatrixData& M, int s, hipStream_t st, DevMem& mem) {
  const ClusterTree& tr = M.blk->tree->tr;
  for (int32_t lv = tr.depth; lv >= 0; --lv) expand_level(M, s, lv, st, mem);
  mem.sync(st, "expand sync");
}

// Projection of every admissible block after both sweeps:
// S_b = omega_b R_tc|s W_sc from the kept own-block columns of the row
// sweep's R and the expanded column basis, in one set of launches for all
// levels.  Tiled kernel for ks <= 64 (one launch per (row tiles per pass,
// column tiles)), the generic kernel above; in the mixed form the blocks of
// ks <= 64 that share W_sc are stacked (k_project_stacked).
static void project_all(MatrixData& M, hipStream_t st, DevMem& mem, SweepStats& ss) {
  Trace tr_;
  Side& S = M.side[0];
  const Side& C = M.side[1];
  const bool mixed = M.precision == DH2_MIXED;
  const size_t esz = mixed ? 2 * sizeof(float) : sizeof(double2);
  constexpr int kGeneric = 32;
  // The task lists are built by a few host threads over chunks of the plan
  // (whole runs of one column item, so that stacking stays within a chunk),
  // then joined in plan order.
  struct PChunk {
    size_t plan, q0, q1;
    int64_t s_off;
    std::vector<ProjDev> tasks;
    std::vector<uint8_t> key;
    std::vector<PBlkDev> pblk;
    std::vector<PTileDev> ptile;
    std::vector<uint8_t> tnc;
    int64_t count[kGeneric + 1] = {0};
    int64_t ncount[17] = {0};
    double flops = 0.0;
  };
  const auto& plans = M.plan->proj;
  int64_t nblk_all = 0;
  for (const auto& pl : plans) nblk_all += (int64_t)pl.size();
  const int nth = (int)std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
  const int64_t target = std::max<int64_t>(2048, nblk_all / (4 * nth));
  std::vector<PChunk> chunks;
  int64_t sumS = 0;
  for (size_t p = 0; p < plans.size(); ++p) {
    const auto& pl = plans[p];
    size_t q0 = 0;
    int64_t s0 = sumS;
    for (size_t q = 0; q < pl.size(); ++q) {
      if (q > q0 && (int64_t)(q - q0) >= target && pl[q].witem != pl[q - 1].witem) {
        chunks.emplace_back();
        chunks.back().plan = p;
        chunks.back().q0 = q0;
        chunks.back().q1 = q;
        chunks.back().s_off = s0;
        q0 = q;
        s0 = sumS;
      }
      sumS += (int64_t)S.items[pl[q].item].k * C.items[pl[q].witem].k;
    }
    if (q0 < pl.size()) {
      chunks.emplace_back();
      chunks.back().plan = p;
      chunks.back().q0 = q0;
      chunks.back().q1 = pl.size();
      chunks.back().s_off = s0;
    }
  }
  // S_b in the form's storage precision (complex FP32 in the mixed form)
  const size_t sesz = M.s32 ? sizeof(float2) : sizeof(double2);
  char* Sarena = (char*)mem.alloc(std::max<int64_t>(1, sumS) * sesz);
  S.keep.push_back(Sarena);
  auto build = [&](PChunk& ch) {
    const auto& pl = plans[ch.plan];
    int64_t o = ch.s_off;
    ch.tasks.reserve(ch.q1 - ch.q0);
    ch.key.reserve(ch.q1 - ch.q0);
    for (size_t x = ch.q0; x < ch.q1; ++x) {
      const ProjPlan& q = pl[x];
      const ItemDev& it = S.items[q.item];
      const int32_t ks = C.items[q.witem].k;
      ProjDev pd{};
      pd.R = (const char*)S.own[q.item] + (q.col - S.P->ninh[q.item]) * it.k * esz;
      pd.W = mixed ? (const void*)C.wexp32[q.witem] : (const void*)C.wexp[q.witem];
      pd.S = Sarena + o * sesz;
      pd.kt = it.k;
      pd.ks = ks;
      pd.ns = q.ns;
      pd.b = q.b;
      M.S_ptr[q.b] = Sarena + o * sesz;
      M.S_rows[q.b] = it.k;
      M.S_cols[q.b] = ks;
      o += (int64_t)it.k * ks;
      ch.flops += 8.0 * it.k * (double)ks * (double)q.ns;
      uint8_t kx = 255;
      if (it.k > 0 && ks > 0 && !(mixed && ks <= 64)) {
        int nj = (ks + 15) / 16, ni = (it.k + 15) / 16;
        int c = kGeneric;
        if (nj <= 4)
          c = (q.ns >= 128 ? 16 : 0) + (std::min(ni, project_rows_per_pass(mixed, nj)) - 1) * 4 +
              (nj - 1);
        kx = (uint8_t)c;
        ++ch.count[c];
      }
      ch.tasks.push_back(pd);
      ch.key.push_back(kx);
    }
    if (!mixed) return;
    // blocks of each run of equal column item (the plan of a level is
    // sorted by it) stacked row-wise and cut into tiles of up to 64 rows;
    // tile block indices are local to the chunk until the join
    for (size_t g0 = ch.q0; g0 < ch.q1;) {
      size_t g1 = g0;
      while (g1 < ch.q1 && pl[g1].witem == pl[g0].witem) ++g1;
      const int32_t ks = C.items[pl[g0].witem].k;
      if (ks == 0 || ks > 64) {
        g0 = g1;
        continue;
      }
      const int32_t b0 = (int32_t)ch.pblk.size();
      for (size_t x = g0; x < g1; ++x) {
        const ProjDev& pd = ch.tasks[x - ch.q0];
        if (pd.kt > 0)
          ch.pblk.push_back(PBlkDev{(const float2*)pd.R, (float2*)pd.S, pd.kt, pd.b});
      }
      const int32_t b1 = (int32_t)ch.pblk.size();
      int32_t bi = b0, i0 = 0;
      while (bi < b1) {
        PTileDev t;
        t.W = C.wexp32[pl[g0].witem];
        t.blk0 = bi;
        t.i0 = i0;
        t.ns = pl[g0].ns;
        t.ks = ks;
        int32_t rows = 0, nblk = 0;
        while (rows < 64 && bi < b1) {
          int32_t take = std::min(64 - rows, ch.pblk[bi].kt - i0);
          rows += take;
          i0 += take;
          ++nblk;
          if (i0 == ch.pblk[bi].kt) {
            ++bi;
            i0 = 0;
          }
        }
        t.rows = rows;
        t.nblk = nblk;
        ch.ptile.push_back(t);
        ch.tnc.push_back((uint8_t)((ks + 3) / 4));
        ++ch.ncount[(ks + 3) / 4];
      }
      g0 = g1;
    }
  };
  {
    std::vector<std::thread> th;
    std::atomic<size_t> next{0};
    for (int t = 0; t < nth; ++t)
      th.emplace_back([&] {
        for (size_t c; (c = next.fetch_add(1)) < chunks.size();) build(chunks[c]);
      });
    for (auto& t : th) t.join();
  }
  // final positions: tasks sorted (stably) by launch class, tiles by
  // ceil(ks / 4), blocks of the stacked tiles in plan order; each chunk
  // scatters its own lists into place in parallel
  const size_t nch = chunks.size();
  int64_t count[kGeneric + 1] = {0};
  int64_t ncount[17] = {0};
  std::vector<int64_t> pbase(nch + 1, 0);
  for (size_t c = 0; c < nch; ++c) {
    for (int k = 0; k <= kGeneric; ++k) count[k] += chunks[c].count[k];
    for (int k = 0; k <= 16; ++k) ncount[k] += chunks[c].ncount[k];
    pbase[c + 1] = pbase[c] + (int64_t)chunks[c].pblk.size();
    ss.flops_prj += chunks[c].flops;
  }
  std::vector<std::array<int64_t, 4>> launches;  // ni, nj, split, count
  std::vector<std::array<int64_t, kGeneric + 1>> toff(nch);
  std::vector<std::array<int64_t, 17>> noff(nch);
  int64_t ntask = 0, ntile = 0;
  {
    int64_t start[kGeneric + 1];
    for (int kx = 0; kx <= kGeneric; ++kx) {
      start[kx] = ntask;
      ntask += count[kx];
      if (count[kx] == 0) continue;
      if (kx < kGeneric)
        launches.push_back({(kx % 16) / 4 + 1, kx % 4 + 1, kx / 16, count[kx]});
      else
        launches.push_back({0, 0, 0, count[kx]});
    }
    int64_t nstart[17];
    for (int k = 0; k <= 16; ++k) {
      nstart[k] = ntile;
      ntile += ncount[k];
    }
    for (size_t c = 0; c < nch; ++c) {
      for (int k = 0; k <= kGeneric; ++k) {
        toff[c][k] = start[k];
        start[k] += chunks[c].count[k];
      }
      for (int k = 0; k <= 16; ++k) {
        noff[c][k] = nstart[k];
        nstart[k] += chunks[c].ncount[k];
      }
    }
  }
  std::vector<ProjDev> sorted(ntask);
  std::vector<PBlkDev> pblk(pbase[nch]);
  std::vector<PTileDev> ptile(ntile);
  {
    auto scatter = [&](size_t c) {
      PChunk& ch = chunks[c];
      for (size_t x = 0; x < ch.tasks.size(); ++x)
        if (ch.key[x] != 255) sorted[toff[c][ch.key[x]]++] = ch.tasks[x];
      std::copy(ch.pblk.begin(), ch.pblk.end(), pblk.begin() + pbase[c]);
      for (size_t x = 0; x < ch.ptile.size(); ++x) {
        PTileDev t = ch.ptile[x];
        t.blk0 += (int32_t)pbase[c];
        ptile[noff[c][ch.tnc[x]]++] = t;
      }
    };
    std::vector<std::thread> th;
    std::atomic<size_t> next{0};
    for (int t = 0; t < nth; ++t)
      th.emplace_back([&] {
        for (size_t c; (c = next.fetch_add(1)) < nch;) scatter(c);
      });
    for (auto& t : th) t.join();
  }
  tr_.mark("proj build", 0, -1, -1);
  ProjDev* d_tasks = upload(mem, sorted, st);
  PBlkDev* d_pblk = upload(mem, pblk, st);
  PTileDev* d_ptile = upload(mem, ptile, st);
  tr_.mark("proj upload", 0, -1, -1);
  PhaseTimer tp(st);
  tp.start();
  // The launches (one per class) are independent: they are spread over
  // kPrjStreams streams (the caller's and three more, default priority),
  // each class to the stream with the least work so far, so that the tails
  // of small launches overlap; the streams join the caller's at the end.
  constexpr int kPrjStreams = 4;
  struct Fork {
    hipStream_t s[kPrjStreams] = {};
    hipEvent_t e[kPrjStreams] = {};
    ~Fork() {
      for (int q = 1; q < kPrjStreams; ++q)
        if (s[q]) (void)hipStreamDestroy(s[q]);
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } fk;
  fk.s[0] = st;
  for (int q = 0; q < kPrjStreams; ++q)
    hip_check(hipEventCreateWithFlags(&fk.e[q], hipEventDisableTiming), "event");
  hip_check(hipEventRecord(fk.e[0], st), "event record");
  for (int q = 1; q < kPrjStreams; ++q) {
    hip_check(hipStreamCreateWithFlags(&fk.s[q], hipStreamNonBlocking), "stream create");
    hip_check(hipStreamWaitEvent(fk.s[q], fk.e[0], 0), "stream wait");
  }
  double load[kPrjStreams] = {0.0};
  auto pick = [&](double work) {
    int q = 0;
    for (int x = 1; x < kPrjStreams; ++x)
      if (load[x] < load[q]) q = x;
    load[q] += work;
    return fk.s[q];
  };
  {
    int64_t toff = 0;
    for (int c = 1; c <= 16; ++c) {
      if (ncount[c] > 0)
        launch_project_stacked(c, d_ptile + toff, ncount[c], d_pblk, M.d_omega,
                               pick((double)ncount[c] * c));
      toff += ncount[c];
    }
    launch_check("project (stacked)");
  }
  int64_t off = 0;
  for (const auto& L : launches) {
    hipStream_t ls = pick((double)L[3] * std::max<int64_t>(1, L[0] * L[1]));
    if (L[0] > 0)
      launch_project_tiled(mixed, (int)L[0], (int)L[1], L[2] != 0, d_tasks + off, L[3], M.d_omega,
                           ls);
    else
      launch_project(mixed, d_tasks + off, L[3], M.d_omega, ls);
    launch_check("project");
    off += L[3];
  }
  for (int q = 1; q < kPrjStreams; ++q) {
    hip_check(hipEventRecord(fk.e[q], fk.s[q]), "event record");
    hip_check(hipStreamWaitEvent(st, fk.e[q], 0), "stream wait");
  }
  tp.stop();
  tr_.mark("proj launch", 0, -1, -1);
  ss.t_prj += tp.total();
  tr_.mark("proj done", 0, -1, -1);
  mem.release(d_tasks);
  mem.release(d_pblk);
  mem.release(d_ptile);
  for (void* q : S.own_keep) mem.release(q);
  S.own_keep.clear();
  std::fill(S.own.begin(), S.own.end(), nullptr);
}

static std::shared_ptr<const SweepSizes> sweep_sizes(const BlocksData& B) {
  const ClusterTree& tr = B.tree->tr;
  auto Z = std::make_shared<SweepSizes>();
  Z->lmin = B.bt.adm_t.empty() ? 0 : first_adm_level(B);
  const int32_t lg = std::max(0, Z->lmin - 1);
  Z->group.assign(tr.nc(), -1);
  for (int32_t t = 0; t < tr.nc(); ++t) {
    if (tr.level[t] == lg) Z->group[t] = Z->ngroups++;
    else if (tr.level[t] > lg) Z->group[t] = Z->group[tr.father[t]];
  }
  Z->lvlN.assign(tr.depth + 2, 0.0);
  Z->grpN.assign(std::max(1, Z->ngroups), 0.0);
  for (int s = 0; s < 2; ++s) {
    const ColumnSets& cs = B.cs[s];
    for (int32_t e = 0; e < cs.nitems(); ++e) {
      int32_t t = cs.item_t[e];
      double N = 0;
      for (int64_t q = cs.begin[e]; q < cs.begin[e + 1]; ++q) N += (double)tr.size[cs.ent[q].s];
      Z->lvlN[tr.level[t]] += N * 0.5;
      if (Z->group[t] >= 0) Z->grpN[Z->group[t]] += N;
    }
  }
  return Z;
}

std::unique_ptr<MatrixData> compress(std::shared_ptr<BlocksData> blk, int src, const void* G,
                                     int64_t ld, const double* w, double eps, const dh2_opts& o,
                                     hipStream_t st, const double* nrm, bool concurrent) {
  auto Mp = std::make_unique<MatrixData>();
  MatrixData& M = *Mp;
  M.blk = blk;
  M.src = src;
  M.eps = eps;
  M.zeta = o.zeta;
  M.precision = o.precision;
  M.s32 = o.precision == DH2_MIXED;
  M.max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 60;
  M.mem = std::make_unique<DevMem>(o.max_device_bytes);
  const ClusterTree& tr = blk->tree->tr;
  const BlockTree& bt = blk->bt;
  int64_t n = tr.n;
  int64_t nadm = (int64_t)bt.adm_t.size();
  DevMem& mem = *M.mem;
  Trace trc;
  // uploads of the compression go through pinned staging, without waits
  mem.begin_staging();

  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "event");
  hip_check(hipEventCreate(&e1), "event");

  // geometry in permuted order
  M.w.assign(n, 4.0 * M_PI / (double)n);
  if (w) M.w.assign(w, w + n);
  std::vector<double> pp(4 * n);
  for (int64_t p = 0; p < n; ++p) {
    int64_t i = tr.perm[p];
    for (int a = 0; a < 3; ++a) pp[4 * p + a] = blk->tree->pts[3 * i + a];
    pp[4 * p + 3] = M.w[i];
  }
  M.d_pts = upload(mem, pp, st);
  M.d_perm = upload(mem, tr.perm, st);
  if (src == SRC_DLP) {
    if (!nrm) fail(DH2_EINVAL, "normals are NULL");
    std::vector<double> pn(4 * n, 0.0);
    for (int64_t p = 0; p < n; ++p)
      for (int a = 0; a < 3; ++a) pn[4 * p + a] = nrm[3 * tr.perm[p] + a];
    M.d_nrm = upload(mem, pn, st);
  }
  {
    // cluster boxes and largest weights (bounds of the entry magnitudes)
    std::vector<double> cb(8 * (size_t)tr.nc(), 0.0);
    for (int32_t t = tr.nc() - 1; t >= 0; --t) {
      for (int a = 0; a < 3; ++a) {
        cb[8 * t + a] = tr.lo[3 * t + a];
        cb[8 * t + 3 + a] = tr.hi[3 * t + a];
      }
      double wm = 0.0;
      if (tr.leaf(t)) {
        for (int64_t p = tr.off[t]; p < tr.off[t] + tr.size[t]; ++p)
          wm = std::max(wm, std::fabs(M.w[tr.perm[p]]));
      } else {
        wm = std::max(cb[8 * tr.son1[t] + 6], cb[8 * tr.son2[t] + 6]);
      }
      cb[8 * t + 6] = wm;
    }
    M.d_cbox = upload(mem, cb, st);
  }
  GeomDev g{};
  g.pts = M.d_pts;
  g.cbox = M.d_cbox;
  g.nrm = M.d_nrm;
  g.G = (const double*)G;
  g.perm = M.d_perm;
  g.ldg = ld;
  g.n = n;
  g.kappa = blk->tree->kappa;

  trc.mark("geometry", -1, -1, -1);
  // batches: subtrees rooted one level above the first admissible level
  std::shared_ptr<const SweepSizes> SZ;
  {
    std::lock_guard<std::mutex> lk(blk->cache_mu);
    if (!blk->sizes) blk->sizes = sweep_sizes(*blk);
    SZ = blk->sizes;
  }
  M.lmin = SZ->lmin;
  const int32_t ngroups = SZ->ngroups;
  const std::vector<int32_t>& group = SZ->group;
  const std::vector<double>& lvlN = SZ->lvlN;
  const std::vector<double>& grpN = SZ->grpN;
  // estimated R memory per level (rank estimate, 16 bytes per coefficient in
  // the FP64 form, 8 in the mixed form)
  // rank estimate: about 48 (at most the leaf size) with the directional
  // admissibility; the standard condition alone admits blocks whose ranks
  // grow with kappa (several times larger in the paper's comparison), so
  // twice the leaf size there
  double kest = o.standard_only ? 2.0 * o.leaf_size : std::min(48.0, (double)o.leaf_size);
  double peak = 0;
  const double csz = o.precision == DH2_MIXED ? 8.0 : 16.0;
  for (int32_t l = 0; l <= tr.depth; ++l) peak = std::max(peak, (lvlN[l] + lvlN[l + 1]) * kest * csz);
  size_t freeb = 0, totalb = 0;
  hip_check(hipMemGetInfo(&freeb, &totalb), "hipMemGetInfo");
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    freeb += g_cached;  // blocks held in the cache are available to this call
  }
  double budget = 0.75 * (double)freeb;
  if (o.max_device_bytes > 0) budget = std::min(budget, 0.75 * (double)o.max_device_bytes);
  {
    // the near field is generated beside the sweeps and held through them
    double near_bytes = 0;
    for (size_t b = 0; b < bt.near_t.size(); ++b)
      near_bytes += (o.precision == DH2_MIXED ? 8.0 : 16.0) * (double)tr.size[bt.near_t[b]] *
                    (double)tr.size[bt.near_s[b]];
    budget = std::max(0.25 * budget, budget - near_bytes);
  }
  // The row and column sweeps are independent (the projection follows both),
  // so they run at the same time, each on its own stream, unless a memory
  // cap is set (then one after the other, so that the cap stays exact).
  // Running together they hold the R matrices of both sides: the batch
  // count leaves room for that.
  M.concurrent = concurrent && o.max_device_bytes == 0;
  const double need = M.concurrent ? 2.0 * peak : peak;
  int32_t nb = o.groups > 0 ? o.groups : (int32_t)std::ceil(need / std::max(1.0, budget));
  nb = std::max(1, std::min(nb, std::max(1, ngroups)));
  M.nbatch = nb;
  std::vector<int32_t> batch_of(tr.nc(), 0);
  {
    double tot = std::accumulate(grpN.begin(), grpN.end(), 0.0), cum = 0;
    std::vector<int32_t> gb(std::max(1, ngroups), 0);
    for (int32_t q = 0; q < ngroups; ++q) {
      gb[q] = tot > 0 ? std::min(nb - 1, (int32_t)(cum * nb / tot)) : 0;
      cum += grpN[q];
    }
    for (int32_t t = 0; t < tr.nc(); ++t) batch_of[t] = group[t] >= 0 ? gb[group[t]] : 0;
  }

  trc.mark("batches", -1, -1, -1);
  M.plan = plan_cache(*blk, nb, batch_of);
  for (int s = 0; s < 2; ++s) {
    Side& S = M.side[s];
    S.P = M.plan->side[s];
    S.nitems = S.P->nitems;
    S.items = S.P->items0;
    S.wexp.assign(S.nitems, nullptr);
    S.own.assign(S.nitems, nullptr);
  }
  trc.mark("plan", -1, -1, -1);
  M.S_ptr.assign(nadm, nullptr);
  M.S_rows.assign(nadm, 0);
  M.S_cols.assign(nadm, 0);

  // per side (row sweep at 0, column sweep at 4): status[0]: error bits of
  // the factorisation; status[1], status[2]: Jacobi sweeps and factorisations
  // (statistics)
  int32_t* d_status = (int32_t*)mem.alloc(8 * sizeof(int32_t));
  hip_check(hipMemsetAsync(d_status, 0, 8 * sizeof(int32_t), st), "memset");

  // block weights and column scales
  hip_check(hipEventRecord(e0, st), "event");
  {
    const int64_t* d_to = M.plan->d_adm;
    const int64_t* d_tl = d_to + nadm;
    const int64_t* d_so = d_to + 2 * nadm;
    const int64_t* d_sl = d_to + 3 * nadm;
    M.d_omega = (double*)mem.alloc(std::max<int64_t>(1, nadm) * sizeof(double));
    if (o.weights == DH2_WEIGHTS_SPECTRAL) {
      for (int64_t b = 0; b < nadm; ++b)
        if (std::max(tr.size[bt.adm_t[b]], tr.size[bt.adm_s[b]]) > block_norm2_max_size())
          fail(DH2_EUNSUPPORTED, "spectral block weights need clusters of at most " +
                                     std::to_string(block_norm2_max_size()) + " points");
      launch_block_norm2(src, g, d_to, d_tl, d_so, d_sl, nadm, 1000, 1e-13, M.d_omega, st);
    } else {
      launch_block_norm(src, g, d_to, d_tl, d_so, d_sl, nadm, M.d_omega, st);
    }
    launch_check("block norms");
    if (o.weights == DH2_WEIGHTS_GLOBAL && nadm > 0) {
      // one weight for every block: the Frobenius norm of G on the
      // admissible blocks (global-relative tolerance)
      std::vector<double> om(nadm);
      copy_from(om.data(), M.d_omega, nadm, st);
      double s2 = 0.0;
      for (double v : om) s2 += v * v;
      std::fill(om.begin(), om.end(), std::sqrt(s2));
      mem.upload(M.d_omega, om.data(), (size_t)nadm * sizeof(double), st);
    }
    for (int s = 0; s < 2; ++s) {
      Side& S = M.side[s];
      S.d_items = upload(mem, S.items, st);
      // per-matrix copy of the plan's column entries (their scales depend on omega)
      size_t nent = S.P->ents.size();
      S.d_ents = (EntDev*)mem.alloc(std::max<size_t>(1, nent) * sizeof(EntDev));
      if (nent)
        hip_check(hipMemcpyAsync(S.d_ents, M.plan->d_ents[s], nent * sizeof(EntDev),
                                 hipMemcpyDeviceToDevice, st),
                  "entries copy");
      launch_entry_scale(S.d_ents, (int64_t)nent, M.d_omega, M.zeta, st);
      launch_check("entry scales");
    }
    mem.sync(st, "weights sync");
  }
  hip_check(hipEventRecord(e1, st), "event");
  hip_check(hipEventSynchronize(e1), "event");
  trc.mark("weights", -1, -1, -1);
  float ms_w = 0;
  hip_check(hipEventElapsedTime(&ms_w, e0, e1), "event");

  // near field: independent of the sweeps, so it is generated on a stream
  // of its own (default priority) beside them and joined at the end
  struct NearFork {
    hipStream_t s = nullptr;
    hipEvent_t e[3] = {nullptr, nullptr, nullptr};
    int64_t* d[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    ~NearFork() {
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } nf;
  const int64_t nnear = (int64_t)bt.near_t.size();
  {
    std::vector<int64_t> to(nnear), tl(nnear), so(nnear), sl(nnear), oo(nnear);
    int64_t tot = 0;
    M.nears.resize(nnear);
    for (int64_t b = 0; b < nnear; ++b) {
      to[b] = tr.off[bt.near_t[b]];
      tl[b] = tr.size[bt.near_t[b]];
      so[b] = tr.off[bt.near_s[b]];
      sl[b] = tr.size[bt.near_s[b]];
      oo[b] = tot;
      M.nears[b] = NearDev{tot, to[b], tl[b], so[b], sl[b]};
      tot += tl[b] * sl[b];
    }
    M.d_near = mem.alloc(std::max<int64_t>(1, tot) * (M.s32 ? sizeof(float2) : sizeof(double2)));
    nf.d[0] = upload(mem, to, st);
    nf.d[1] = upload(mem, tl, st);
    nf.d[2] = upload(mem, so, st);
    nf.d[3] = upload(mem, sl, st);
    nf.d[4] = upload(mem, oo, st);
    hip_check(hipStreamCreateWithFlags(&nf.s, hipStreamNonBlocking), "stream create");
    for (auto& x : nf.e) hip_check(hipEventCreate(&x), "event");
    hip_check(hipEventRecord(nf.e[2], st), "event");
    hip_check(hipStreamWaitEvent(nf.s, nf.e[2], 0), "stream wait");
    hip_check(hipEventRecord(nf.e[0], nf.s), "event");
    launch_near(src, g, nf.d[0], nf.d[1], nf.d[2], nf.d[3], nf.d[4], nnear, M.d_near, M.s32, nf.s);
    launch_check("near field");
    hip_check(hipEventRecord(nf.e[1], nf.s), "event");
  }

  SweepStats ss_col, ss_row;
  float ms_col = 0, ms_row = 0, ms_sweeps = 0;
  if (!M.concurrent) {
    // column basis (expanded), then the row basis
    hip_check(hipEventRecord(e0, st), "event");
    sweep(M, 1, g, st, ss_col, d_status + 4, mem);
    expand_side(M, 1, st, mem);
    hip_check(hipEventRecord(e1, st), "event");
    hip_check(hipEventSynchronize(e1), "event");
    hip_check(hipEventElapsedTime(&ms_col, e0, e1), "event");
    hip_check(hipEventRecord(e0, st), "event");
    sweep(M, 0, g, st, ss_row, d_status, mem);
    hip_check(hipEventRecord(e1, st), "event");
    hip_check(hipEventSynchronize(e1), "event");
    hip_check(hipEventElapsedTime(&ms_row, e0, e1), "event");
    ms_sweeps = ms_col + ms_row;
  } else {
    // both sweeps at once: the column sweep (and the expansion of its basis)
    // on a second stream (default priority), driven by a second host thread
    // with its own device-memory owner.  Kernels of the two sweeps fill each
    // other's idle time (small factorisations, rank read-backs, launch tails).
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    hipStream_t sc = nullptr;
    hip_check(hipStreamCreateWithFlags(&sc, hipStreamNonBlocking), "stream create");
    struct Cleanup {
      hipStream_t s = nullptr;
      hipEvent_t e[3] = {nullptr, nullptr, nullptr};
      ~Cleanup() {
        if (s) {
          (void)hipStreamSynchronize(s);
          (void)hipStreamDestroy(s);
        }
        for (hipEvent_t x : e)
          if (x) (void)hipEventDestroy(x);
      }
    } cleanup;
    cleanup.s = sc;
    for (auto& x : cleanup.e) hip_check(hipEventCreate(&x), "event");
    hipEvent_t c0 = cleanup.e[0], c1 = cleanup.e[1], r1 = cleanup.e[2];
    hip_check(hipEventRecord(e0, st), "event");
    hip_check(hipStreamWaitEvent(sc, e0, 0), "stream wait");
    hip_check(hipEventRecord(c0, sc), "event");
    M.mem_col = std::make_unique<DevMem>(0);
    Error cerr{DH2_OK, ""};
    std::thread th([&] {
      try {
        hip_check(hipSetDevice(dev), "hipSetDevice");
        M.mem_col->begin_staging();
        sweep(M, 1, g, sc, ss_col, d_status + 4, *M.mem_col);
        expand_side(M, 1, sc, *M.mem_col);
        hip_check(hipEventRecord(c1, sc), "event");
        M.mem_col->end_staging(sc);
      } catch (const Error& e) {
        cerr = e;
      } catch (const std::bad_alloc&) {
        cerr = Error{DH2_ENOMEM, "host allocation failed"};
      } catch (const std::exception& e) {
        cerr = Error{DH2_EDEVICE, e.what()};
      }
    });
    try {
      sweep(M, 0, g, st, ss_row, d_status, mem);
    } catch (...) {
      th.join();
      throw;
    }
    th.join();
    if (cerr.code != DH2_OK) fail(cerr.code, cerr.msg);
    hip_check(hipEventRecord(r1, st), "event");
    hip_check(hipStreamWaitEvent(st, c1, 0), "stream wait");
    hip_check(hipEventRecord(e1, st), "event");
    // the projection's task lists are built on the host while the device
    // finishes the sweeps; its launches follow the sweeps on st
    project_all(M, st, mem, ss_row);
    hip_check(hipEventSynchronize(e1), "event");
    hip_check(hipEventElapsedTime(&ms_sweeps, e0, e1), "event");
    hip_check(hipEventElapsedTime(&ms_col, c0, c1), "event");
    hip_check(hipEventElapsedTime(&ms_row, e0, r1), "event");
  }
  // projection of every admissible block (needs both bases)
  if (!M.concurrent) project_all(M, st, mem, ss_row);
  ms_sweeps += (float)(ss_row.t_prj * 1e3);

  // near field done (it ran beside the sweeps)
  hip_check(hipStreamWaitEvent(st, nf.e[1], 0), "stream wait");
  hip_check(hipEventRecord(e1, st), "event");
  hip_check(hipEventSynchronize(e1), "event");
  float ms_near = 0, ms_span = 0;
  hip_check(hipEventElapsedTime(&ms_near, nf.e[0], nf.e[1]), "event");
  hip_check(hipEventElapsedTime(&ms_span, nf.e[2], e1), "event");
  for (int64_t* q : nf.d) mem.release(q);
  trc.mark("sweeps+near", -1, -1, -1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (trace_on()) {
    int32_t stat[8];
    copy_from(stat, d_status, 8, st);
    std::fprintf(stderr, "[dh2 trace] factorisations %d, mean Jacobi sweeps %.2f, %s sweeps\n",
                 stat[2] + stat[6],
                 stat[2] + stat[6] ? (double)(stat[1] + stat[5]) / (stat[2] + stat[6]) : 0.0,
                 M.concurrent ? "concurrent" : "sequential");
    std::fprintf(stderr,
                 "[dh2 trace] factor classes r<=32 %lld, <=48 %lld, <=64 %lld, <=128 %lld, "
                 "in memory %lld; factored again %lld, in memory %lld\n",
                 (long long)(ss_row.n_fac[0] + ss_col.n_fac[0]),
                 (long long)(ss_row.n_fac[1] + ss_col.n_fac[1]),
                 (long long)(ss_row.n_fac[2] + ss_col.n_fac[2]),
                 (long long)(ss_row.n_fac[3] + ss_col.n_fac[3]),
                 (long long)(ss_row.n_fac[4] + ss_col.n_fac[4]),
                 (long long)(ss_row.n_redo + ss_col.n_redo),
                 (long long)(ss_row.n_redo_mem + ss_col.n_redo_mem));
  }
  mem.release(d_status);
  // the dense matrix is borrowed only for this call
  M.omega.resize(nadm);
  copy_from(M.omega.data(), M.d_omega, nadm, st);

  // statistics
  dh2_stats& S = M.stats;
  S.n = n;
  S.nadm = nadm;
  S.nnear = nnear;
  S.items[0] = M.side[0].nitems;
  S.items[1] = M.side[1].nitems;
  int32_t kmax = 0;
  double words = 0;
  for (int s = 0; s < 2; ++s)
    for (const ItemDev& it : M.side[s].items) {
      kmax = std::max(kmax, it.k);
      words += (double)it.r * it.k;  // leaf Q or transfer [E1;E2]
    }
  const double bwords = words;
  for (int64_t b = 0; b < nadm; ++b) words += (double)M.S_rows[b] * M.S_cols[b];
  for (const NearDev& nd : M.nears) words += (double)nd.t_len * nd.s_len;
  S.repr_bytes = bwords * 16.0 + (words - bwords) * (M.s32 ? 8.0 : 16.0);
  S.k_max = kmax;
  S.mem_bytes = words * 16.0;
  S.mem_per_n_kib = S.mem_bytes / 1024.0 / (double)n;
  S.t_col = ms_col * 1e-3;
  S.t_prj = ss_row.t_prj;
  S.t_row = ms_row * 1e-3;
  S.t_near = ms_near * 1e-3;
  // the near field overlaps the sweeps: the total is the device span
  S.t_total = (ms_w + ms_span) * 1e-3;
  S.flops_row = ss_row.flops_gram + ss_row.flops_rprod;
  S.flops_col = ss_col.flops_gram + ss_col.flops_rprod;
  S.flops_prj = ss_row.flops_prj;
  S.flops_gram = ss_row.flops_gram + ss_col.flops_gram;
  S.flops_rprod = ss_row.flops_rprod + ss_col.flops_rprod;
  S.t_gram_kernel = ss_row.t_gram + ss_col.t_gram;
  S.groups = M.nbatch;
  S.precision = M.precision;
  S.flops_gram_leaf = ss_row.flops_gram_leaf + ss_col.flops_gram_leaf;
  S.t_gram_leaf = ss_row.t_gram_leaf + ss_col.t_gram_leaf;
  S.n_gram_leaf = ss_row.n_gram_leaf + ss_col.n_gram_leaf;
  S.flops_rprod_leaf = ss_row.flops_rprod_leaf + ss_col.flops_rprod_leaf;
  S.ops_gram_leaf_i8 = ss_row.ops_gram_leaf_i8 + ss_col.ops_gram_leaf_i8;
  mem.end_staging(st);
  trc.mark("finish", -1, -1, -1);
  return Mp;
}

// Independent Helmholtz instances: worker threads, each with its own stream
// (default priority), take instances in turn; concurrent kernels of several
// instances fill the device where one small instance would not.  All work
// is ordered after the caller's stream and complete on return.
// instances of a batch run their two sweeps one after the other: the
// instances on several streams already fill the device
constexpr bool kBatchConcurrent = false;

std::vector<std::unique_ptr<MatrixData>> compress_batch(
    const std::vector<std::shared_ptr<BlocksData>>& blks, const std::vector<const double*>& w,
    double eps, const dh2_opts& o, hipStream_t st, int nstreams) {
  const int n = (int)blks.size();
  std::vector<std::unique_ptr<MatrixData>> out(n);
  if (n == 0) return out;
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  hipEvent_t ready;
  hip_check(hipEventCreateWithFlags(&ready, hipEventDisableTiming), "event");
  hip_check(hipEventRecord(ready, st), "event record");
  // the largest instances first (their work grows with n^2), so that the
  // last instances to start are small and the streams finish together
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return blks[a]->tree->tr.n > blks[b]->tree->tr.n;
  });
  std::atomic<int> next{0};
  std::atomic<bool> failed{false};
  std::mutex emu;
  Error first{DH2_OK, ""};
  auto record = [&](dh2_status c, const std::string& m) {
    std::lock_guard<std::mutex> lk(emu);
    if (!failed.exchange(true)) first = Error{c, m};
  };
  auto worker = [&]() {
    hipStream_t s = nullptr;
    try {
      hip_check(hipSetDevice(dev), "hipSetDevice");
      hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "stream create");
      hip_check(hipStreamWaitEvent(s, ready, 0), "stream wait");
      for (;;) {
        const int q = next.fetch_add(1);
        if (q >= n || failed.load()) break;
        const int i = order[q];
        out[i] = compress(blks[i], SRC_HELMHOLTZ, nullptr, 0, w[i], eps, o, s, nullptr,
                          kBatchConcurrent);
      }
    } catch (const Error& e) {
      record(e.code, e.msg);
    } catch (const std::bad_alloc&) {
      record(DH2_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
      record(DH2_EDEVICE, e.what());
    }
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  };
  int nt = std::max(1, std::min(nstreams, n));
  std::vector<std::thread> th;
  for (int q = 0; q < nt; ++q) th.emplace_back(worker);
  for (auto& t : th) t.join();
  (void)hipEventDestroy(ready);
  if (failed.load()) {
    out.clear();
    fail(first.code, first.msg);
  }
  return out;
}

// ---------------------------------------------------------------------------
// matrix-vector product
// ---------------------------------------------------------------------------
static void build_mv(MatrixData& M, hipStream_t st) {
  auto P = std::make_unique<MatvecPlan>();
  const BlocksData& B = *M.blk;
  const ClusterTree& tr = B.tree->tr;
  const Directions& dr = B.tree->dr;
  const BlockTree& bt = B.bt;
  DevMem& mem = *M.mem;
  int64_t nadm = (int64_t)bt.adm_t.size();
  int64_t maxh = 0;
  for (int s = 0; s < 2; ++s) {
    Side& S = M.side[s];
    SideMV& V = P->s[s];
    std::vector<int64_t> hoff(S.nitems + 1, 0);
    for (int32_t i = 0; i < S.nitems; ++i) hoff[i + 1] = hoff[i] + S.items[i].k;
    V.total = hoff[S.nitems];
    maxh = std::max(maxh, V.total);
    V.d_hoff = upload(mem, hoff, st);
    // coupling lists: this side receives; blocks whose cluster on this side is the item
    std::vector<std::vector<std::pair<int32_t, int32_t>>> lst(S.nitems);
    for (int64_t b = 0; b < nadm; ++b) {
      int32_t t = s == 0 ? bt.adm_t[b] : bt.adm_s[b];
      int32_t o = s == 0 ? bt.adm_s[b] : bt.adm_t[b];
      int32_t c = bt.adm_c[b];
      int32_t me = S.P->ext2int[B.cs[s].find(t, c)];
      int32_t pe = M.side[1 - s].P->ext2int[B.cs[1 - s].find(o, c)];
      lst[me].push_back({(int32_t)b, pe});
    }
    std::vector<int64_t> cb(S.nitems + 1, 0);
    std::vector<int32_t> cblk, cpar;
    for (int32_t i = 0; i < S.nitems; ++i) {
      for (auto& pr : lst[i]) {
        cblk.push_back(pr.first);
        cpar.push_back(pr.second);
      }
      cb[i + 1] = (int64_t)cblk.size();
    }
    V.d_cbegin = upload(mem, cb, st);
    V.d_cblock = upload(mem, cblk, st);
    V.d_cpartner = upload(mem, cpar, st);
    {
      // the items with the most coupling entries first: one wave per item,
      // and an item has up to several times the mean number of blocks
      std::vector<int64_t> work(S.nitems, 0);
      for (int32_t i = 0; i < S.nitems; ++i)
        for (int64_t c = cb[i]; c < cb[i + 1]; ++c)
          work[i] += (int64_t)M.S_rows[cblk[c]] * M.S_cols[cblk[c]];
      std::vector<int32_t> ord(S.nitems);
      for (int32_t i = 0; i < S.nitems; ++i) ord[i] = i;
      std::stable_sort(ord.begin(), ord.end(),
                       [&](int32_t a, int32_t b) { return work[a] > work[b]; });
      V.d_corder = upload(mem, ord, st);
      // items with more than four times the mean work get four waves
      int64_t tot = 0;
      for (int64_t x : work) tot += x;
      const double lim = 4.0 * (double)tot / std::max<int32_t>(1, S.nitems);
      V.nheavy = 0;
      while (V.nheavy < S.nitems && (double)work[ord[V.nheavy]] > lim) ++V.nheavy;
    }
    // forward lists
    std::vector<int32_t> leafs;
    std::vector<std::vector<int32_t>> byl(tr.depth + 1);
    for (int32_t i = 0; i < S.nitems; ++i) {
      if (S.items[i].leaf) leafs.push_back(i);
      else byl[S.items[i].level].push_back(i);
    }
    V.d_fwd_leaf = upload(mem, leafs, st);
    V.n_fwd_leaf = (int32_t)leafs.size();
    for (int32_t l = tr.depth; l >= 0; --l) {
      V.d_fwd_lvl.push_back(upload(mem, byl[l], st));
      V.fwd_count.push_back((int32_t)byl[l].size());
    }
    // backward lists: per level, items with father items
    for (int32_t l = 0; l <= tr.depth; ++l) {
      std::vector<int32_t> items, fitem, fson;
      std::vector<int64_t> fb{0};
      for (int32_t i = 0; i < S.nitems; ++i) {
        if (S.items[i].level != l) continue;
        int32_t t = S.P->t[i], c = S.P->c[i];
        int32_t fa = tr.father[t];
        std::vector<std::pair<int32_t, int32_t>> fl;
        if (fa >= 0) {
          const auto& sdl = dr.sd[tr.level[fa]];
          const ColumnSets& cs = B.cs[s];
          for (int32_t e = cs.first[fa]; e < cs.first[fa] + cs.count[fa]; ++e)
            if (sdl[cs.item_c[e]] == c) fl.push_back({S.P->ext2int[e], tr.son1[fa] == t ? 0 : 1});
        }
        if (fl.empty()) continue;
        items.push_back(i);
        for (auto& pr : fl) {
          fitem.push_back(pr.first);
          fson.push_back(pr.second);
        }
        fb.push_back((int64_t)fitem.size());
      }
      V.d_bl_items.push_back(upload(mem, items, st));
      V.bl_count.push_back((int32_t)items.size());
      V.d_bl_fbegin.push_back(upload(mem, fb, st));
      V.d_bl_fitem.push_back(upload(mem, fitem, st));
      V.d_bl_fson.push_back(upload(mem, fson, st));
    }
    // leaves with their items and near-field references
    std::vector<LeafDev> leaves;
    std::vector<NearRefDev> refs;
    std::vector<std::vector<std::pair<int64_t, int64_t>>> nl(tr.nc());
    for (int64_t b = 0; b < (int64_t)bt.near_t.size(); ++b) {
      int32_t t = s == 0 ? bt.near_t[b] : bt.near_s[b];
      // every leaf below t
      std::vector<int32_t> stk{t};
      while (!stk.empty()) {
        int32_t u = stk.back();
        stk.pop_back();
        if (tr.leaf(u)) nl[u].push_back({b, tr.off[u] - tr.off[t]});
        else {
          stk.push_back(tr.son1[u]);
          stk.push_back(tr.son2[u]);
        }
      }
    }
    // A leaf's near-field work (entries of its rows) varies by more than an
    // order of magnitude: a leaf at a shallow level meets large clusters in
    // its inadmissible blocks.  Leaves with more than twice the mean work
    // are split into tasks of about that size that write partial sums, added
    // per leaf in task order afterwards (deterministic); tasks run heaviest
    // first.
    int64_t task_entries = 0;
    {
      int64_t tot = 0, nlf = 0;
      for (int32_t t = 0; t < tr.nc(); ++t) {
        if (!tr.leaf(t)) continue;
        ++nlf;
        for (auto& pr : nl[t])
          tot += tr.size[t] * (s == 0 ? tr.size[bt.near_s[pr.first]] : tr.size[bt.near_t[pr.first]]);
      }
      task_entries = std::max<int64_t>(2048, 2 * tot / std::max<int64_t>(1, nlf));
    }
    std::vector<std::pair<int64_t, LeafDev>> tasks;
    std::vector<LeafDev> split, basis;
    int32_t slots = 0;
    for (int32_t t = 0; t < tr.nc(); ++t) {
      if (!tr.leaf(t)) continue;
      if (tr.size[t] > 64) fail(DH2_EUNSUPPORTED, "leaf clusters with more than 64 points");
      LeafDev L{};
      L.row_off = tr.off[t];
      L.len = (int32_t)tr.size[t];
      // items of t are contiguous in internal order
      int32_t cnt = B.cs[s].count[t];
      L.item_first = cnt ? S.P->ext2int[B.cs[s].first[t]] : 0;
      L.item_count = cnt;
      for (int32_t q = 1; q < cnt; ++q)
        if (S.P->ext2int[B.cs[s].first[t] + q] != L.item_first + q) fail(DH2_EDEVICE, "internal: leaf items not contiguous");
      L.slot = -1;
      // the basis terms go into a task list of their own; the near-field
      // tasks carry none
      {
        LeafDev Bt = L;
        Bt.near_begin = Bt.near_end = 0;
        basis.push_back(Bt);
      }
      L.item_count = 0;
      const int64_t r0 = (int64_t)refs.size();
      int64_t total = 0;
      std::vector<int64_t> wref;
      for (auto& pr : nl[t]) {
        refs.push_back(NearRefDev{pr.first, pr.second});
        const int64_t b = pr.first;
        wref.push_back((int64_t)L.len * (s == 0 ? tr.size[bt.near_s[b]] : tr.size[bt.near_t[b]]));
        total += wref.back();
      }
      const int64_t r1 = (int64_t)refs.size();
      if (total <= task_entries) {
        L.near_begin = r0;
        L.near_end = r1;
        tasks.push_back({total, L});
        continue;
      }
      const int64_t nt = (total + task_entries - 1) / task_entries;
      const int64_t per = (total + nt - 1) / nt;
      LeafDev R = L;
      R.item_first = slots;
      R.item_count = 0;
      int64_t q = r0;
      while (q < r1) {
        LeafDev T = L;
        T.slot = slots++;
        T.near_begin = q;
        int64_t wsum = 0;
        while (q < r1 && (wsum == 0 || wsum + wref[q - r0] <= per)) wsum += wref[q++ - r0];
        T.near_end = q;
        tasks.push_back({wsum, T});
        ++R.item_count;
      }
      split.push_back(R);
    }
    std::stable_sort(tasks.begin(), tasks.end(),
                     [](const auto& a, const auto& b) { return a.first > b.first; });
    for (const auto& tk : tasks) leaves.push_back(tk.second);
    V.d_leaves = upload(mem, leaves, st);
    V.d_nref = upload(mem, refs, st);
    V.nleaves = (int32_t)leaves.size();
    V.d_split = split.empty() ? nullptr : upload(mem, split, st);
    V.nsplit = (int32_t)split.size();
    V.d_basis = upload(mem, basis, st);
    V.nbasis = (int32_t)basis.size();
    V.nslots = slots;
    P->maxslots = std::max(P->maxslots, slots);
  }
  // the adjoint reads the near field through a transposed copy
  {
    int64_t tot = 0;
    for (const NearDev& nb : M.nears) tot = std::max(tot, nb.off + nb.t_len * nb.s_len);
    P->d_nearT = mem.alloc(std::max<int64_t>(1, tot) * (M.s32 ? sizeof(float2) : sizeof(double2)));
  }
  P->d_nears = upload(mem, M.nears, st);
  hip_check(hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking), "stream create");
  hip_check(hipEventCreateWithFlags(&P->ev_x, hipEventDisableTiming), "event");
  hip_check(hipEventCreateWithFlags(&P->ev_near, hipEventDisableTiming), "event");
  launch_near_transpose(P->d_nears, (int64_t)M.nears.size(), M.d_near, P->d_nearT, M.s32, st);
  launch_check("near-field transpose");
  P->d_Sptr = upload(mem, M.S_ptr, st);
  P->d_Srows = upload(mem, M.S_rows, st);
  P->d_Scols = upload(mem, M.S_cols, st);
  {
    // the adjoint's coupling reads S_b^T (kc x kr), a copy made here
    int64_t tot = 0;
    for (int64_t b = 0; b < nadm; ++b) tot += (int64_t)M.S_rows[b] * M.S_cols[b];
    const size_t sesz = M.s32 ? sizeof(float2) : sizeof(double2);
    char* arena = (char*)mem.alloc(std::max<int64_t>(1, tot) * sesz);
    std::vector<void*> tp(nadm);
    int64_t o = 0;
    for (int64_t b = 0; b < nadm; ++b) {
      tp[b] = arena + o * sesz;
      o += (int64_t)M.S_rows[b] * M.S_cols[b];
    }
    P->d_STptr = upload(mem, tp, st);
    launch_coupling_transpose(P->d_Sptr, P->d_STptr, P->d_Srows, P->d_Scols, nadm, M.s32, st);
    launch_check("coupling transpose");
  }
  int64_t n = tr.n;
  P->xp = (double2*)mem.alloc(n * kMvRhs * sizeof(double2));
  P->yp = (double2*)mem.alloc(n * kMvRhs * sizeof(double2));
  P->xh = (double2*)mem.alloc(std::max<int64_t>(1, maxh) * kMvRhs * sizeof(double2));
  P->yh = (double2*)mem.alloc(std::max<int64_t>(1, maxh) * kMvRhs * sizeof(double2));
  P->part = (double2*)mem.alloc(std::max<int64_t>(1, (int64_t)P->maxslots * 64) * kMvRhs *
                                sizeof(double2));
  P->maxh = maxh;
  M.mv = std::move(P);
}

// nr <= kMvRhs products (x, y column-major n x nr) in one pass of the
// kernels, into the given work vectors (no allocation, no wait): each
// element of the representation is read once for all nr right-hand sides
static void matvec_core(MatrixData& M, char op, int nr, const double2* x, double2* y,
                        const MatvecBufs& w, hipStream_t st) {
  MatvecPlan& P = *M.mv;
  const ClusterTree& tr = M.blk->tree->tr;
  int64_t n = tr.n;
  int adj = (op == 'C' || op == 'c') ? 1 : 0;
  int src_side = adj ? 0 : 1, dst_side = adj ? 1 : 0;
  Side& A = M.side[src_side];
  Side& Bs = M.side[dst_side];
  SideMV& VA = P.s[src_side];
  SideMV& VB = P.s[dst_side];
  launch_gather_perm(x, M.d_perm, n, w.xp, st, nr);
  // the near-field rows (about half of the representation's bytes) on the
  // second stream, beside the chain of small basis kernels
  hip_check(hipEventRecord(P.ev_x, st), "event record");
  hip_check(hipStreamWaitEvent(P.side, P.ev_x, 0), "stream wait");
  launch_bwd_leaf(Bs.d_items, VB.d_leaves, VB.nleaves, VB.d_nref, P.d_nears, M.d_near,
                  P.d_nearT, VB.d_hoff, w.yh, w.xp, w.yp, w.part, adj, nr, 1, 0, M.s32, P.side);
  launch_leaf_sum(VB.d_split, VB.nsplit, w.part, w.yp, nr, P.side);
  hip_check(hipEventRecord(P.ev_near, P.side), "event record");
  launch_fwd_leaf(A.d_items, VA.d_fwd_leaf, VA.n_fwd_leaf, VA.d_hoff, w.xp, w.xh, nr, st);
  for (size_t q = 0; q < VA.d_fwd_lvl.size(); ++q)
    launch_fwd_inner(A.d_items, VA.d_fwd_lvl[q], VA.fwd_count[q], VA.d_hoff, w.xh, nr, st);
  // op N: S_b (kt x ks); adjoint: S_b^T (ks x kt)
  launch_coupling(Bs.d_items, Bs.nitems, VB.nheavy, VB.d_corder, VB.d_cbegin, VB.d_cblock,
                  VB.d_cpartner,
                  adj ? P.d_STptr : P.d_Sptr, adj ? P.d_Scols : P.d_Srows,
                  adj ? P.d_Srows : P.d_Scols, VA.d_hoff, w.xh, VB.d_hoff, w.yh, adj, nr, M.s32,
                  st);
  for (size_t l = 0; l < VB.d_bl_items.size(); ++l)
    launch_bwd_inner(Bs.d_items, VB.d_bl_items[l], VB.bl_count[l], VB.d_bl_fbegin[l],
                     VB.d_bl_fitem[l], VB.d_bl_fson[l], VB.d_hoff, w.yh, nr, st);
  // basis terms added to the near-field rows
  hip_check(hipStreamWaitEvent(st, P.ev_near, 0), "stream wait");
  launch_bwd_leaf(Bs.d_items, VB.d_basis, VB.nbasis, VB.d_nref, P.d_nears, M.d_near, P.d_nearT,
                  VB.d_hoff, w.yh, w.xp, w.yp, w.part, adj, nr, 0, 1, M.s32, st);
  launch_scatter_perm(w.yp, M.d_perm, n, y, st, nr);
  launch_check("matvec");
}

void matvec(MatrixData& M, char op, int64_t nrhs, const double2* x, double2* y, hipStream_t st) {
  if (!M.mv) build_mv(M, st);
  MatvecPlan& P = *M.mv;
  const int64_t n = M.blk->tree->tr.n;
  for (int64_t q = 0; q < nrhs; q += kMvRhs) {
    const int nr = (int)std::min<int64_t>(kMvRhs, nrhs - q);
    matvec_core(M, op, nr, x + q * n, y + q * n, MatvecBufs{P.xp, P.yp, P.xh, P.yh, P.part},
                st);
  }
}

// The same product with its work vectors in the library's static scratch
// array: no device allocation and no wait.  The plan of the product (its
// index lists) must exist already; the first dh2_matvec on the matrix builds
// it.  Calls that overlap on one device share the array and race.
void matvec_noalloc(MatrixData& M, char op, int64_t nrhs, const double2* x, double2* y,
                    hipStream_t st) {
  if (!M.mv)
    fail(DH2_EINVAL, "the matrix has no matvec plan yet: call dh2_matvec on it once first");
  const int64_t n = M.blk->tree->tr.n;
  const int64_t maxh = std::max<int64_t>(1, M.mv->maxh);
  const int64_t maxp = std::max<int64_t>(1, (int64_t)M.mv->maxslots * 64);
  // 256-byte aligned parts: xp, yp (n each), xh, yh (maxh each), partial
  // sums of split leaves (64 per slot), per right-hand side of a pass; as
  // many right-hand sides per pass as fit
  auto part = [](int64_t cnt) { return ((size_t)cnt * sizeof(double2) + 255) / 256 * 256; };
  auto total = [&](int r) { return 2 * part(n * r) + 2 * part(maxh * r) + part(maxp * r); };
  int nr = kMvRhs;
  while (nr > 1 && total(nr) > noalloc_scratch_bytes()) --nr;
  const size_t need = total(nr);
  if (need > noalloc_scratch_bytes())
    fail(DH2_EUNSUPPORTED, "the allocation-free product needs " + std::to_string(need) +
                               " bytes of scratch, more than the library's " +
                               std::to_string(noalloc_scratch_bytes()));
  void* base = nullptr;
  hip_check(noalloc_scratch(&base), "scratch address");
  char* p = static_cast<char*>(base);
  MatvecBufs w;
  w.xp = (double2*)p;
  w.yp = (double2*)(p + part(n * nr));
  w.xh = (double2*)(p + 2 * part(n * nr));
  w.yh = (double2*)(p + 2 * part(n * nr) + part(maxh * nr));
  w.part = (double2*)(p + 2 * part(n * nr) + 2 * part(maxh * nr));
  for (int64_t q = 0; q < nrhs; q += nr) {
    const int m = (int)std::min<int64_t>(nr, nrhs - q);
    matvec_core(M, op, m, x + q * n, y + q * n, w, st);
  }
}

// ---------------------------------------------------------------------------
// error measures
// ---------------------------------------------------------------------------
static GeomDev geom(MatrixData& M, const void* G, int64_t ld) {
  GeomDev g{};
  g.pts = M.d_pts;
  g.cbox = M.d_cbox;
  g.nrm = M.d_nrm;
  g.G = (const double*)G;
  g.perm = M.d_perm;
  g.ldg = ld;
  g.n = M.blk->tree->tr.n;
  g.kappa = M.blk->tree->kappa;
  return g;
}

// y = G x or G^* x, all vectors in original order on the device
static void direct_apply(MatrixData& M, int src, const GeomDev& g, const double2* x, double2* y,
                         int adj, double2* tmp_p, double2* tmp_o, hipStream_t st) {
  int64_t n = g.n;
  launch_gather_perm(x, M.d_perm, n, tmp_p, st);
  launch_direct(src, g, nullptr, n, tmp_p, adj, tmp_o, st);
  launch_scatter_perm(tmp_o, M.d_perm, n, y, st);
  launch_check("direct product");
}

double error_estimate(MatrixData& M, const void* G, int64_t ld, int iters, uint64_t seed,
                      hipStream_t st) {
  int64_t n = M.blk->tree->tr.n;
  int src = G ? SRC_DENSE : (M.src == SRC_DLP ? SRC_DLP : SRC_HELMHOLTZ);
  if (src == SRC_HELMHOLTZ && M.src == SRC_DENSE)
    fail(DH2_EINVAL, "the matrix was compressed from a dense input: pass G");
  GeomDev g = geom(M, G, ld);
  DevMem& mem = *M.mem;
  double2* bufs = (double2*)mem.alloc(6 * n * sizeof(double2));
  double2 *x = bufs, *y1 = bufs + n, *y2 = bufs + 2 * n, *z = bufs + 3 * n, *tp = bufs + 4 * n,
          *to = bufs + 5 * n;
  std::vector<double2> hx(n), hy(n), hz(n);
  auto run = [&](bool diff) {
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd;
    double nrm = 0;
    for (int64_t i = 0; i < n; ++i) {
      hx[i] = make_double2(nd(rng), nd(rng));
      nrm += hx[i].x * hx[i].x + hx[i].y * hx[i].y;
    }
    nrm = std::sqrt(nrm);
    for (auto& v : hx) v = make_double2(v.x / nrm, v.y / nrm);
    double lam = 0, lam_old = 0;
    for (int it = 0; it < iters; ++it) {
      copy_to(mem, x, hx.data(), n, st);
      direct_apply(M, src, g, x, y1, 0, tp, to, st);
      if (diff) {
        matvec(M, 'N', 1, x, y2, st);
        copy_from(hy.data(), y1, n, st);
        copy_from(hz.data(), y2, n, st);
        for (int64_t i = 0; i < n; ++i) hy[i] = make_double2(hy[i].x - hz[i].x, hy[i].y - hz[i].y);
        copy_to(mem, y1, hy.data(), n, st);
      }
      direct_apply(M, src, g, y1, z, 1, tp, to, st);
      if (diff) {
        matvec(M, 'C', 1, y1, y2, st);
        copy_from(hz.data(), z, n, st);
        copy_from(hy.data(), y2, n, st);
        for (int64_t i = 0; i < n; ++i) hz[i] = make_double2(hz[i].x - hy[i].x, hz[i].y - hy[i].y);
      } else {
        copy_from(hz.data(), z, n, st);
      }
      double re = 0, zn = 0;
      for (int64_t i = 0; i < n; ++i) {
        re += hx[i].x * hz[i].x + hx[i].y * hz[i].y;
        zn += hz[i].x * hz[i].x + hz[i].y * hz[i].y;
      }
      lam = re;
      zn = std::sqrt(zn);
      if (zn == 0) return 0.0;
      for (int64_t i = 0; i < n; ++i) hx[i] = make_double2(hz[i].x / zn, hz[i].y / zn);
      if (lam_old > 0 && std::fabs(lam - lam_old) <= 1e-4 * lam) break;
      lam_old = lam;
    }
    return std::sqrt(std::max(lam, 0.0));
  };
  double num = run(true);
  double den = run(false);
  mem.release(bufs);
  return den > 0 ? num / den : 0.0;
}

void rows_check(MatrixData& M, const int64_t* rows, int32_t nrows, const double2* x,
                double* direct, double* approx, double* max_rel, hipStream_t st) {
  const ClusterTree& tr = M.blk->tree->tr;
  int64_t n = tr.n;
  if (M.src == SRC_DENSE) fail(DH2_EINVAL, "rows_check needs a matrix generated from points");
  std::vector<int64_t> inv(n);
  for (int64_t p = 0; p < n; ++p) inv[tr.perm[p]] = p;
  std::vector<int64_t> pos(nrows);
  for (int32_t q = 0; q < nrows; ++q) {
    if (rows[q] < 0 || rows[q] >= n) fail(DH2_EINVAL, "row index out of range");
    pos[q] = inv[rows[q]];
  }
  DevMem& mem = *M.mem;
  GeomDev g = geom(M, nullptr, 0);
  int64_t* d_pos = upload(mem, pos, st);
  double2* bufs = (double2*)mem.alloc((2 * n + nrows) * sizeof(double2));
  double2 *xp = bufs, *y = bufs + n, *out = bufs + 2 * n;
  launch_gather_perm(x, M.d_perm, n, xp, st);
  launch_direct(M.src, g, d_pos, nrows, xp, 0, out, st);
  launch_check("rows direct");
  matvec(M, 'N', 1, x, y, st);
  std::vector<double2> hd(nrows), hy(n);
  copy_from(hd.data(), out, nrows, st);
  copy_from(hy.data(), y, n, st);
  double num = 0, den = 0;
  for (int32_t q = 0; q < nrows; ++q) {
    double2 a = hy[rows[q]];
    if (direct) {
      direct[2 * q] = hd[q].x;
      direct[2 * q + 1] = hd[q].y;
    }
    if (approx) {
      approx[2 * q] = a.x;
      approx[2 * q + 1] = a.y;
    }
    num = std::max(num, std::hypot(a.x - hd[q].x, a.y - hd[q].y));
    den = std::max(den, std::hypot(hd[q].x, hd[q].y));
  }
  if (max_rel) *max_rel = den > 0 ? num / den : 0.0;
  mem.release(bufs);
  mem.release(d_pos);
}

}  // namespace dh2
