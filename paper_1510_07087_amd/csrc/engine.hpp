// Host engine: plan handles, device memory, the compression sweep, the DH2
// matrix-vector product and the error measures.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dh2.h"
#include "common.hpp"
#include "plan.hpp"

namespace dh2 {

struct Error {
  dh2_status code;
  std::string msg;
};

[[noreturn]] void fail(dh2_status code, const std::string& msg);
void hip_check(hipError_t e, const char* what);
// Return the cached (freed but kept) device blocks to the driver.
void release_cached_memory();

// Device allocations with an optional cap (max_device_bytes), owned by one
// host thread that queues its work on one stream at a time.
class DevMem {
 public:
  explicit DevMem(int64_t cap = 0) : cap_(cap) {}
  ~DevMem();
  void* alloc(size_t bytes);
  // The block stops counting against the cap at once; it joins the
  // process-wide cache, where work on other streams may take it, only at the
  // next sync(), when no queued work of this owner can still use it.
  void release(void* p);
  // Wait for the stream, then hand the released blocks to the cache and
  // recycle the staging buffer.
  void sync(hipStream_t st, const char* what);
  // Host-to-device copy.  While staging is on, the bytes are copied into a
  // pinned buffer at once and the transfer is queued without waiting (the
  // host data may change on return); otherwise the call waits for the stream.
  void upload(void* d, const void* h, size_t bytes, hipStream_t st);
  // Staging on: a pinned buffer from a process-wide pool.  Off: sync(st),
  // buffer back to the pool.
  void begin_staging();
  void end_staging(hipStream_t st);
  int64_t used() const { return used_; }
  int64_t peak() const { return peak_; }

 private:
  void flush_released();
  int64_t cap_;
  int64_t used_ = 0;
  int64_t peak_ = 0;
  std::vector<std::pair<void*, size_t>> live_;
  std::vector<std::pair<void*, size_t>> released_;
  char* pin_ = nullptr;
  size_t pin_off_ = 0;
};

struct TreeData {
  ClusterTree tr;
  Directions dr;
  std::vector<double> pts;  // original order, n x 3
  double kappa = 0;
  dh2_opts opts;
};

struct PlanCache;

// Sizes that choose the batch count of a compression: the first level with
// admissible blocks, the subtree group of every cluster (subtrees rooted one
// level above it) and the column counts of the bases per level and group.
struct SweepSizes {
  int32_t lmin = 0;
  int32_t ngroups = 0;
  std::vector<int32_t> group;  // per cluster, -1 above the group level
  std::vector<double> lvlN;    // columns per level (mean of both bases)
  std::vector<double> grpN;    // columns per group (both bases)
};

struct BlocksData {
  std::shared_ptr<TreeData> tree;
  BlockTree bt;
  ColumnSets cs[2];
  dh2_opts opts;
  // plan data of the compression for the last batch count used
  mutable std::mutex cache_mu;
  mutable std::shared_ptr<PlanCache> cache;
  mutable std::shared_ptr<const SweepSizes> sizes;  // built by the first compression
};

// Plan-derived data of one basis for a given batch count (side 0: rows of G,
// side 1: rows of G^*), items in internal order: sorted by (batch, level
// descending, cluster, direction).  Built once per block tree and batch count.
struct SidePlan {
  int32_t nitems = 0;
  std::vector<ItemDev> items0;      // plan fields of every item
  std::vector<int32_t> ext2int;     // column-set order -> internal
  std::vector<int32_t> int2ext;
  std::vector<int32_t> t, c;        // per internal item
  std::vector<EntDev> ents;         // leaf column-set entries (scale filled per matrix)
  std::vector<int64_t> ent_col;     // per column-set entry: column start inside its item
  // per internal item: columns inherited from the father's sets (the first
  // ninh columns; the item's own blocks follow them)
  std::vector<int64_t> ninh;
  // (batch, level) ranges of internal items
  std::vector<std::vector<std::pair<int32_t, int32_t>>> range;  // [batch][level] -> [lo,hi)
};

// Projection task of the row sweep: admissible block b = (t, s) of row item
// `item` whose column basis is item `witem` of side 1; per (batch, level),
// sorted by witem (expanded bases shared in L2).
struct ProjPlan {
  int32_t item, witem, b, ns;
  int64_t col;  // first column of s inside the row item
};

struct PlanCache {
  int32_t nbatch = -1;
  std::shared_ptr<const SidePlan> side[2];
  std::vector<std::vector<ProjPlan>> proj;  // [batch * (depth + 1) + level]
  EntDev* d_ents[2] = {nullptr, nullptr};   // device copies of side[s]->ents
  int64_t* d_adm = nullptr;                 // admissible blocks: t_off, t_len, s_off, s_len
  ~PlanCache();
};

// One basis of a matrix under compression.
struct Side {
  std::shared_ptr<const SidePlan> P;
  int32_t nitems = 0;
  std::vector<ItemDev> items;       // host mirror of the device array
  ItemDev* d_items = nullptr;
  EntDev* d_ents = nullptr;
  std::vector<void*> keep;          // Q and sigma arenas
  // expanded basis (column side): per internal item pointer, rows x k row-major
  std::vector<double2*> wexp;
  std::vector<float2*> wexp32;      // mixed form: FP32 copies for the projection
  // row sweep: own-block columns of each item's R^T kept for the projection
  std::vector<void*> own;
  std::vector<void*> own_keep;      // their arenas, released after the projection
};

struct MatvecPlan;

struct MatrixData {
  std::shared_ptr<BlocksData> blk;
  std::shared_ptr<PlanCache> plan;
  std::unique_ptr<DevMem> mem;
  // device memory of the column sweep when it runs beside the row sweep (its
  // own owner, since it queues work on another stream)
  std::unique_ptr<DevMem> mem_col;
  bool concurrent = false;     // the two sweeps ran at the same time
  int src = SRC_HELMHOLTZ;
  int precision = DH2_FP64;
  double eps = 0, zeta = 0;
  int32_t nbatch = 1;
  int32_t lmin = 0;
  int32_t max_sweeps = 60;     // Jacobi sweep limit of the small SVDs
  // device geometry
  double* d_pts = nullptr;     // permuted n x 4
  double* d_cbox = nullptr;    // per cluster: box and largest weight
  int64_t* d_perm = nullptr;
  double* d_nrm = nullptr;     // double layer: permuted n x 4 normals
  std::vector<double> w;       // original-order weights
  Side side[2];
  double* d_omega = nullptr;
  std::vector<double> omega;
  // coupling matrices and near field: complex FP32 in the mixed form (s32),
  // complex FP64 otherwise
  bool s32 = false;
  std::vector<void*> S_ptr;    // per admissible block
  std::vector<int32_t> S_rows, S_cols;
  void* d_near = nullptr;
  std::vector<NearDev> nears;
  dh2_stats stats{};
  std::unique_ptr<MatvecPlan> mv;
  ~MatrixData();
};

std::shared_ptr<TreeData> make_tree(const double* pts, int64_t n, double kappa, const dh2_opts& o);
std::shared_ptr<BlocksData> make_blocks(std::shared_ptr<TreeData> t, const dh2_opts& o);
// nrm: host n x 3 unit normals in the original order (SRC_DLP only);
// concurrent: the two sweeps may run at once (without a memory cap)
std::unique_ptr<MatrixData> compress(std::shared_ptr<BlocksData> b, int src, const void* G,
                                     int64_t ld, const double* w, double eps, const dh2_opts& o,
                                     hipStream_t st, const double* nrm = nullptr,
                                     bool concurrent = true);
std::vector<std::unique_ptr<MatrixData>> compress_batch(
    const std::vector<std::shared_ptr<BlocksData>>& blks, const std::vector<const double*>& w,
    double eps, const dh2_opts& o, hipStream_t st, int nstreams);
// y = G~ x or G~^* x for nrhs right-hand sides (column-major, ld = n), in passes of up
// to eight right-hand sides that read the representation once each
void matvec(MatrixData& M, char op, int64_t nrhs, const double2* x, double2* y, hipStream_t st);
// nrhs products with the work vectors in the static scratch array (no
// allocation, no wait); needs the matvec plan built by an earlier matvec()
void matvec_noalloc(MatrixData& M, char op, int64_t nrhs, const double2* x, double2* y,
                    hipStream_t st);
double error_estimate(MatrixData& M, const void* G, int64_t ld, int iters, uint64_t seed,
                      hipStream_t st);
void rows_check(MatrixData& M, const int64_t* rows, int32_t nrows, const double2* x,
                double* direct, double* approx, double* max_rel, hipStream_t st);

}  // namespace dh2
